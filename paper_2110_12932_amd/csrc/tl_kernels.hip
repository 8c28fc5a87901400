// HIP kernels of the two-level thermal solver for gfx950 (MI355X).
//
// Every kernel works on structured Q1 grids in the padded layout described in
// tl_internal.h (one ghost layer, zero-filled), so the 27-point gathers of the
// matrix-free operator need no bounds checks: ghost elements carry zero
// conductivity and ghost nodes hold zeros.  Work is spread with grid-stride
// loops over the real nodes (workgroups of 256 = 4 wavefronts of 64).
// Reductions are deterministic: fixed per-thread order, a fixed-shape
// workgroup tree, then a sum of the per-workgroup partials in index order.
// That last sum is never done with grid-wide fences or atomics (a
// device-scope release on this multi-XCD part writes back the XCD's L2 and
// costs more than the kernel): either the next kernel of the CG iteration
// re-sums the partials in every workgroup (kernel boundaries make them
// visible), or a one-workgroup finalize kernel does it.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "tl_internal.h"

namespace tl {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
// Arrays reached through the item tables are plain pointers there, and
// loads through them would compile to flat instructions: a 64-bit address
// per lane, and every such load counted against the LDS counter as well,
// so that a wait for an LDS result also waits for the loads in flight.
// Taken as global-address-space pointers they compile to global loads and
// stores, which count against the vector-memory counter only, and uniform
// reads of an item's state to scalar loads.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> gmem(T* p) {
  return (gptr<T>)p;
}
// Element n (>= 0) of an array of a level or of its tables, addressed with
// a 32-bit byte offset: a level holds at most 2e8 padded nodes (1.6 GB in
// FP64), so the offset fits, and a load or store takes the array's scalar
// base plus one 32-bit offset per lane, which every array indexed with the
// same n shares.
template <class T>
__device__ __forceinline__ gptr<T> at(gptr<T> p, int n) {
  return (gptr<T>)((gptr<const char>)p + (unsigned)n * (unsigned)sizeof(T));
}
// Whole-struct copies from and to global memory, word by word (a struct's
// implicit copy works in the generic address space only).
template <class T>
__device__ __forceinline__ T gload(gptr<const T> p) {
  static_assert(sizeof(T) % 4 == 0, "word-sized struct");
  unsigned w[sizeof(T) / 4];
  const gptr<const unsigned> src = (gptr<const unsigned>)p;
#pragma unroll
  for (unsigned q = 0; q < sizeof(T) / 4; ++q) w[q] = src[q];
  T v;
  __builtin_memcpy(&v, w, sizeof(T));
  return v;
}
template <class T>
__device__ __forceinline__ void gstore(gptr<T> p, const T& v) {
  static_assert(sizeof(T) % 4 == 0, "word-sized struct");
  unsigned w[sizeof(T) / 4];
  __builtin_memcpy(w, &v, sizeof(T));
  const gptr<unsigned> dst = (gptr<unsigned>)p;
#pragma unroll
  for (unsigned q = 0; q < sizeof(T) / 4; ++q) dst[q] = w[q];
}

static inline int grid_for(long n) {
  long b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > kMaxBlocks) b = kMaxBlocks;
  return (int)b;
}

// Wave-wide reductions with DPP lane moves (no trip through the LDS
// crossbar): pairs within quads, then half rows and rows by mirroring,
// then rows 1 and 3 take the last lane of the row before them and rows 2
// and 3 that of row 1, so that lane 63 holds the result, which is then
// read by every lane (the rows a broadcast skips take a dummy zero, which
// never reaches lane 63).  A fixed pattern: the same order of operations
// on every call.  Every lane of the wave must be active.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_move(int v) {
  return __builtin_amdgcn_update_dpp(0, v, kCtrl, kRowMask, 0xf, false);
}
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_move<kCtrl, kRowMask>((int)b);
  const int hi = dpp_move<kCtrl, kRowMask>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
template <int kCtrl, int kRowMask = 0xf>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(
      float, dpp_move<kCtrl, kRowMask>(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double lane63(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float lane63(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
template <class T, class Op>
__device__ __forceinline__ T wave_reduce(T v, Op op) {
  v = op(v, dpp_move<0xb1>(v));        // quad_perm [1,0,3,2]
  v = op(v, dpp_move<0x4e>(v));        // quad_perm [2,3,0,1]
  v = op(v, dpp_move<0x141>(v));       // row_half_mirror
  v = op(v, dpp_move<0x140>(v));       // row_mirror
  v = op(v, dpp_move<0x142, 0xa>(v));  // row_bcast:15 into rows 1, 3
  v = op(v, dpp_move<0x143, 0xc>(v));  // row_bcast:31 into rows 2, 3
  return lane63(v);
}
template <class T>
__device__ inline T wave_sum(T v) {
  return wave_reduce(v, [](T a, T b) { return a + b; });
}
template <class T>
__device__ inline T wave_max(T v) {
  return wave_reduce(v, [](T a, T b) { return fmax(a, b); });
}

// Block-wide sum of NV values per thread; result valid in thread 0.
template <int NV, class T>
__device__ inline void block_sum(T (&v)[NV], T* lds) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int a = 0; a < NV; ++a) v[a] = wave_sum(v[a]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < NV; ++a) lds[wid * NV + a] = v[a];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int a = 0; a < NV; ++a) {
      T s = lds[a];
      for (int w = 1; w < kBlock / 64; ++w) s += lds[w * NV + a];
      v[a] = s;
    }
  }
}

// One-workgroup finalize of a generic sum: *slot = scale * sum (assign) or
// *slot += scale * sum.
__global__ void __launch_bounds__(kBlock)
finalize_sum_kernel(const double* __restrict__ part, int n, double scale,
                    double* slot, int assign) {
  __shared__ double lds[kBlock / 64];
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < n; b += kBlock) v[0] += part[b];
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) *slot = assign ? scale * v[0] : *slot + scale * v[0];
}

static void finalize_sum(Launch L, const double* part, int n, double scale,
                         double* slot, int assign) {
  hipLaunchKernelGGL(finalize_sum_kernel, dim3(1), dim3(kBlock), 0,
                     (hipStream_t)L.stream, part, n, scale, slot, assign);
}

__device__ inline void node_ijk(const Geo& g, int t, int& i, int& j, int& k) {
  i = t % g.nx;
  int r = t / g.nx;
  j = r % g.ny;
  k = r / g.ny;
}
__device__ inline int pidx(const Geo& g, int i, int j, int k) {
  return (k + 1) * g.pxy + (j + 1) * g.px + (i + 1);
}

// ---------------------------------------------------------------------------
// material law (paper Section 2)
// ---------------------------------------------------------------------------
__device__ inline double clampT(double T, const MatDev& m) {
  return fmin(fmax(T, m.T_lo), m.T_hi);
}
__device__ inline double kappa_of(double T, const MatDev& m) {
  return m.k_lo + m.kslope * (clampT(T, m) - m.T_lo);
}
__device__ inline double heatcap_of(double T, const MatDev& m) {
  return m.c_lo + m.cslope * (clampT(T, m) - m.T_lo);
}
// tanh for the phase-change sigmoid, from expm1: t = -em / (2 + em) with
// em = expm1(-2|x|), sign restored.  For |x| > 20, tanh(x) rounds to +-1 in
// double precision (1 - tanh(20) < 1e-17), so the exponential is skipped --
// the case of every node more than 20/S from the melting centre.
__device__ inline double sigmoid_tanh(double x) {
  const double ax = fabs(x);
  if (ax > 20.0) return copysign(1.0, x);
  const double em = expm1(-2.0 * ax);
  return copysign(-em / (2.0 + em), x);
}
// rho int_{T_lo}^T c (sensible part of the enthalpy)
__device__ inline double sensible(double T, const MatDev& m) {
  if (T < m.T_lo) return m.c_lo * (T - m.T_lo);
  if (T > m.T_hi) return m.sens_full + m.c_hi * (T - m.T_hi);
  const double u = T - m.T_lo;
  return m.c_lo * u + 0.5 * m.cslope * u * u;
}
// H(T) = rho int_{T_lo}^T c + rho chi f_pc(T), f_pc = (1 + tanh(S(T - Tm)))/2
__device__ inline double enthalpy(double T, const MatDev& m) {
  const double th = sigmoid_tanh(m.S * (T - m.Tm));
  return m.rho * (sensible(T, m) + m.latent * 0.5 * (1.0 + th));
}
// H(T) and H'(T) sharing one tanh
__device__ inline void enthalpy_and_slope(double T, const MatDev& m, double& H,
                                          double& dH) {
  const double th = sigmoid_tanh(m.S * (T - m.Tm));
  H = m.rho * (sensible(T, m) + m.latent * 0.5 * (1.0 + th));
  dH = m.rho * (heatcap_of(T, m) + m.latent * 0.5 * m.S * (1.0 - th * th));
}

// Trial temperature of one node for the Newton step `step` (= alpha dx):
// T - step, except that a step crossing the centre T_m of the melting
// sigmoid lands on T_m.  Plain Newton on the enthalpy form cycles across the
// sharp latent-heat peak of H' (the tangent on one side overshoots to the
// other); from T_m the next step no longer crosses.  The converged solution
// R(T) = 0 is unchanged.
__device__ inline double trial_T(double T, double step, const MatDev& m) {
  const double t1 = T - step;
  return ((T - m.Tm) * (t1 - m.Tm) < 0.0) ? m.Tm : t1;
}

// ---------------------------------------------------------------------------
// region rules (which elements are active, which nodes are Dirichlet)
// ---------------------------------------------------------------------------
__device__ inline bool in_window_box(const Region& rg, int ei, int ej, int ek) {
  return ei >= rg.I0 && ei < rg.I1 && ej >= rg.J0 && ej < rg.J1 && ek >= rg.K0;
}
__device__ inline bool elem_active(const Geo& g, const Region& rg, int ei,
                                   int ej, int ek) {
  if (ei < 0 || ej < 0 || ek < 0 || ei > g.nx - 2 || ej > g.ny - 2 ||
      ek > g.nz - 2)
    return false;
  if (rg.mode == kOutside) return !in_window_box(rg, ei, ej, ek);
  return true;
}
// An active element with the constant global coefficients of the consistent
// formulation (inside the window box of a kFictitious region).
__device__ inline bool elem_fictitious(const Region& rg, int ei, int ej, int ek) {
  return rg.mode == kFictitious && in_window_box(rg, ei, ej, ek);
}
__device__ inline bool on_immersed_face(const Region& rg, int i, int j, int k,
                                        int i0, int i1, int j0, int j1,
                                        int k0) {
  return ((rg.faces & kFx0) && i == i0) || ((rg.faces & kFx1) && i == i1) ||
         ((rg.faces & kFy0) && j == j0) || ((rg.faces & kFy1) && j == j1) ||
         ((rg.faces & kFz0) && k == k0);
}
__device__ inline bool node_dirichlet(const Geo& g, const Region& rg, int i,
                                      int j, int k) {
  if (rg.mode == kAllBottom || rg.mode == kFictitious) return k == 0;
  if (rg.mode == kOutside) {
    if (k == 0) return true;
    bool inwin = i >= rg.I0 && i <= rg.I1 && j >= rg.J0 && j <= rg.J1 &&
                 k >= rg.K0;
    return inwin && !on_immersed_face(rg, i, j, k, rg.I0, rg.I1, rg.J0,
                                      rg.J1, rg.K0);
  }
  // kWindow
  if (rg.bottom && k == 0) return true;
  return on_immersed_face(rg, i, j, k, 0, g.nx - 1, 0, g.ny - 1, 0);
}

// Top-surface loss (paper Section 2): lumped area of the top faces around
// top node (i, j) -- a quarter of each face -- counting only faces the
// region keeps (the coarse outside solve drops the window's faces).
__device__ inline double top_area(const Geo& g, const Region& rg, int i, int j) {
  int n = 0;
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int fi = i - a, fj = j - b;
      bool keep = fi >= 0 && fj >= 0 && fi <= g.nx - 2 && fj <= g.ny - 2;
      if (keep && (rg.mode == kOutside || rg.mode == kFictitious))
        keep = !(fi >= rg.I0 && fi < rg.I1 && fj >= rg.J0 && fj < rg.J1);
      n += keep ? 1 : 0;
    }
  return 0.25 * g.hx * g.hy * n;
}
__device__ inline double surface_flux(double T, const SurfDev& sf) {
  const double T2 = T * T, a2 = sf.T_amb * sf.T_amb;
  return sf.h * (T - sf.T_amb) + sf.es * (T2 * T2 - a2 * a2);
}
__device__ inline double surface_slope(double T, const SurfDev& sf) {
  return sf.h + 4.0 * sf.es * T * T * T;
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------
__global__ void fill_kernel(double* a, double v, long n) {
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x)
    a[t] = v;
}
__global__ void zero_kernel(uint32_t* a, long n) {
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x)
    a[t] = 0u;
}
__global__ void copy_kernel(double* dst, const double* src, long n) {
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x)
    dst[t] = src[t];
}

__global__ void extrapolate_kernel(double* dst, const double* a,
                                   const double* b, long n) {
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x)
    dst[t] = 2.0 * a[t] - b[t];
}
void k_extrapolate(Launch L, double* dst, const double* a, const double* b,
                   long n) {
  hipLaunchKernelGGL(extrapolate_kernel, dim3(grid_for(n)), dim3(kBlock), 0,
                     (hipStream_t)L.stream, dst, a, b, n);
}

void k_fill(Launch L, double* a, double v, long n) {
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(kBlock), 0,
                     (hipStream_t)L.stream, a, v, n);
}
void k_zero_bytes(Launch L, void* a, size_t bytes) {
  long n = (long)(bytes / 4);
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n)), dim3(kBlock), 0,
                     (hipStream_t)L.stream, (uint32_t*)a, n);
}
void k_copy(Launch L, double* dst, const double* src, long n) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n)), dim3(kBlock), 0,
                     (hipStream_t)L.stream, dst, src, n);
}

// ---------------------------------------------------------------------------
// the matrix-free Q1 heat operator
// ---------------------------------------------------------------------------
// Neighbour offset table: n27(dx,dy,dz) = (dx+1) + 3(dy+1) + 9(dz+1).
#define N27(dx, dy, dz) (((dx) + 1) + 3 * ((dy) + 1) + 9 * ((dz) + 1))

// K v at a node, with v27 the 27 values around the node and k8[e] the
// conductivity of element e = ex + 2 ey + 4 ez (the element at offset
// (-ex, -ey, -ez), of which the node is corner e).  The element sums
// sum_e k8[e] sum_c W[e ^ c] v_c are regrouped by neighbour: the elements
// holding both the node and its neighbour at offset d are those with
// e_a = (d_a < 0) on every axis where d_a != 0 (either value where d_a = 0),
// and for all of them the pattern e ^ c is (|dx|, |dy|, |dz|).  So
//   K v = sum_d W[|dx| + 2|dy| + 4|dz|] Ksum(d) v_d,
// with Ksum(d) the sum of those elements' conductivities: partial sums of
// k8 along one axis (edges), two axes (faces) and all three (centre).  This
// takes 19 additions and 35 multiply-adds per node instead of 72, and uses
// each neighbour value once.
// V(dx, dy, dz) supplies the neighbour values.
template <class R, class VF>
__device__ inline R stencil_grouped(VF V, const R (&k8)[8], const R (&w)[8]) {
  auto I = [](int dd) { return dd < 0 ? 1 : 0; };
  R kz[2][2], ky[2][2], kx[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      kz[a][b] = k8[a + 2 * b] + k8[a + 2 * b + 4];   // (ex, ey), both ez
      ky[a][b] = k8[a + 4 * b] + k8[a + 2 + 4 * b];   // (ex, ez), both ey
      kx[a][b] = k8[2 * a + 4 * b] + k8[1 + 2 * a + 4 * b];  // (ey, ez)
    }
  const R fx0 = kz[0][0] + kz[0][1], fx1 = kz[1][0] + kz[1][1];
  const R fy0 = kz[0][0] + kz[1][0], fy1 = kz[0][1] + kz[1][1];
  const R fz0 = ky[0][0] + ky[1][0], fz1 = ky[0][1] + ky[1][1];
  // every multiply-add is an explicit fma, so that no kernel's compiler
  // can fuse a sum of two products the other way round: the result is the
  // same bits in every kernel that calls this
  const R tot = fx0 + fx1;
  const R s1 = fma(fx1, V(-1, 0, 0), fx0 * V(1, 0, 0));
  const R s2 = fma(fy1, V(0, -1, 0), fy0 * V(0, 1, 0));
  const R s4 = fma(fz1, V(0, 0, -1), fz0 * V(0, 0, 1));
  R s3 = (R)0, s5 = (R)0, s6 = (R)0, s7 = (R)0;
#pragma unroll
  for (int a = -1; a <= 1; a += 2)
#pragma unroll
    for (int b = -1; b <= 1; b += 2) {
      s3 = fma(kz[I(a)][I(b)], V(a, b, 0), s3);
      s5 = fma(ky[I(a)][I(b)], V(a, 0, b), s5);
      s6 = fma(kx[I(a)][I(b)], V(0, a, b), s6);
#pragma unroll
      for (int c = -1; c <= 1; c += 2)
        s7 = fma(k8[I(a) + 2 * I(b) + 4 * I(c)], V(a, b, c), s7);
    }
  R acc = w[0] * (tot * V(0, 0, 0));
  acc = fma(w[1], s1, acc);
  acc = fma(w[2], s2, acc);
  acc = fma(w[3], s3, acc);
  acc = fma(w[4], s4, acc);
  acc = fma(w[5], s5, acc);
  acc = fma(w[6], s6, acc);
  acc = fma(w[7], s7, acc);
  return acc;
}
template <class R>
__device__ inline R stencil_apply(const R (&v27)[27], const R (&k8)[8],
                                  const R (&w)[8]) {
  return stencil_grouped(
      [&](int dx, int dy, int dz) { return v27[N27(dx, dy, dz)]; }, k8, w);
}

// The same K v summed element by element (8 x 8 multiply-adds): more
// arithmetic, but fewer values live at once, which keeps the FP64 z-march
// kernel at a higher occupancy.
template <class R, class VF>
__device__ inline R stencil_elementwise(VF V, const R (&k8)[8],
                                        const R (&w)[8]) {
  R acc = (R)0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
    R s = (R)0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
      s = fma(w[e ^ c], V(cx - ex, cy - ey, cz - ez), s);
    }
    acc = fma(k8[e], s, acc);
  }
  return acc;
}
template <class R>
__device__ inline R stencil_apply_elementwise(const R (&v27)[27],
                                              const R (&k8)[8],
                                              const R (&w)[8]) {
  return stencil_elementwise(
      [&](int dx, int dy, int dz) { return v27[N27(dx, dy, dz)]; }, k8, w);
}

template <class R>
__device__ inline void gather27(const Geo& g, const R* __restrict__ a, int n,
                                R (&v27)[27]) {
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx)
        v27[N27(dx, dy, dz)] = a[n + dx + dy * g.px + dz * g.pxy];
}

template <class R>
__device__ inline void gather8(const Geo& g, const R* __restrict__ kap, int n,
                               R (&k8)[8]) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
    k8[e] = kap[n - ex - ey * g.px - ez * g.pxy];
  }
}

// ---------------------------------------------------------------------------
// LDS-tiled CG kernels.  A workgroup owns a TX x TY x TZ tile of nodes (one
// node per thread).  The halo tile (TX+2)(TY+2)(TZ+2) of the operator input
// is formed once into LDS from coalesced global loads, together with the
// (TX+1)(TY+1)(TZ+1) element conductivities; the 27-point stencil then reads
// LDS only.  Halo loads are issued before the scalar reduction so that both
// latencies overlap.  Tiles past the grid's far edge are partially empty;
// their out-of-range halo entries are zero.
// ---------------------------------------------------------------------------
constexpr int TX = 16, TY = 4, TZ = 4;
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HN = HX * HY * HZ;
constexpr int EX = TX + 1, EY = TY + 1, EZ = TZ + 1, EN = EX * EY * EZ;
constexpr int HPT = (HN + kBlock - 1) / kBlock;
constexpr int EPT = (EN + kBlock - 1) / kBlock;
static_assert(TX * TY * TZ == kBlock, "one node per thread");

struct Tile {
  int ox, oy, oz;   // first node of the tile
  int tx, ty, tz;   // this thread's node inside the tile
};

// XCD-aware tile order.  Workgroups are dealt round-robin to the 8 XCDs
// (blockIdx.x % 8), each with its own L2.  The tiles (in the order of
// tile_at for the batched kernels, of tile_of for the bare operator) are
// cut into 8 contiguous chunks and chunk c is processed by the
// workgroups with blockIdx.x % 8 == c, so tiles that share halo entries sit
// on the same L2.  The workgroup count nb is a multiple of 8 and the first
// workgroup's index too; local workgroup b visits tiles first(b),
// first(b) + step, ... below last(b).
constexpr int kXcd = 8;
struct TileRange {
  int first, last, step;
};
__device__ inline TileRange tile_range(int b, int nb, int ntiles) {
  const int per = nb / kXcd;                       // workgroups per XCD
  const int chunk = (ntiles + kXcd - 1) / kXcd;    // tiles per XCD
  const int c = b % kXcd, slot = b / kXcd;
  TileRange r;
  r.first = c * chunk + slot;
  r.last = min((c + 1) * chunk, ntiles);
  r.step = per;
  return r;
}
static inline int tiled_grid(int ntiles) {
  const int per = (ntiles + kXcd - 1) / kXcd;
  return std::min(per * kXcd, kMaxBlocks);
}

__device__ inline Tile tile_of(int b, int ntx, int nty) {
  Tile t;
  t.ox = (b % ntx) * TX;
  t.oy = ((b / ntx) % nty) * TY;
  t.oz = (b / (ntx * nty)) * TZ;
  t.tx = threadIdx.x % TX;
  t.ty = (threadIdx.x / TX) % TY;
  t.tz = threadIdx.x / (TX * TY);
  return t;
}

// Tile b of a batched item, numbered x fastest, then z, then y: each XCD's
// contiguous chunk (tile_range) is a slab across y, whose halo faces are
// x-z planes -- smaller than the x-y planes of a chunk across z on the
// shallow grids of this method -- while tiles next to each other in x,
// which share 128-byte lines along their rows, still run side by side.
// On the raster build's window this cut the CG iteration's fetched bytes
// from 1.37 to 1.28 times the algorithmic reads.
__device__ inline Tile tile_at(const SolveItem& it, int b) {
  const int ntz = it.ntiles / (it.ntx * it.nty);
  Tile t;
  t.ox = (b % it.ntx) * TX;
  t.oz = ((b / it.ntx) % ntz) * TZ;
  t.oy = (b / (it.ntx * ntz)) * TY;
  t.tx = threadIdx.x % TX;
  t.ty = (threadIdx.x / TX) % TY;
  t.tz = threadIdx.x / (TX * TY);
  return t;
}
// padded index of halo entry h of the tile, or -1 when it lies past the
// ghost layer of the grid
__device__ inline int halo_index(const Geo& g, const Tile& t, int h) {
  const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
  const int i = t.ox + hx - 1, j = t.oy + hy - 1, k = t.oz + hz - 1;
  if (i > g.nx || j > g.ny || k > g.nz) return -1;
  return (k + 1) * g.pxy + (j + 1) * g.px + (i + 1);
}
// The same for the batched kernels, -1 also on the ghost layer itself:
// ghost nodes enter the stencil only through ghost elements, whose
// conductivity is zero, so the value taken for them does not change any
// sum as long as it is finite; zero is used and the ghost rows and planes
// are not fetched.
__device__ inline int halo_index_real(const Geo& g, const Tile& t, int h) {
  const int hx = h % HX, hy = (h / HX) % HY, hz = h / (HX * HY);
  const int i = t.ox + hx - 1, j = t.oy + hy - 1, k = t.oz + hz - 1;
  if (i < 0 || j < 0 || k < 0 || i >= g.nx || j >= g.ny || k >= g.nz)
    return -1;
  return (k + 1) * g.pxy + (j + 1) * g.px + (i + 1);
}
// padded index of element entry e (element with lowest corner at
// (ox-1+ex, ...)), or -1 past the ghost layer
__device__ inline int elem_index(const Geo& g, const Tile& t, int e) {
  const int ex = e % EX, ey = (e / EX) % EY, ez = e / (EX * EY);
  const int i = t.ox + ex - 1, j = t.oy + ey - 1, k = t.oz + ez - 1;
  if (i > g.nx || j > g.ny || k > g.nz) return -1;
  return (k + 1) * g.pxy + (j + 1) * g.px + (i + 1);
}
// The same, -1 for every element outside the grid (their stored
// conductivity is zero: never written on the ghost layer, written as zero
// by the residual kernel for the element past a grid's last node)
__device__ inline int elem_index_real(const Geo& g, const Tile& t, int e) {
  const int ex = e % EX, ey = (e / EX) % EY, ez = e / (EX * EY);
  const int i = t.ox + ex - 1, j = t.oy + ey - 1, k = t.oz + ez - 1;
  if (i < 0 || j < 0 || k < 0 || i >= g.nx - 1 || j >= g.ny - 1 ||
      k >= g.nz - 1)
    return -1;
  return (k + 1) * g.pxy + (j + 1) * g.px + (i + 1);
}

template <class R>
__device__ inline void load_kappa_tile(const Geo& g, const Tile& t,
                                       const R* __restrict__ kap, R* k_s) {
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = threadIdx.x + q * kBlock;
    if (e < EN) {
      const int n = elem_index(g, t, e);
      k_s[e] = n >= 0 ? kap[n] : (R)0;
    }
  }
}

// stencil of the node (tx,ty,tz) from the LDS tiles
template <class R>
__device__ inline R stencil_lds(const Tile& t, const R* u_s, const R* k_s,
                                const R (&w)[8]) {
  R u27[27], k8[8];
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx)
        u27[N27(dx, dy, dz)] =
            u_s[(t.tz + 1 + dz) * (HX * HY) + (t.ty + 1 + dy) * HX + (t.tx + 1 + dx)];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
    k8[e] = k_s[(t.tz + 1 - ez) * (EX * EY) + (t.ty + 1 - ey) * EX + (t.tx + 1 - ex)];
  }
  if constexpr (sizeof(R) == 8)
    return stencil_apply_elementwise(u27, k8, w);   // fewer live registers
  else
    return stencil_apply(u27, k8, w);
}

// Tiled matrix-free operator y = d v + K[kap] v (every node).
template <class R>
__global__ void __launch_bounds__(kBlock)
op_apply_tiled_kernel(Geo g, int ntx, int nty, int ntiles,
                      const R* __restrict__ d,
                      const R* __restrict__ kap, const R* __restrict__ v,
                      R* __restrict__ y) {
  __shared__ R u_s[HN];
  __shared__ R k_s[EN];
  R wts[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) wts[q] = (R)g.w[q];
  const TileRange tr = tile_range(blockIdx.x, gridDim.x, ntiles);
  for (int tile = tr.first; tile < tr.last; tile += tr.step) {
    const Tile t = tile_of(tile, ntx, nty);
#pragma unroll
    for (int q = 0; q < HPT; ++q) {
      const int h = threadIdx.x + q * kBlock;
      if (h < HN) {
        const int n = halo_index(g, t, h);
        u_s[h] = n >= 0 ? v[n] : (R)0;
      }
    }
    load_kappa_tile(g, t, kap, k_s);
    __syncthreads();
    const int i = t.ox + t.tx, j = t.oy + t.ty, k = t.oz + t.tz;
    if (i < g.nx && j < g.ny && k < g.nz) {
      const int n = pidx(g, i, j, k);
      const R vc = u_s[(t.tz + 1) * (HX * HY) + (t.ty + 1) * HX + (t.tx + 1)];
      y[n] = fma(d[n], vc, stencil_lds(t, u_s, k_s, wts));
    }
    __syncthreads();  // LDS is reused by the next tile
  }
}

// ---------------------------------------------------------------------------
// z-marching operator for grids too large for the caches.  A workgroup owns
// a ZX x ZY column of nodes (one wave per row of ZX = 64 nodes, so every row
// is one contiguous 512-byte (FP64) or 256-byte (FP32) segment) over a run
// of z planes and walks up the column.  Each thread keeps the 3 x 3 x 3
// values of v around its node and the 2 x 2 x 2 element conductivities in
// registers as a sliding window, so a step reads from LDS only the nine
// values of the next node plane and the four of the next element layer;
// LDS holds two node planes and two element layers (with x-y halo).  Global
// loads run three planes ahead of the stencil (two steps' loads in flight),
// so each input value is read from memory once (its x-y halo copies hit the
// L2 of neighbouring columns on the same XCD) and one barrier per plane
// suffices.
// ---------------------------------------------------------------------------
constexpr int ZX = 64, ZY = kBlock / ZX;
constexpr int ZHX = ZX + 2, ZHY = ZY + 2, ZHN = ZHX * ZHY;   // node plane
constexpr int ZEX = ZX + 1, ZEY = ZY + 1, ZEN = ZEX * ZEY;   // element layer
constexpr int ZHPT = (ZHN + kBlock - 1) / kBlock;
constexpr int ZEPT = (ZEN + kBlock - 1) / kBlock;

// Column tiles and z runs of the z-marching kernels.  Work units (x column
// fastest, then y column, then run) are cut into 8 contiguous chunks, one
// per XCD as in tile_range, so that columns sharing halo rows share an L2.
struct ZPlan {
  int ncx, ncy, nrun, run;   // columns per axis, runs per column, run length
};
template <class R>
static inline ZPlan zplan_of(const Geo& g) {
  ZPlan z;
  z.ncx = (g.nx + 1 + ZX - 1) / ZX;   // columns start at i = -1 (see below)
  z.ncy = (g.ny + ZY - 1) / ZY;
  const int cols = z.ncx * z.ncy;
  // Long runs: the two halo planes of a run are read twice.  Runs of at
  // least 64 planes in FP64 and whole columns in FP32 were the fastest on
  // a 640 x 640 x 160 grid (runs of 16 to 161 planes tried: 6 % and 5 %
  // faster than runs of 18); and no more runs than about 8 work units per
  // workgroup of a full grid (kMaxBlocks) need.  A grid with few columns
  // is still cut into at least 512 work units (two per compute unit), in
  // runs of at least 8 planes: on a 300 x 120 x 132 grid (155 columns)
  // that took 27 % (FP64) and 60 % (FP32) off the time of long runs, and
  // 1024 or 2048 units were no better
  const int min_run = sizeof(R) == 8 ? 64 : g.nz + 1;
  int nrun = std::max(1, std::min(8 * kMaxBlocks / cols, g.nz / min_run));
  nrun = std::max(nrun, std::min(g.nz / 8, (512 + cols - 1) / cols));
  z.run = (g.nz + nrun - 1) / nrun;
  z.nrun = (g.nz + z.run - 1) / z.run;
  return z;
}

template <class R>
__global__ void __launch_bounds__(kBlock)
op_apply_zmarch_kernel(Geo g, ZPlan zp, const R* __restrict__ d,
                       const R* __restrict__ kap, const R* __restrict__ v,
                       R* __restrict__ y) {
  // LDS planes padded to whole rounds of the workgroup, so that every
  // thread stores unconditionally
  __shared__ R v_s[2][ZHPT * kBlock];
  __shared__ R k_s[2][ZEPT * kBlock];
  const int nunits = zp.ncx * zp.ncy * zp.nrun;
  const TileRange tr = tile_range(blockIdx.x, gridDim.x, nunits);
  R wts[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) wts[q] = (R)g.w[q];
  const int tx = threadIdx.x % ZX, ty = threadIdx.x / ZX;
  for (int u = tr.first; u < tr.last; u += tr.step) {
    const int cx = u % zp.ncx, cy = (u / zp.ncx) % zp.ncy,
              run = u / (zp.ncx * zp.ncy);
    // column cx covers i = 64 cx - 1 ... 64 cx + 62: with the row pitch a
    // multiple of 32, its own row is then a whole number of 128-byte lines
    const int ox = cx * ZX - 1, oy = cy * ZY;
    const int k0 = run * zp.run, k1 = min(g.nz, k0 + zp.run);
    const int i = ox + tx, j = oy + ty;
    const bool col_active = i >= 0 && i < g.nx && j < g.ny;
    // padded offset within a plane of this thread's halo entries; entries
    // past the ghost layer (and the padding threads) read offset 0, the
    // plane's corner ghost, which is zero -- so every load is unconditional
    int voff[ZHPT], koff[ZEPT];
#pragma unroll
    for (int q = 0; q < ZHPT; ++q) {
      const int h = threadIdx.x + q * kBlock;
      const int ii = ox + h % ZHX - 1, jj = oy + h / ZHX - 1;
      voff[q] = (h >= ZHN || ii < -1 || ii > g.nx || jj > g.ny)
                    ? 0 : (jj + 1) * g.px + (ii + 1);
    }
#pragma unroll
    for (int q = 0; q < ZEPT; ++q) {
      const int e = threadIdx.x + q * kBlock;
      const int ii = ox + e % ZEX - 1, jj = oy + e / ZEX - 1;
      koff[q] = (e >= ZEN || ii < -1 || ii > g.nx || jj > g.ny)
                    ? 0 : (jj + 1) * g.px + (ii + 1);
    }
    const int doff = col_active ? (j + 1) * g.px + (i + 1) : 0;
    // node plane / element layer p (-1 <= p <= nz) at padded z offset
    // (p + 1) * pxy; planes past the grid are zero without a load
    auto load_plane = [&](int p, R (&rv)[ZHPT]) {
      if (p <= g.nz) {
        const R* __restrict__ pl = v + (long)(p + 1) * g.pxy;
#pragma unroll
        for (int q = 0; q < ZHPT; ++q) rv[q] = pl[voff[q]];
      } else {
#pragma unroll
        for (int q = 0; q < ZHPT; ++q) rv[q] = (R)0;
      }
    };
    auto load_layer = [&](int l, R (&rk)[ZEPT]) {
      if (l <= g.nz) {
        const R* __restrict__ la = kap + (long)(l + 1) * g.pxy;
#pragma unroll
        for (int q = 0; q < ZEPT; ++q) rk[q] = la[koff[q]];
      } else {
#pragma unroll
        for (int q = 0; q < ZEPT; ++q) rk[q] = (R)0;
      }
    };
    auto load_d = [&](int k) {
      // d and y are touched once per node: streamed past the caches
      // (nontemporal), which leaves them to the halo-shared v and kappa
      return k < k1 ? __builtin_nontemporal_load(&d[(long)(k + 1) * g.pxy + doff])
                    : (R)0;
    };
    auto put_plane = [&](int p, const R (&rv)[ZHPT]) {
#pragma unroll
      for (int q = 0; q < ZHPT; ++q) v_s[(p + 2) & 1][threadIdx.x + q * kBlock] = rv[q];
    };
    auto put_layer = [&](int l, const R (&rk)[ZEPT]) {
#pragma unroll
      for (int q = 0; q < ZEPT; ++q) k_s[(l + 2) & 1][threadIdx.x + q * kBlock] = rk[q];
    };
    // the 9 values of plane p around the node, the 4 conductivities of
    // layer l around it (element (ex, ey) at offset (-ex, -ey))
    auto get_plane = [&](int p, R (&w9)[9]) {
      const R* pl = v_s[(p + 2) & 1];
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx)
          w9[(dx + 1) + 3 * (dy + 1)] = pl[(ty + 1 + dy) * ZHX + (tx + 1 + dx)];
    };
    auto get_layer = [&](int l, R (&w4)[4]) {
      const R* la = k_s[(l + 2) & 1];
#pragma unroll
      for (int e = 0; e < 4; ++e)
        w4[e] = la[(ty + 1 - (e >> 1)) * ZEX + (tx + 1 - (e & 1))];
    };
    // Register window: planes k-1, k, k+1 (VM, V0, VP) and element layers
    // k-1, k (KM, K0).  Global loads run three planes ahead, so that two
    // steps' loads are in flight: queue slots QA (node plane k+2, element
    // layer k+1, loaded two steps earlier), QB (plane k+3, layer k+2, loaded
    // one step earlier) and QC (plane k+4, layer k+3, loaded now); the
    // node's own d at k, k+1, k+2.
    R V1[9], V2[9], V3[9], K1[4], K2[4];
    R Q1[ZHPT], Q1k[ZEPT], Q2[ZHPT], Q2k[ZEPT], Q3[ZHPT], Q3k[ZEPT];
    R dq0, dq1, dq2;
    {
      R a[ZHPT], b[ZHPT], c[ZHPT], ka[ZEPT], kb[ZEPT];
      load_plane(k0 - 1, a);
      load_plane(k0, b);
      load_layer(k0 - 1, ka);
      load_plane(k0 + 1, c);
      load_layer(k0, kb);
      dq0 = load_d(k0);
      dq1 = load_d(k0 + 1);
      dq2 = load_d(k0 + 2);
      load_plane(k0 + 2, Q1);
      load_layer(k0 + 1, Q1k);
      load_plane(k0 + 3, Q2);
      load_layer(k0 + 2, Q2k);
      put_plane(k0 - 1, a);
      put_plane(k0, b);
      put_layer(k0 - 1, ka);
      __syncthreads();
      get_plane(k0 - 1, V1);
      get_plane(k0, V2);
      get_layer(k0 - 1, K1);
      __syncthreads();
      put_plane(k0 + 1, c);
      put_layer(k0, kb);
      __syncthreads();
    }
    // One plane.  The register roles rotate between calls instead of being
    // copied: the window by three (VM, V0, VP -> V0, VP, VM), the element
    // layers by two and the load queue by three (QA, QB, QC -> QB, QC, QA).
    auto step = [&](int k, R (&VM)[9], R (&V0)[9], R (&VP)[9], R (&KM)[4],
                    R (&K0)[4], R (&QA)[ZHPT], R (&QAk)[ZEPT], R (&QC)[ZHPT],
                    R (&QCk)[ZEPT]) {
      // steps are not interleaved by the scheduler (that would only raise
      // the register count); nothing loaded here is waited for before the
      // step after next (memory counters complete in issue order)
      __builtin_amdgcn_sched_barrier(0);
      const R dn = load_d(k + 3);
      load_plane(k + 4, QC);
      load_layer(k + 3, QCk);
      get_plane(k + 1, VP);
      get_layer(k, K0);
      if (col_active) {
        R k8[8];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          k8[e] = K0[e];
          k8[4 + e] = KM[e];
        }
        auto V = [&](int dx, int dy, int dz) {
          const int q = (dx + 1) + 3 * (dy + 1);
          return dz < 0 ? VM[q] : (dz == 0 ? V0[q] : VP[q]);
        };
        R yn;
        if constexpr (sizeof(R) == 8)
          yn = fma(dq0, V0[4], stencil_elementwise(V, k8, wts));
        else
          yn = fma(dq0, V0[4], stencil_grouped(V, k8, wts));
        __builtin_nontemporal_store(yn, &y[(long)(k + 1) * g.pxy + doff]);
      }
      // plane k+2 replaces plane k, layer k+1 replaces layer k-1: both were
      // last read before the previous barrier
      put_plane(k + 2, QA);
      put_layer(k + 1, QAk);
      __syncthreads();
      dq0 = dq1;
      dq1 = dq2;
      dq2 = dn;
    };
    // a step names the slot it drains (QA) and the one it fills (QC); the
    // middle slot (QB) waits
    int k = k0;
    for (; k + 6 <= k1; k += 6) {
      step(k, V1, V2, V3, K1, K2, Q1, Q1k, Q3, Q3k);
      step(k + 1, V2, V3, V1, K2, K1, Q2, Q2k, Q1, Q1k);
      step(k + 2, V3, V1, V2, K1, K2, Q3, Q3k, Q2, Q2k);
      step(k + 3, V1, V2, V3, K2, K1, Q1, Q1k, Q3, Q3k);
      step(k + 4, V2, V3, V1, K1, K2, Q2, Q2k, Q1, Q1k);
      step(k + 5, V3, V1, V2, K2, K1, Q3, Q3k, Q2, Q2k);
    }
    if (k < k1) {
      step(k, V1, V2, V3, K1, K2, Q1, Q1k, Q3, Q3k);
      if (k + 1 < k1) {
        step(k + 1, V2, V3, V1, K2, K1, Q2, Q2k, Q1, Q1k);
        if (k + 2 < k1) {
          step(k + 2, V3, V1, V2, K1, K2, Q3, Q3k, Q2, Q2k);
          if (k + 3 < k1) {
            step(k + 3, V1, V2, V3, K2, K1, Q1, Q1k, Q3, Q3k);
            if (k + 4 < k1) step(k + 4, V2, V3, V1, K1, K2, Q2, Q2k, Q1, Q1k);
          }
        }
      }
    }
    __syncthreads();  // LDS is reused by the next work unit
  }
}

static inline void tiles_of(const Geo& g, int& ntx, int& nty, int& ntz) {
  ntx = (g.nx + TX - 1) / TX;
  nty = (g.ny + TY - 1) / TY;
  ntz = (g.nz + TZ - 1) / TZ;
}

// ---------------------------------------------------------------------------
// Batched Newton/CG kernels.  One launch serves a table of independent level
// solves ("items": one simulation's fine or coarse step, or many served
// requests' steps at once).  Item i owns a contiguous range of workgroups
// starting at a multiple of 8, so the XCD-aware tile order holds inside each
// item; every item has its own scalars and partial-sum regions.
// ---------------------------------------------------------------------------
// ---- composite-grid coupling helpers --------------------------------------
// Fine node (i, j, k) of the window lies on an immersed face (and not on the
// plate bottom): its value is slaved to the coarse interface nodes.
__device__ inline bool fine_gamma(const Geo& gf, const Window& w, int i, int j,
                                  int k);
// Coarse node (I, J, K) is an interface node: on an immersed face of the
// closed window box.
__device__ inline bool coarse_gamma(const Window& w, int I, int J, int K) {
  if (I < w.I0 || I > w.I0 + w.wx || J < w.J0 || J > w.J0 + w.wy || K < w.K0)
    return false;
  return ((w.faces & kFx0) && I == w.I0) ||
         ((w.faces & kFx1) && I == w.I0 + w.wx) ||
         ((w.faces & kFy0) && J == w.J0) ||
         ((w.faces & kFy1) && J == w.J0 + w.wy) ||
         ((w.faces & kFz0) && K == w.K0);
}
// Trilinear prolongation weight between fine node offset (di, dj, dk) (fine
// cells from the coarse node, |d| < r) -- the same formula in both
// directions, so P and P^T agree.
__device__ inline double pweight(int di, int dj, int dk, int r) {
  return (double)((r - abs(di)) * (r - abs(dj)) * (r - abs(dk))) /
         (double)(r * r * r);
}
// f(padded coarse index, weight) for the coarse nodes with a nonzero
// weight at window-local fine node (i, j, k).
template <class F>
__device__ inline void prolong_each(const Geo& gc, const Window& w, int i,
                                    int j, int k, F f) {
  const int r = w.r;
  const int ci = i / r, cj = j / r, ck = k / r;
  const int ri = i - ci * r, rj = j - cj * r, rk = k - ck * r;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int a = c & 1, b = (c >> 1) & 1, e = c >> 2;
    if ((a && ri == 0) || (b && rj == 0) || (e && rk == 0)) continue;
    const double wt = pweight(a ? r - ri : ri, b ? r - rj : rj,
                              e ? r - rk : rk, r);
    f(pidx(gc, w.I0 + ci + a, w.J0 + cj + b, w.K0 + ck + e), wt);
  }
}
// Fine coordinates of halo entry h, and whether it is a slaved interface
// node of a composite pair's fine side.
__device__ inline bool halo_gamma(const Geo& g, const Window& w, const Tile& t,
                                  int h, int& i, int& j, int& k) {
  i = t.ox + h % HX - 1;
  j = t.oy + (h / HX) % HY - 1;
  k = t.oz + h / (HX * HY) - 1;
  if (i < 0 || j < 0 || k < 0 || i >= g.nx || j >= g.ny || k >= g.nz)
    return false;
  return fine_gamma(g, w, i, j, k);
}
// Adds this thread's share of a region's tile partials to v: entries
// threadIdx.x, threadIdx.x + kBlock, ... in that order.  The loads of up to
// kSumBatch entries are issued together before any is added, so a
// workgroup waits on memory once per kSumBatch * kBlock tiles rather than
// once per kBlock (the order of the additions is unchanged).
// Region reg + qmax (qmax >= 0) takes the maximum instead of the sum.
constexpr int kSumBatch = 6;
template <int NV, class T, int B = kSumBatch>
__device__ inline void add_partials(gptr<const double> __restrict__ tp, int ts,
                                    int nt, int reg, T (&v)[NV],
                                    int qmax = -1) {
  for (int b0 = threadIdx.x; b0 < nt; b0 += B * kBlock) {
    double x[B][NV];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int b = b0 + u * kBlock;
#pragma unroll
      for (int q = 0; q < NV; ++q)
        x[u][q] = b < nt ? tp[(reg + q) * ts + b] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < B; ++u)
      if (b0 + u * kBlock < nt) {
#pragma unroll
        for (int q = 0; q < NV; ++q)
          v[q] = q == qmax ? fmax(v[q], (T)x[u][q]) : v[q] + (T)x[u][q];
      }
  }
}
// Sums of NV consecutive tile-partial regions starting at `reg` over an
// item's tiles -- for a composite pair, the fine tiles and then the coarse
// tiles, the same order on both sides.  Per-thread sums; the caller reduces
// over the workgroup.  (FP32 CG kernels keep one load per pass: their
// first tile's loads are in flight at the same time, and batching measured
// slower there.)
template <int NV, class T>
__device__ inline void pair_partials(const Couple& cp, int reg, T (&v)[NV]) {
  constexpr int B = sizeof(T) == 8 ? kSumBatch : 1;
  add_partials<NV, T, B>(gmem(cp.tpA), cp.tsA, cp.ntA, reg, v);
  add_partials<NV, T, B>(gmem(cp.tpB), cp.tsB, cp.ntB, reg, v);
}

// Every item of a batched launch has the same number of workgroups
// (`per_item`), so a workgroup finds its item and its rank within the item
// without reading the table.
__device__ inline int item_of_block(int per_item) { return blockIdx.x / per_item; }

// K4 + K1: nonlinear residual at the trial T - alpha dx, Jacobian
// coefficients, CG initial residual; partials of |R_free|^2, max|alpha dx|,
// r.(Dinv r).  LDS-tiled like the CG kernels: the trial temperature is
// formed once per halo node and each element's conductivity once per tile.
//
// Composite pairs (CP = kFineSide(P) / kCoarseSide): the fine side takes
// the trial values of its interface nodes prolonged from the coarse trial
// (kFineSide here, kFineSideP from couple_prolong_kernel), scales its rows
// by 1/m and keeps its
// Jacobian diagonal on the interface rows (in place of the preconditioner,
// which is the coarse row's there); the coarse side adds the gathered fine
// rows on its interface nodes.
template <class R, int CP>
__global__ void __launch_bounds__(kBlock)
residual_batched_kernel(const SolveItem* __restrict__ items, int per_item,
                        int round) {
  __shared__ double t_s[HN];
  __shared__ double k_s[EN];
  __shared__ double lds[6 * kBlock / 64];
  const SolveItem& it = items[item_of_block(per_item)];
  const gptr<const LevelScalars> lsc = gmem((const LevelScalars*)it.sc);
  const auto& st = lsc->ns[round & 1];
  if (st.status != kRunning) return;
  if (st.pending) {
    // the CG that should have produced the direction broke down at once:
    // the CG-start kernel of this round records the failure
    const auto& cgp = lsc->cg[(round + 1) & 1];
    if (cgp.breakdown && cgp.iters == 0) return;
  }
  const int blk = blockIdx.x % per_item, nblk = per_item;
  const Geo& g = it.g;
  const MatDev& m = it.m;
  const gptr<const double> __restrict__ T = gmem((const double*)it.Tb[st.cur]);
  const gptr<double> __restrict__ Tt = gmem(it.Tb[1 - st.cur]);
  const gptr<const R> __restrict__ dx =
      st.first ? nullptr : gmem((const R*)it.xb[st.xi]);
  const gptr<const double> __restrict__ Told = gmem(it.Told);
  const gptr<double> __restrict__ Hold = gmem(it.Hold);
  const gptr<const double> __restrict__ Fn = gmem(it.F);
  const gptr<const double> __restrict__ Fext = gmem(it.Fext);
  const gptr<double> __restrict__ Rout = gmem(it.R);
  const double alpha = st.alpha;
  const gptr<R> __restrict__ kap = gmem((R*)it.kap);
  const gptr<R> __restrict__ d = gmem((R*)it.d);
  const gptr<R> __restrict__ dinv = gmem((R*)it.dinv);
  const gptr<R> __restrict__ r = gmem((R*)it.r[0]);
  double w[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) w[q] = g.w[q];
  const gptr<double> __restrict__ tp = gmem(it.tpart);
  const int ts = it.tstride;
  // a tile's global inputs, loaded into registers in one batch at the top
  // of its turn (holding the next tile's during this one's work would cost
  // the kernel a wave per SIMD)
  double hT[HPT];
  R hd[HPT];
  // o_H: T_old in the first round (H(T_old) is formed and kept), H(T_old)
  // in later rounds
  double o_T = 0.0, o_H = 0.0, o_F = 0.0, o_Fx = 0.0;
  const bool first = st.first != 0;
  auto load_tile = [&](const Tile& t) {
#pragma unroll
    for (int q = 0; q < HPT; ++q) {
      const int h = threadIdx.x + q * kBlock;
      const int hn = h < HN ? halo_index_real(g, t, h) : -1;
      int fi, fj, fk;
      if (CP == kFineSide && hn >= 0 &&
          halo_gamma(g, it.cp.w, t, h, fi, fj, fk)) {
        // interface node: P of the coarse trial, no step of its own
        const gptr<const double> Tc = gmem(it.cp.oT[st.cur]);
        const gptr<const R> dxc =
            st.first ? nullptr : gmem((const R*)it.cp.ox[st.xi]);
        double v = 0.0;
        prolong_each(it.cp.go, it.cp.w, fi, fj, fk, [&](int cn, double wt) {
          v += wt * (dxc != nullptr ? trial_T(*at(Tc, cn), alpha * (double)*at(dxc, cn), m)
                                    : *at(Tc, cn));
        });
        hT[q] = v;
        hd[q] = (R)0;
      } else {
        hT[q] = hn >= 0 ? *at(T, hn) : 0.0;
        hd[q] = (hn >= 0 && dx != nullptr) ? *at(dx, hn) : (R)0;
      }
    }
    const int i = t.ox + t.tx, j = t.oy + t.ty, k = t.oz + t.tz;
    if (i < g.nx && j < g.ny && k < g.nz) {
      const int n = pidx(g, i, j, k);
      o_T = *at(T, n);
      o_H = first ? *at(Told, n) : *at(Hold, n);
      o_F = *at(Fn, n);
      if (Fext != nullptr) o_Fx = *at(Fext, n);
    }
  };
  const TileRange tr = tile_range(blk, nblk, it.ntiles);
  for (int tile = tr.first; tile < tr.last; tile += tr.step) {
    double acc[3] = {0.0, 0.0, 0.0};  // |R_free|^2, max|alpha dx|, r.z
    const Tile t = tile_at(it, tile);
    load_tile(t);
    const int i = t.ox + t.tx, j = t.oy + t.ty, k = t.oz + t.tz;
    const bool active = i < g.nx && j < g.ny && k < g.nz;
    const int n = active ? pidx(g, i, j, k) : 0;
    const double Tc0 = o_T, H_old = o_H, F_n = o_F, Fx_n = o_Fx;
    // trial temperature on the halo tile (entries past the grid are 0)
#pragma unroll
    for (int q = 0; q < HPT; ++q) {
      const int h = threadIdx.x + q * kBlock;
      if (h < HN)
        t_s[h] = dx != nullptr ? trial_T(hT[q], alpha * (double)hd[q], m) : hT[q];
    }
    __syncthreads();
    // conductivity of each element of the tile at its mean trial temperature
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = threadIdx.x + q * kBlock;
      if (e < EN) {
        const int ex = e % EX, ey = (e / EX) % EY, ez = e / (EX * EY);
        double ke = 0.0;
        const int gi = t.ox + ex - 1, gj = t.oy + ey - 1, gk = t.oz + ez - 1;
        if (elem_fictitious(it.rg, gi, gj, gk) && elem_active(g, it.rg, gi, gj, gk)) {
          ke = it.rg.kf;
        } else if (elem_active(g, it.rg, gi, gj, gk)) {
          double sm = 0.0;
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
            sm += t_s[(ez + cz) * (HX * HY) + (ey + cy) * HX + (ex + cx)];
          }
          ke = kappa_of(0.125 * sm, m);
        }
        k_s[e] = ke;
      }
    }
    __syncthreads();
    if (active) {
      const int c0 = (t.tz + 1) * (HX * HY) + (t.ty + 1) * HX + (t.tx + 1);
      auto TV = [&](int dxx, int dy, int dz) {
        return t_s[c0 + dz * (HX * HY) + dy * HX + dxx];
      };
      double k8[8];
      double nact = 0.0, nfict = 0.0;
      double diagK = 0.0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
        const double ke = k_s[(t.tz + 1 - ez) * (EX * EY) +
                              (t.ty + 1 - ey) * EX + (t.tx + 1 - ex)];
        if (elem_active(g, it.rg, i - ex, j - ey, k - ez)) {
          if (elem_fictitious(it.rg, i - ex, j - ey, k - ez))
            nfict += 1.0;
          else
            nact += 1.0;
        }
        k8[e] = ke;
        diagK += ke;
      }
      const double Tn = t_s[c0];
      const double mass = g.vol8 * nact;
      double Hn, dHn;
      enthalpy_and_slope(Tn, m, Hn, dHn);
      double Ho = H_old;
      if (first) {
        Ho = enthalpy(H_old, m);   // H_old holds T_old here
        *at(Hold, n) = Ho;
      }
      // K T, element by element.  Each element reads its eight corners from
      // LDS afresh (the empty asm keeps the compiler from holding all 27
      // values in registers across elements): 114-117 registers, 4 waves
      // per SIMD, where holding them took 146-154 and 3 waves; the same
      // sums in the same order as stencil_elementwise.
      double st_acc = 0.0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
        double sk = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int cx = c & 1, cy = (c >> 1) & 1, cz = c >> 2;
          sk = fma(w[e ^ c], TV(cx - ex, cy - ey, cz - ez), sk);
        }
        st_acc = fma(k8[e], sk, st_acc);
        asm volatile("" ::: "memory");
      }
      double Rn = mass * (Hn - Ho) / it.tau + st_acc - F_n;
      // elements with the consistent global problem's own coefficients:
      // their lumped mass takes rhoc_f (T - T_old) / tau
      const double mfict = g.vol8 * nfict * it.rg.rhocf;
      if (nfict > 0.0) Rn += mfict * (Tn - *at(Told, n)) / it.tau;
      if (Fext != nullptr) Rn -= Fx_n;
      // heat loss through the top surface and its (exact) slope
      double sd = 0.0;
      if (k == g.nz - 1 && (it.sf.h != 0.0 || it.sf.es != 0.0)) {
        const double A = top_area(g, it.rg, i, j);
        Rn += A * surface_flux(Tn, it.sf);
        sd = A * surface_slope(Tn, it.sf);
      }
      // coefficients of the frozen-kappa Jacobian J = diag(m H'/tau) + K[kap]
      const bool dir = node_dirichlet(g, it.rg, i, j, k);
      double dn = (mass * dHn + mfict) / it.tau + sd;
      double diag = dn + diagK * g.w[0];
      double kown = k8[0];
      bool keep_diag = false;
      if constexpr (CP == kFineSide || CP == kFineSideP) {
        const double sc = it.cp.rscale;
        Rn *= sc;
        dn *= sc;
        diag *= sc;
        kown *= sc;
        keep_diag = fine_gamma(g, it.cp.w, i, j, k);
      }
      if constexpr (CP == kCoarseSide) {
        if (coarse_gamma(it.cp.w, i, j, k)) {
          Rn += gmem(it.cp.gR)[n];
          diag += gmem((const double*)it.cp.gDW)[n];
        }
      }
      *at(Tt, n) = Tn;
      *at(Rout, n) = Rn;
      // this node owns the element whose lowest corner it is (k8[0])
      *at(kap, n) = (R)kown;
      *at(d, n) = (R)dn;
      const R di = dir ? (R)0 : (R)(1.0 / diag);
      *at(dinv, n) = keep_diag ? (R)diag : di;
      const R rn = dir ? (R)0 : (R)Rn;
      const R zn = di * rn;
      *at(r, n) = rn;
      if (!dir) {
        acc[0] += Rn * Rn;
        acc[1] = fmax(acc[1], fabs(Tn - Tc0));
        acc[2] += (double)(rn * zn);
      }
    }
    // the tile's partials; the max is taken separately from the two sums
    const double mx = wave_max(acc[1]);
    double sums[2] = {acc[0], acc[2]};
    block_sum<2>(sums, lds);
    if ((threadIdx.x & 63) == 0) lds[2 * kBlock / 64 + (threadIdx.x >> 6)] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      double bm = lds[2 * kBlock / 64];
      for (int wv = 1; wv < kBlock / 64; ++wv)
        bm = fmax(bm, lds[2 * kBlock / 64 + wv]);
      *at(tp, kTRes * ts + tile) = sums[0];
      *at(tp, (kTRes + 1) * ts + tile) = bm;
      *at(tp, (kTRes + 2) * ts + tile) = sums[1];
    }
    __syncthreads();  // LDS is reused by the next tile
  }
}

// Work units of the CG start and iteration kernels: stacks of S tiles
// along z (S = 1 or 2), so a thread holds node (tx, ty, tz) of each of the
// S tiles and a workgroup has S times the loads of one tile in flight.
// Stacks are numbered like tile_at (x fastest, then z, then y), with the z
// index in steps of S, and the partial sums stay per tile: the reductions
// add the same numbers in the same order whatever S is.  A launch takes
// stacks of two when each workgroup would walk two tiles (its largest item
// has more tiles than the workgroups it gets, but at most twice as many):
// one turn instead of two.  On the raster build's 1344-tile window that
// took 3 % off the FP64 macro step.  With fewer tiles, stacks would leave
// workgroups idle (the single track: 10 % slower); with many more tiles
// per workgroup (the served mix: 64 workgroups for 546 tiles) stacks lose
// the FP32 kernel's overlap of the next tile's loads with the stencil, and
// serving ran 1.5 % slower.
template <int S>
struct Stack {
  static constexpr int HN = HX * HY * (S * TZ + 2);   // halo nodes
  static constexpr int EN = EX * EY * (S * TZ + 1);   // elements
  static constexpr int HPT = (HN + kBlock - 1) / kBlock;
  static constexpr int EPT = (EN + kBlock - 1) / kBlock;
};
__device__ inline int item_ntz(const SolveItem& it) {
  return it.ntiles / (it.ntx * it.nty);
}
template <int S>
__device__ inline int stack_count(const SolveItem& it) {
  return it.ntx * it.nty * ((item_ntz(it) + S - 1) / S);
}
// Stack w: the tile of its lowest tile (this thread's node in it), the
// index of that tile in tile_at's numbering (tile s of the stack is
// b0 + s * ntx) and the number of tiles the stack holds (the top stack of
// an odd column of tiles holds fewer than S).
template <int S>
__device__ inline Tile stack_at(const SolveItem& it, int w, int& b0,
                                int& nsub) {
  const int ntz = item_ntz(it), nwz = (ntz + S - 1) / S;
  const int x = w % it.ntx, wz = (w / it.ntx) % nwz, y = w / (it.ntx * nwz);
  b0 = x + it.ntx * (wz * S + ntz * y);
  nsub = min(S, ntz - wz * S);
  Tile t;
  t.ox = x * TX;
  t.oy = y * TY;
  t.oz = wz * S * TZ;
  t.tx = threadIdx.x % TX;
  t.ty = (threadIdx.x / TX) % TY;
  t.tz = threadIdx.x / (TX * TY);
  return t;
}

// Newton state machine and CG start of round `round` (see the CG
// recurrences below).  Every workgroup of an item computes the same next
// state from the round's input state, the previous round's CG outcome and
// the residual partials; workgroup 0 stores it.
//  * A direction produced by the previous round's CG is accounted for
//    (Newton and CG counts, the most CG iterations a direction needed, 2
//    more when the budget cut the CG), or the solve fails when that CG broke
//    down at once.
//  * The trial is accepted on the first evaluation, on sufficient decrease
//    |R| <= (1 - 1e-4 alpha) rn0, when its step is within tol, or on the last
//    halving; Newton has converged when an accepted step is within tol
//    (and, when its direction's CG was cut by the budget, the accepted step
//    before it was within tol too).
//  * Rejected: the step is halved for the next round.  Accepted and not
//    converged: the trial becomes the accepted temperature and this round's
//    CG computes the next direction; w0 = J u0 (u0 = Dinv r0) and the
//    partials of gamma0 = r.u, delta0 = w.u are formed here.
//
// Composite pairs: both sides take the same decisions from the pair's
// partials; the fine side takes u0 on its interface nodes prolonged from
// the coarse u0 (kFineSide here, kFineSideP from couple_prolong_kernel) and
// leaves those rows out of its dot
// products, the coarse side adds the gathered fine rows of w0 on its
// interface nodes.
template <class R, int CP, int S>
__global__ void __launch_bounds__(kBlock)
cg_start_batched_kernel(const SolveItem* __restrict__ items, int per_item,
                        int round) {
  using ST = Stack<S>;
  __shared__ R u_s[ST::HN];
  __shared__ R k_s[ST::EN];
  __shared__ double lds[2 * kBlock / 64];
  __shared__ double ldm[kBlock / 64];
  __shared__ double bc[3];
  __shared__ R ldr[2 * S * kBlock / 64];
  const SolveItem& it = items[item_of_block(per_item)];
  const int blk = blockIdx.x % per_item, nblk = per_item;
  const Geo& g = it.g;
  const gptr<LevelScalars> sc = gmem(it.sc);
  const NewtonState st = gload<NewtonState>(&sc->ns[round & 1]);
  const auto& cgp = sc->cg[(round + 1) & 1];  // previous round's CG
  NewtonState nx = st;
  const int prev_iters = round > 0 ? cgp.iters : 0;
  if (st.status == kRunning && st.pending) {
    nx.pending = 0;
    if (cgp.breakdown && cgp.iters == 0) {
      nx.status = kFailBreakdown;
    } else {
      nx.n_newton += 1;
      nx.n_cg += cgp.iters;
      nx.cg_need = max(nx.cg_need, cgp.done ? cgp.iters : cgp.iters + 2);
      nx.dir_cut = cgp.done ? 0 : 1;
    }
  }
  // inputs of w0 = J u0 for a stack of tiles (the CG iteration's work
  // units), loaded into registers in one batch
  const gptr<const R> __restrict__ r = gmem((const R*)it.r[0]);
  const gptr<const R> __restrict__ dinv = gmem((const R*)it.dinv);
  const gptr<const R> __restrict__ d = gmem((const R*)it.d);
  const gptr<const R> __restrict__ kap = gmem((const R*)it.kap);
  R hr[ST::HPT], hd[ST::HPT], kr[ST::EPT];
  R o_r[S], o_d[S];
  int o_n[S];
  bool o_act[S], o_gam[S];
  auto load_stack = [&](const Tile& t) {
#pragma unroll
    for (int q = 0; q < ST::HPT; ++q) {
      const int h = threadIdx.x + q * kBlock;
      const int n = h < ST::HN ? halo_index_real(g, t, h) : -1;
      int fi, fj, fk;
      if (CP == kFineSide && n >= 0 &&
          halo_gamma(g, it.cp.w, t, h, fi, fj, fk)) {
        // interface node: u0 = P (Dinv r0) of the coarse side
        const gptr<const R> rc = gmem((const R*)it.cp.orr[0]);
        const gptr<const R> dc = gmem((const R*)it.cp.odinv);
        double v = 0.0;
        prolong_each(it.cp.go, it.cp.w, fi, fj, fk, [&](int cn, double wt) {
          v += wt * (double)(*at(dc, cn) * *at(rc, cn));
        });
        hr[q] = (R)v;
        hd[q] = (R)1;
      } else {
        hr[q] = n >= 0 ? *at(r, n) : (R)0;
        hd[q] = n >= 0 ? *at(dinv, n) : (R)0;
      }
    }
#pragma unroll
    for (int q = 0; q < ST::EPT; ++q) {
      const int e = threadIdx.x + q * kBlock;
      const int n = e < ST::EN ? elem_index_real(g, t, e) : -1;
      kr[q] = n >= 0 ? *at(kap, n) : (R)0;
    }
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const int i = t.ox + t.tx, j = t.oy + t.ty, k = t.oz + u * TZ + t.tz;
      o_act[u] = i < g.nx && j < g.ny && k < g.nz;
      o_n[u] = o_act[u] ? pidx(g, i, j, k) : 0;
      o_gam[u] = false;
      if (CP == kFineSide || CP == kFineSideP)
        o_gam[u] = o_act[u] && fine_gamma(g, it.cp.w, i, j, k);
      if (CP == kCoarseSide) o_gam[u] = o_act[u] && coarse_gamma(it.cp.w, i, j, k);
      o_r[u] = o_d[u] = (R)0;
      if (o_act[u]) {
        o_r[u] = *at(r, o_n[u]);
        o_d[u] = *at(d, o_n[u]);
      }
    }
  };
  const TileRange tr = tile_range(blk, nblk, stack_count<S>(it));
  int b0, nsub;
  // Loads ahead of use: the first stack's during the reduction, the next
  // one's during this one's stencil.  FP64 stacks of two load each stack at
  // the top of its turn instead (with loads ahead they take 168 to 179
  // registers and drop to 2 waves per SIMD, or spill when held to 3).
  constexpr bool kAhead = sizeof(R) == 4 || S == 1;
  double rnorm2 = 0.0, dmax = 0.0, rz = 0.0;
  bool run = false;
  if (nx.status == kRunning) {
    // the first stack's inputs are in flight during the reduction (not in
    // FP64 stacks of two: see below)
    if (kAhead && tr.first < tr.last)
      load_stack(stack_at<S>(it, tr.first, b0, nsub));
    // residual reductions over the item's tiles (every workgroup, same
    // order)
    const Couple& cp = it.cp;
    double a3[3] = {0.0, 0.0, 0.0};   // |R|^2, max|dx|, r.z
    add_partials<3, double, 2>(gmem(cp.tpA), cp.tsA, cp.ntA, kTRes, a3, 1);
    add_partials<3, double, 2>(gmem(cp.tpB), cp.tsB, cp.ntB, kTRes, a3, 1);
    double v[2] = {a3[0], a3[2]};
    double bm = wave_max(a3[1]);
    block_sum<2>(v, lds);
    if ((threadIdx.x & 63) == 0) ldm[threadIdx.x >> 6] = bm;
    __syncthreads();
    if (threadIdx.x == 0) {
      double mm = ldm[0];
      for (int wv = 1; wv < kBlock / 64; ++wv) mm = fmax(mm, ldm[wv]);
      bc[0] = v[0];
      bc[1] = mm;
      bc[2] = v[1];
    }
    __syncthreads();
    rnorm2 = bc[0];
    dmax = bc[1];
    rz = bc[2];
    const double rn = sqrt(rnorm2);
    const bool finite = isfinite(rnorm2) && isfinite(dmax);
    const bool accepted =
        st.first || !finite || rn <= (1.0 - 1e-4 * st.alpha) * st.rn0 ||
        dmax <= it.tol || st.h == kLineSearchMax - 1;
    // A step from a CG cut short by its budget can be shorter than the
    // Newton correction; it ends the iteration only when the accepted step
    // before it was within tol as well.
    const bool converged = !st.first && accepted && finite && dmax <= it.tol &&
                           (!st.dir_cut || st.dmax_last <= it.tol);
    if (!finite) {
      nx.status = kFailNonFinite;
    } else if (!accepted) {
      nx.h = st.h + 1;
      nx.alpha = ldexp(1.0, -nx.h);
      nx.n_halvings += 1;
    } else {
      nx.cur = 1 - st.cur;
      nx.rn0 = rn;
      nx.first = 0;
      if (!st.first) {
        nx.dmax_prev = st.dmax_last;
        nx.dmax_last = dmax;
      }
      if (converged || rz == 0.0) {
        nx.status = kConverged;
      } else if (nx.n_newton >= it.newton_max) {
        nx.status = kFailNewtonMax;
      } else {
        nx.xi = 1 - st.xi;
        nx.h = 0;
        nx.alpha = 1.0;
        nx.pending = 1;
        run = rz > 0.0;
        if (!run) nx.status = kFailBreakdown;
      }
    }
  }
  if (blk == 0 && threadIdx.x == 0) {
    gstore<NewtonState>(&sc->ns[(round + 1) & 1], nx);
    auto& cg = sc->cg[round & 1];
    cg.rz0 = rz;
    cg.iters = 0;
    cg.done = run ? 0 : 1;
    cg.breakdown = 0;
    if (st.status == kRunning && nx.status == kRunning) {
      sc->rnorm2 = rnorm2;
      sc->dmax = dmax;
    }
    if (round > 0) sc->cg_log[(round - 1) % kRoundLog] = prev_iters;
  }
  if (!run) return;
  // w0 = J u0, u0 = Dinv r0, on the stacks
  const gptr<R> __restrict__ w = gmem((R*)it.w[0]);
  R wts[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) wts[q] = (R)g.w[q];
  for (int ws = tr.first; ws < tr.last; ws += tr.step) {
    R acc[2 * S];
#pragma unroll
    for (int q = 0; q < 2 * S; ++q) acc[q] = (R)0;
    const Tile t = stack_at<S>(it, ws, b0, nsub);
    if (!kAhead) load_stack(t);
#pragma unroll
    for (int q = 0; q < ST::HPT; ++q) {
      const int h = threadIdx.x + q * kBlock;
      if (h < ST::HN) u_s[h] = hd[q] * hr[q];
    }
#pragma unroll
    for (int q = 0; q < ST::EPT; ++q) {
      const int e = threadIdx.x + q * kBlock;
      if (e < ST::EN) k_s[e] = kr[q];
    }
    __syncthreads();
    bool act[S], gam[S];
    int nn[S];
    R r_own[S], d_own[S];
#pragma unroll
    for (int u = 0; u < S; ++u) {
      act[u] = o_act[u];
      gam[u] = o_gam[u];
      nn[u] = o_n[u];
      r_own[u] = o_r[u];
      d_own[u] = o_d[u];
    }
    if (kAhead && ws + tr.step < tr.last) {
      int nb0, nns;
      load_stack(stack_at<S>(it, ws + tr.step, nb0, nns));
    }
#pragma unroll
    for (int u = 0; u < S; ++u) {
      if (!act[u]) continue;
      Tile tu = t;
      tu.tz += u * TZ;
      const int n = nn[u];
      const R un = u_s[(tu.tz + 1) * (HX * HY) + (tu.ty + 1) * HX + (tu.tx + 1)];
      R wn = fma(d_own[u], un, stencil_lds(tu, u_s, k_s, wts));
      if (CP == kCoarseSide && gam[u]) wn += gmem((const R*)it.cp.gDW)[n];
      *at(w, n) = wn;
      if ((CP != kFineSide && CP != kFineSideP) || !gam[u]) {
        acc[2 * u] = fma(r_own[u], un, acc[2 * u]);
        acc[2 * u + 1] = fma(wn, un, acc[2 * u + 1]);
      }
    }
    block_sum<2 * S>(acc, ldr);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int u = 0; u < S; ++u)
        if (u < nsub) {
          gmem(it.tpart)[kTCG * it.tstride + b0 + u * it.ntx] = (double)acc[2 * u];
          gmem(it.tpart)[(kTCG + 1) * it.tstride + b0 + u * it.ntx] = (double)acc[2 * u + 1];
        }
    }
    __syncthreads();  // LDS is reused by the next stack
  }
}

// One Chronopoulos-Gear PCG iteration `kit` for every item (LDS-tiled, in
// stacks of S tiles).
// Composite pairs: the fine side takes its interface nodes' inputs
// prolonged from the coarse vectors of iteration k (kFineSide here,
// kFineSideP from couple_prolong_kernel) and leaves those rows out of its
// dot products; the coarse side adds the
// gathered fine rows of w_{k+1} on its interface nodes.
template <class R, int CP, int S>
__global__ void __launch_bounds__(kBlock)
cg_iter_batched_kernel(const SolveItem* __restrict__ items, int per_item,
                       int round, int kit) {
  using ST = Stack<S>;
  __shared__ R u_s[ST::HN];
  __shared__ R k_s[ST::EN];
  __shared__ R lds[2 * S * kBlock / 64];
  __shared__ R bc[2];
  const SolveItem& it = items[item_of_block(per_item)];
  // the state written by this round's CG-start kernel
  const gptr<LevelScalars> lsc = gmem(it.sc);
  const auto& nst = lsc->ns[(round + 1) & 1];
  const gptr<CGScalars> sc = &lsc->cg[round & 1];
  // past the item's own budget (other items of the batch may run more): no
  // work, so the item's result does not depend on the batch
  if (sc->done || kit >= nst.budget) return;
  const int blk = blockIdx.x % per_item, nblk = per_item;
  const Geo& g = it.g;
  const int a = kit & 1;
  const gptr<const R> __restrict__ r_in = gmem((const R*)it.r[a]);
  const gptr<const R> __restrict__ w_in = gmem((const R*)it.w[a]);
  const gptr<const R> __restrict__ s_old = gmem((const R*)it.s[1 - a]);
  const gptr<R> __restrict__ r_out = gmem((R*)it.r[1 - a]);
  const gptr<R> __restrict__ w_out = gmem((R*)it.w[1 - a]);
  const gptr<R> __restrict__ s_out = gmem((R*)it.s[a]);
  const gptr<R> __restrict__ p = gmem((R*)it.p);
  const gptr<R> __restrict__ x = gmem((R*)it.xb[nst.xi]);
  const gptr<const R> __restrict__ d = gmem((const R*)it.d);
  const gptr<const R> __restrict__ kap = gmem((const R*)it.kap);
  const gptr<const R> __restrict__ dinv = gmem((const R*)it.dinv);
  // Every global input of a stack is loaded into registers in one batch:
  // the halo of r, w, s_{k-1}, Dinv (for u_{k+1}), the element
  // conductivities, and each node's own d, p, x, s_{k-1}.  Single tiles:
  // the first tile's batch is issued before the scalar reduction; in FP32
  // each later tile's while the previous tile's stencil is computed, in
  // FP64 at the top of its turn (overlapping the stencil as well takes 164
  // registers), so a workgroup waits on memory about once per tile.  Stacks
  // of two: FP32 as single tiles without the overlap with the stencil,
  // FP64 each stack at the top of its turn (with the first in flight during
  // the reduction the kernel takes 208 registers, 2 waves per SIMD).
  R hr[ST::HPT], hw[ST::HPT], hs[ST::HPT], hd[ST::HPT], kr[ST::EPT];
  R o_r[S], o_w[S], o_di[S], o_d[S], o_s[S], o_p[S], o_x[S];
  int o_n[S];
  bool o_act[S], o_gam[S];
  auto load_stack = [&](const Tile& t) {
#pragma unroll
    for (int q = 0; q < ST::HPT; ++q) {
      const int h = threadIdx.x + q * kBlock;
      const int n = h < ST::HN ? halo_index_real(g, t, h) : -1;
      int fi, fj, fk;
      if (CP == kFineSide && n >= 0 &&
          halo_gamma(g, it.cp.w, t, h, fi, fj, fk)) {
        // interface node: P (Dinv r), P (Dinv w), P (Dinv s) of the coarse
        // side with a unit preconditioner, so that the recurrence below
        // gives u_{k+1} = P (Dinv (r - alpha (w + beta s))) there
        const gptr<const R> rc = gmem((const R*)it.cp.orr[a]);
        const gptr<const R> wc = gmem((const R*)it.cp.ow[a]);
        const gptr<const R> scs = gmem((const R*)it.cp.os[1 - a]);
        const gptr<const R> dc = gmem((const R*)it.cp.odinv);
        double vr = 0.0, vw = 0.0, vs = 0.0;
        prolong_each(it.cp.go, it.cp.w, fi, fj, fk, [&](int cn, double wt) {
          const R dv = *at(dc, cn);
          vr += wt * (double)(dv * *at(rc, cn));
          vw += wt * (double)(dv * *at(wc, cn));
          if (kit > 0) vs += wt * (double)(dv * *at(scs, cn));
        });
        hr[q] = (R)vr;
        hw[q] = (R)vw;
        hs[q] = (R)vs;
        hd[q] = (R)1;
      } else {
        hr[q] = n >= 0 ? *at(r_in, n) : (R)0;
        hw[q] = n >= 0 ? *at(w_in, n) : (R)0;
        hs[q] = (n >= 0 && kit > 0) ? *at(s_old, n) : (R)0;
        hd[q] = n >= 0 ? *at(dinv, n) : (R)0;
      }
    }
#pragma unroll
    for (int q = 0; q < ST::EPT; ++q) {
      const int e = threadIdx.x + q * kBlock;
      const int n = e < ST::EN ? elem_index_real(g, t, e) : -1;
      kr[q] = n >= 0 ? *at(kap, n) : (R)0;
    }
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const int i = t.ox + t.tx, j = t.oy + t.ty, k = t.oz + u * TZ + t.tz;
      o_act[u] = i < g.nx && j < g.ny && k < g.nz;
      o_n[u] = o_act[u] ? pidx(g, i, j, k) : 0;
      o_gam[u] = false;
      if (CP == kFineSide || CP == kFineSideP)
        o_gam[u] = o_act[u] && fine_gamma(g, it.cp.w, i, j, k);
      if (CP == kCoarseSide) o_gam[u] = o_act[u] && coarse_gamma(it.cp.w, i, j, k);
      o_r[u] = o_w[u] = o_di[u] = o_d[u] = o_s[u] = o_p[u] = o_x[u] = (R)0;
      if (o_act[u]) {
        const int n = o_n[u];
        o_r[u] = *at(r_in, n);
        o_w[u] = *at(w_in, n);
        o_di[u] = *at(dinv, n);
        o_d[u] = *at(d, n);
        if (kit > 0) {
          o_s[u] = *at(s_old, n);
          o_p[u] = *at(p, n);
          o_x[u] = *at(x, n);
        }
      }
    }
  };
  const TileRange tr = tile_range(blk, nblk, stack_count<S>(it));
  int b0, nsub;
  constexpr bool kPre = sizeof(R) == 4 || S == 1;
  constexpr bool kNext = sizeof(R) == 4 && S == 1;
  if (kPre && tr.first < tr.last)
    load_stack(stack_at<S>(it, tr.first, b0, nsub));
  // gamma_k, delta_k from the previous kernel's partials (CG start or
  // iteration k-1), held in the region pair this kernel does not write
  const int rd = (kit & 1) ? kTCG2 : kTCG;
  const int wr = (kit & 1) ? kTCG : kTCG2;
  const int ts = it.tstride;
  {
    R v[2] = {(R)0, (R)0};
    pair_partials<2>(it.cp, rd, v);
    block_sum<2>(v, lds);
    if (threadIdx.x == 0) {
      bc[0] = v[0];
      bc[1] = v[1];
    }
    __syncthreads();
  }
  const R gamma = bc[0], delta = bc[1];
  R alpha, beta;
  if (kit == 0) {
    beta = (R)0;
    alpha = gamma / delta;
  } else {
    const R gamma_prev = (R)sc->gbuf[(kit - 1) & 1];
    const R alpha_prev = (R)sc->abuf[(kit - 1) & 1];
    if ((double)gamma <= it.rtol2 * sc->rz0 || !isfinite((double)gamma)) {
      if (blk == 0 && threadIdx.x == 0) {
        sc->done = 1;
        sc->iters = kit;
        if (!isfinite((double)gamma)) sc->breakdown = 2;
      }
      return;
    }
    beta = gamma / gamma_prev;
    alpha = gamma / (delta - beta * gamma / alpha_prev);
  }
  if (!(alpha > (R)0) || !isfinite((double)alpha)) {
    if (blk == 0 && threadIdx.x == 0) {
      sc->done = 1;
      sc->iters = kit;
      sc->breakdown = 1;
    }
    return;
  }
  if (blk == 0 && threadIdx.x == 0) {
    sc->gbuf[kit & 1] = (double)gamma;
    sc->abuf[kit & 1] = (double)alpha;
    sc->iters = kit + 1;
  }
  R wts[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) wts[q] = (R)g.w[q];
  for (int w = tr.first; w < tr.last; w += tr.step) {
    R acc[2 * S];
#pragma unroll
    for (int q = 0; q < 2 * S; ++q) acc[q] = (R)0;
    const Tile t = stack_at<S>(it, w, b0, nsub);
    if (!kNext && (!kPre || w != tr.first)) load_stack(t);
    // u_{k+1} = Dinv (r_k - alpha (w_k + beta s_{k-1})) on the halo
#pragma unroll
    for (int q = 0; q < ST::HPT; ++q) {
      const int h = threadIdx.x + q * kBlock;
      if (h < ST::HN)
        u_s[h] = hd[q] * fma(-alpha, fma(beta, hs[q], hw[q]), hr[q]);
    }
#pragma unroll
    for (int q = 0; q < ST::EPT; ++q) {
      const int e = threadIdx.x + q * kBlock;
      if (e < ST::EN) k_s[e] = kr[q];
    }
    __syncthreads();
    bool act[S], gamv[S];
    int nn[S];
    R r_own[S], w_own[S], di_own[S], d_own[S], s_prev[S], p_own[S], x_own[S];
#pragma unroll
    for (int u = 0; u < S; ++u) {
      act[u] = o_act[u];
      gamv[u] = o_gam[u];
      nn[u] = o_n[u];
      r_own[u] = o_r[u];
      w_own[u] = o_w[u];
      di_own[u] = o_di[u];
      d_own[u] = o_d[u];
      s_prev[u] = o_s[u];
      p_own[u] = o_p[u];
      x_own[u] = o_x[u];
    }
    if (kNext && w + tr.step < tr.last) {
      int nb0, nns;
      load_stack(stack_at<S>(it, w + tr.step, nb0, nns));
    }
    // the nodes' own recurrences and w_{k+1} = J u_{k+1}
#pragma unroll
    for (int u = 0; u < S; ++u) {
      if (!act[u]) continue;
      const int n = nn[u];
      Tile tu = t;
      tu.tz += u * TZ;
      // (a slaved interface node of a fine side keeps zero recurrences: its
      // values come from the coarse side)
      const bool gam = gamv[u];
      const bool slave = (CP == kFineSide || CP == kFineSideP) && gam;
      // (explicit fma throughout: every kernel instance rounds alike)
      const R s_k = slave ? (R)0 : fma(beta, s_prev[u], w_own[u]);
      const R u_k = di_own[u] * r_own[u];
      const R pn = slave ? (R)0 : fma(beta, p_own[u], u_k);
      *at(p, n) = pn;
      *at(s_out, n) = s_k;
      *at(x, n) = fma(alpha, pn, x_own[u]);
      const R r1 = slave ? (R)0 : fma(-alpha, s_k, r_own[u]);
      *at(r_out, n) = r1;
      const R u1 = u_s[(tu.tz + 1) * (HX * HY) + (tu.ty + 1) * HX + (tu.tx + 1)];
      R w1 = fma(d_own[u], u1, stencil_lds(tu, u_s, k_s, wts));
      if (CP == kCoarseSide && gam) w1 += gmem((const R*)it.cp.gDW)[n];
      *at(w_out, n) = w1;
      if ((CP != kFineSide && CP != kFineSideP) || !gam) {
        acc[2 * u] = fma(r1, u1, acc[2 * u]);
        acc[2 * u + 1] = fma(w1, u1, acc[2 * u + 1]);
      }
    }
    block_sum<2 * S>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int u = 0; u < S; ++u)
        if (u < nsub) {
          gmem(it.tpart)[wr * ts + b0 + u * it.ntx] = (double)acc[2 * u];
          gmem(it.tpart)[(wr + 1) * ts + b0 + u * it.ntx] = (double)acc[2 * u + 1];
        }
    }
    __syncthreads();  // LDS is reused by the next stack
  }
}

// Gather of composite pairs (over the coarse sides' table): for every
// coarse interface node J, sum_k P_kJ v_k over the fine interface nodes k
// in its support (fewer than r fine cells away on every axis) -- phase 0:
// the fine residual rows, and sum_k P_kJ^2 of the fine Jacobian diagonal as
// the preconditioner's share; phases 1 and 2: the fine rows of w = J u of
// the CG start or of iteration kit.  One workgroup per interface node, one
// thread per entry of a face patch, so all loads are in flight at once.
// The support's interface nodes lie on the immersed faces through J; each
// face's (2r-1)^2 patch is walked, and a node on two faces is taken on the
// first, so every fine node enters once.  Runs under the same conditions as
// the coarse side it feeds.
template <class R>
__global__ void __launch_bounds__(kBlock)
couple_gather_kernel(const SolveItem* __restrict__ items, int per_item,
                     int round, int phase, int kit) {
  __shared__ double lds[2 * kBlock / 64];
  const SolveItem& it = items[blockIdx.x / per_item];
  const Couple& cp = it.cp;
  const gptr<const LevelScalars> sc = gmem((const LevelScalars*)it.sc);
  if (phase == 0) {
    const auto& st = sc->ns[round & 1];
    if (st.status != kRunning) return;
    if (st.pending) {
      const auto& cgp = sc->cg[(round + 1) & 1];
      if (cgp.breakdown && cgp.iters == 0) return;
    }
  } else {
    const auto& nx = sc->ns[(round + 1) & 1];
    if (nx.status != kRunning || !nx.pending) return;
    if (phase == 2) {
      const auto& c = sc->cg[round & 1];
      if (c.done || kit >= nx.budget) return;
    }
  }
  const int q = blockIdx.x % per_item;
  if (q >= cp.ngamma) return;   // the whole workgroup
  const Geo& gc = it.g;
  const Geo& gf = cp.go;
  const Window& w = cp.w;
  const int n = gmem(cp.gidx)[q];
  const int I = n % gc.px - 1, J = (n / gc.px) % (gc.ny + 2) - 1,
            K = n / gc.pxy - 1;
  const int r = w.r, span = 2 * r - 1;
  // fine coordinates of the coarse node
  const int ci = r * (I - w.I0), cj = r * (J - w.J0), ck = r * (K - w.K0);
  const gptr<const R> fw = gmem((const R*)cp.fw[phase == 2 ? 1 - (kit & 1) : 0]);
  const gptr<const R> fdg = gmem((const R*)cp.fdiag);
  const gptr<const double> fR = gmem(cp.fR);
  double a[2] = {0.0, 0.0};
  for (int face = 0; face < 5; ++face) {
    const bool on =
        face == 0 ? ((w.faces & kFx0) && ci == 0)
      : face == 1 ? ((w.faces & kFx1) && ci == gf.nx - 1)
      : face == 2 ? ((w.faces & kFy0) && cj == 0)
      : face == 3 ? ((w.faces & kFy1) && cj == gf.ny - 1)
                  : ((w.faces & kFz0) && ck == 0);
    if (!on) continue;
    for (int t = threadIdx.x; t < span * span; t += kBlock) {
      const int u = t % span - (r - 1), v = t / span - (r - 1);
      const int fi = face < 2 ? ci : ci + u;
      const int fj = face < 2 ? cj + u : (face < 4 ? cj : cj + v);
      const int fk = face < 4 ? ck + v : ck;
      if (fi < 0 || fj < 0 || fk < 0 || fi >= gf.nx || fj >= gf.ny ||
          fk >= gf.nz)
        continue;
      if (w.bottom && fk == 0) continue;   // plate bottom: fixed, not slaved
      // a node also on an earlier immersed face was taken there
      if ((face > 0 && (w.faces & kFx0) && fi == 0) ||
          (face > 1 && (w.faces & kFx1) && fi == gf.nx - 1) ||
          (face > 2 && (w.faces & kFy0) && fj == 0) ||
          (face > 3 && (w.faces & kFy1) && fj == gf.ny - 1))
        continue;
      const double wt = pweight(fi - ci, fj - cj, fk - ck, r);
      const int fn = pidx(gf, fi, fj, fk);
      if (phase == 0) {
        a[0] += wt * fR[fn];
        a[1] += wt * wt * (double)fdg[fn];
      } else {
        a[0] += wt * (double)fw[fn];
      }
    }
  }
  block_sum<2>(a, lds);
  if (threadIdx.x == 0) {
    if (phase == 0) {
      gmem(cp.gR)[n] = a[0];
      gmem((double*)cp.gDW)[n] = a[1];
    } else {
      gmem((R*)cp.gDW)[n] = (R)a[0];
    }
  }
}

// Prolongation of composite pairs (over the fine sides' table), before each
// fine-side launch: the slaved interface nodes of the window get the
// prolonged coarse values the fine kernel then reads like any other --
// phase 0, the trial temperature P trial(T+, alpha dx+) into the accepted
// buffer (its own direction there stays zero); phase 1, u0 = P (Dinv r0)
// with a unit preconditioner; phase 2, P (Dinv r), P (Dinv w) and
// P (Dinv s) of CG iteration kit, so that the fine recurrence gives
// u_{k+1} = P (Dinv (r - alpha (w + beta s))) there by linearity.  The
// nodes are enumerated face by face (a node on two immersed faces is taken
// on the first); each is written once.  Runs under the same conditions as
// the fine side that follows it.
template <class R>
__global__ void __launch_bounds__(kBlock)
couple_prolong_kernel(const SolveItem* __restrict__ items, int per_item,
                      int round, int phase, int kit) {
  const SolveItem& it = items[blockIdx.x / per_item];
  const int blk = blockIdx.x % per_item;
  const gptr<const LevelScalars> sc = gmem((const LevelScalars*)it.sc);
  const auto& st = sc->ns[round & 1];
  if (phase <= 1) {
    if (st.status != kRunning) return;
    if (st.pending) {
      const auto& cgp = sc->cg[(round + 1) & 1];
      if (cgp.breakdown && cgp.iters == 0) return;
    }
  } else {
    const auto& nx = sc->ns[(round + 1) & 1];
    const auto& c = sc->cg[round & 1];
    if (c.done || kit >= nx.budget) return;
  }
  const Geo& g = it.g;
  const Couple& cp = it.cp;
  const Window& w = cp.w;
  const int a = kit & 1;
  const long sx = (long)g.ny * g.nz, sy = (long)g.nx * g.nz,
             sz = (long)g.nx * g.ny;
  const long total = 2 * sx + 2 * sy + sz;
  for (long t = (long)blk * kBlock + threadIdx.x; t < total;
       t += (long)per_item * kBlock) {
    int face, i, j, k;
    long u = t;
    if (u < 2 * sx) {
      face = u < sx ? 0 : 1;
      u -= face * sx;
      i = face == 0 ? 0 : g.nx - 1;
      j = (int)(u % g.ny);
      k = (int)(u / g.ny);
    } else if (u < 2 * sx + 2 * sy) {
      u -= 2 * sx;
      face = u < sy ? 2 : 3;
      u -= (face - 2) * sy;
      j = face == 2 ? 0 : g.ny - 1;
      i = (int)(u % g.nx);
      k = (int)(u / g.nx);
    } else {
      u -= 2 * sx + 2 * sy;
      face = 4;
      k = 0;
      i = (int)(u % g.nx);
      j = (int)(u / g.nx);
    }
    const int bit = face == 0 ? kFx0 : face == 1 ? kFx1 : face == 2 ? kFy0
                  : face == 3 ? kFy1 : kFz0;
    if (!(w.faces & bit)) continue;
    if (w.bottom && k == 0) continue;   // plate bottom: fixed, not slaved
    // taken on an earlier immersed face
    if ((face > 0 && (w.faces & kFx0) && i == 0) ||
        (face > 1 && (w.faces & kFx1) && i == g.nx - 1) ||
        (face > 2 && (w.faces & kFy0) && j == 0) ||
        (face > 3 && (w.faces & kFy1) && j == g.ny - 1))
      continue;
    const int n = pidx(g, i, j, k);
    if (phase == 0) {
      const gptr<const double> Tc = gmem(cp.oT[st.cur]);
      const gptr<const R> dxc =
          st.first ? nullptr : gmem((const R*)cp.ox[st.xi]);
      double v = 0.0;
      prolong_each(cp.go, w, i, j, k, [&](int cn, double wt) {
        v += wt * (dxc != nullptr ? trial_T(Tc[cn], st.alpha * (double)dxc[cn], it.m)
                                  : Tc[cn]);
      });
      gmem(it.Tb[st.cur])[n] = v;
    } else if (phase == 1) {
      const gptr<const R> rc = gmem((const R*)cp.orr[0]);
      const gptr<const R> dc = gmem((const R*)cp.odinv);
      double v = 0.0;
      prolong_each(cp.go, w, i, j, k, [&](int cn, double wt) {
        v += wt * (double)(dc[cn] * rc[cn]);
      });
      gmem((R*)it.r[0])[n] = (R)v;
      gmem((R*)it.dinv)[n] = (R)1;
    } else {
      const gptr<const R> rc = gmem((const R*)cp.orr[a]);
      const gptr<const R> wc = gmem((const R*)cp.ow[a]);
      const gptr<const R> scs = gmem((const R*)cp.os[1 - a]);
      const gptr<const R> dc = gmem((const R*)cp.odinv);
      double vr = 0.0, vw = 0.0, vs = 0.0;
      prolong_each(cp.go, w, i, j, k, [&](int cn, double wt) {
        const R dv = dc[cn];
        vr += wt * (double)(dv * rc[cn]);
        vw += wt * (double)(dv * wc[cn]);
        if (kit > 0) vs += wt * (double)(dv * scs[cn]);
      });
      gmem((R*)it.r[a])[n] = (R)vr;
      gmem((R*)it.w[a])[n] = (R)vw;
      gmem((R*)it.s[1 - a])[n] = (R)vs;
    }
  }
}

int grid_tiles(const Geo& g, int& ntx, int& nty) {
  int ntz;
  tiles_of(g, ntx, nty, ntz);
  return ntx * nty * ntz;
}
int cg_stacks(const Geo& g) {
  int ntx, nty, ntz;
  tiles_of(g, ntx, nty, ntz);
  return ntx * nty * ((ntz + 1) / 2);
}

// Workgroups of a kernel that the device holds at once: the occupancy
// limit per compute unit (set by its registers and LDS) times the compute
// units.  Taken once per kernel.
template <class F>
static int resident_blocks(F kernel) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
          hipSuccess ||
      cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) !=
          hipSuccess ||
      per_cu <= 0)
    per_cu = 1;
  return per_cu * cus;
}

int item_tile_blocks(int ntiles, int n_items, int resident) {
  const int share =
      std::max(64, (int)(kResidentShare * resident) / std::max(1, n_items)) /
      kXcd * kXcd;
  return std::min(tiled_grid(ntiles), share);
}

// The tiled launches below take the tile count of the batch's largest item
// and size the grid from the kernel's own residency.
template <class R, int CP>
static void launch_residual(Launch L, const SolveItem* items, int n_items,
                            int ntiles, int round) {
  static const int resident = resident_blocks(residual_batched_kernel<R, CP>);
  const int per_item = item_tile_blocks(ntiles, n_items, resident);
  hipLaunchKernelGGL((residual_batched_kernel<R, CP>),
                     dim3(n_items * per_item), dim3(kBlock), 0,
                     (hipStream_t)L.stream, items, per_item, round);
}
// The CG kernels in stacks of two when each workgroup would walk two
// single tiles (see Stack).
static inline bool use_stacks(int per1, int ntiles) {
  return per1 < ntiles && ntiles <= 2 * per1;
}
template <class R, int CP>
static void launch_cg_start(Launch L, const SolveItem* items, int n_items,
                            int ntiles, int nstacks, int round) {
  static const int res1 = resident_blocks(cg_start_batched_kernel<R, CP, 1>);
  static const int res2 = resident_blocks(cg_start_batched_kernel<R, CP, 2>);
  const int per1 = item_tile_blocks(ntiles, n_items, res1);
  if (!use_stacks(per1, ntiles)) {
    hipLaunchKernelGGL((cg_start_batched_kernel<R, CP, 1>),
                       dim3(n_items * per1), dim3(kBlock), 0,
                       (hipStream_t)L.stream, items, per1, round);
  } else {
    const int per2 = item_tile_blocks(nstacks, n_items, res2);
    hipLaunchKernelGGL((cg_start_batched_kernel<R, CP, 2>),
                       dim3(n_items * per2), dim3(kBlock), 0,
                       (hipStream_t)L.stream, items, per2, round);
  }
}
template <class R, int CP, int S>
static void launch_cg_iter_s(Launch L, const SolveItem* items, int n_items,
                             int per_item, int round, int kit, void* ev_start,
                             void* ev_stop) {
  if (ev_start != nullptr)
    hipExtLaunchKernelGGL((cg_iter_batched_kernel<R, CP, S>),
                          dim3(n_items * per_item), dim3(kBlock), 0,
                          (hipStream_t)L.stream, (hipEvent_t)ev_start,
                          (hipEvent_t)ev_stop, 0, items, per_item, round, kit);
  else
    hipLaunchKernelGGL((cg_iter_batched_kernel<R, CP, S>),
                       dim3(n_items * per_item), dim3(kBlock), 0,
                       (hipStream_t)L.stream, items, per_item, round, kit);
}
template <class R, int CP>
static void launch_cg_iter(Launch L, const SolveItem* items, int n_items,
                           int ntiles, int nstacks, int round, int kit,
                           void* ev_start, void* ev_stop) {
  static const int res1 = resident_blocks(cg_iter_batched_kernel<R, CP, 1>);
  static const int res2 = resident_blocks(cg_iter_batched_kernel<R, CP, 2>);
  const int per1 = item_tile_blocks(ntiles, n_items, res1);
  if (!use_stacks(per1, ntiles))
    launch_cg_iter_s<R, CP, 1>(L, items, n_items, per1, round, kit, ev_start,
                               ev_stop);
  else
    launch_cg_iter_s<R, CP, 2>(L, items, n_items,
                               item_tile_blocks(nstacks, n_items, res2), round,
                               kit, ev_start, ev_stop);
}
template <class R>
void k_residual_batched(Launch L, const SolveItem* items, int n_items,
                        int ntiles, int round) {
  launch_residual<R, kAlone>(L, items, n_items, ntiles, round);
}
template <class R>
void k_cg_start_batched(Launch L, const SolveItem* items, int n_items,
                        int ntiles, int nstacks, int round) {
  launch_cg_start<R, kAlone>(L, items, n_items, ntiles, nstacks, round);
}
template <class R>
void k_cg_iter_batched(Launch L, const SolveItem* items, int n_items,
                       int ntiles, int nstacks, int round, int kit,
                       void* ev_start, void* ev_stop) {
  launch_cg_iter<R, kAlone>(L, items, n_items, ntiles, nstacks, round, kit,
                            ev_start, ev_stop);
}
template <class R>
void k_residual_pair(Launch L, const SolveItem* items, int n_items,
                     int ntiles, int round, int side) {
  if (side == kFineSide)
    launch_residual<R, kFineSide>(L, items, n_items, ntiles, round);
  else if (side == kFineSideP)
    launch_residual<R, kFineSideP>(L, items, n_items, ntiles, round);
  else
    launch_residual<R, kCoarseSide>(L, items, n_items, ntiles, round);
}
template <class R>
void k_cg_start_pair(Launch L, const SolveItem* items, int n_items,
                     int ntiles, int nstacks, int round, int side) {
  if (side == kFineSide)
    launch_cg_start<R, kFineSide>(L, items, n_items, ntiles, nstacks, round);
  else if (side == kFineSideP)
    launch_cg_start<R, kFineSideP>(L, items, n_items, ntiles, nstacks, round);
  else
    launch_cg_start<R, kCoarseSide>(L, items, n_items, ntiles, nstacks, round);
}
template <class R>
void k_cg_iter_pair(Launch L, const SolveItem* items, int n_items,
                    int ntiles, int nstacks, int round, int kit, int side,
                    void* ev_start, void* ev_stop) {
  if (side == kFineSide)
    launch_cg_iter<R, kFineSide>(L, items, n_items, ntiles, nstacks, round,
                                 kit, ev_start, ev_stop);
  else if (side == kFineSideP)
    launch_cg_iter<R, kFineSideP>(L, items, n_items, ntiles, nstacks, round,
                                  kit, ev_start, ev_stop);
  else
    launch_cg_iter<R, kCoarseSide>(L, items, n_items, ntiles, nstacks, round,
                                   kit, ev_start, ev_stop);
}
template <class R>
void k_couple_prolong(Launch L, const SolveItem* fine_items, int n_items,
                      int per_item, int round, int phase, int kit) {
  hipLaunchKernelGGL(couple_prolong_kernel<R>, dim3(n_items * per_item),
                     dim3(kBlock), 0, (hipStream_t)L.stream, fine_items,
                     per_item, round, phase, kit);
}
template <class R>
void k_couple_gather(Launch L, const SolveItem* coarse_items, int n_items,
                     int max_gamma, int round, int phase, int kit) {
  const int per = std::max(1, max_gamma);   // one workgroup per interface node
  hipLaunchKernelGGL(couple_gather_kernel<R>, dim3(n_items * per),
                     dim3(kBlock), 0, (hipStream_t)L.stream, coarse_items, per,
                     round, phase, kit);
}
#define TL_BATCH_INST(R)                                                     \
  template void k_residual_batched<R>(Launch, const SolveItem*, int, int,    \
                                      int);                                  \
  template void k_cg_start_batched<R>(Launch, const SolveItem*, int, int,    \
                                      int, int);                             \
  template void k_cg_iter_batched<R>(Launch, const SolveItem*, int, int, int, \
                                     int, int, void*, void*);                \
  template void k_residual_pair<R>(Launch, const SolveItem*, int, int, int,  \
                                   int);                                     \
  template void k_cg_start_pair<R>(Launch, const SolveItem*, int, int, int,  \
                                   int, int);                                \
  template void k_cg_iter_pair<R>(Launch, const SolveItem*, int, int, int,   \
                                  int, int, int, void*, void*);              \
  template void k_couple_gather<R>(Launch, const SolveItem*, int, int, int,  \
                                   int, int);                                \
  template void k_couple_prolong<R>(Launch, const SolveItem*, int, int, int, \
                                    int, int);
TL_BATCH_INST(float)
TL_BATCH_INST(double)
#undef TL_BATCH_INST

// Grids of more than kZmarchNodes nodes take the z-marching kernel; smaller
// ones, cache-resident and latency-bound, the 3D-tiled kernel.
constexpr long kZmarchNodes = 4l << 20;

template <class R>
void k_op_apply(Launch L, const Geo& g, int kernel, int blocks, const R* d,
                const R* kap, const R* v, R* y) {
  if (kernel == kOpAuto)
    kernel = (long)g.nreal > kZmarchNodes && g.nz >= 8 ? kOpZmarch : kOpTiled;
  if (kernel == kOpZmarch) {
    const ZPlan zp = zplan_of<R>(g);
    const int units = zp.ncx * zp.ncy * zp.nrun;
    // one round of workgroups, no more than the device holds at once, each
    // walking its XCD's units: on a 640 x 640 x 160 grid that is 768
    // workgroups in FP64 and 1024 in FP32, 0.6-2 % faster than 2048, while
    // 1024 in FP64 (a partial second round) was 12 % slower
    static const int resident =
        std::max(kXcd, resident_blocks(op_apply_zmarch_kernel<R>) / kXcd * kXcd);
    hipLaunchKernelGGL(op_apply_zmarch_kernel<R>,
                       dim3(blocks > 0 ? blocks
                                       : std::min(tiled_grid(units), resident)),
                       dim3(kBlock), 0, (hipStream_t)L.stream, g, zp, d, kap,
                       v, y);
    return;
  }
  int ntx, nty, ntz;
  tiles_of(g, ntx, nty, ntz);
  const int ntiles = ntx * nty * ntz;
  hipLaunchKernelGGL(op_apply_tiled_kernel<R>,
                     dim3(blocks > 0 ? blocks : tiled_grid(ntiles)),
                     dim3(kBlock), 0, (hipStream_t)L.stream, g, ntx, nty,
                     ntiles, d, kap, v, y);
}
template void k_op_apply<float>(Launch, const Geo&, int, int, const float*,
                                const float*, const float*, float*);
template void k_op_apply<double>(Launch, const Geo&, int, int, const double*,
                                 const double*, const double*, double*);

// ---------------------------------------------------------------------------
// K6: surface laser load F_i = sum over top faces of int q phi_i dA (n_q x n_q
// Gauss per face), averaged over the spots with their weights.  Faces with
// fI0 <= i < fI1 and fJ0 <= j < fJ1 are skipped (the window's faces in the
// coarse outside load).  Adds scale * sum(F) into *ledger_slot.
// ---------------------------------------------------------------------------
// The flux and the face's bilinear basis are products of an x and a y
// factor, and so is the tensor Gauss rule: the integral over face (fi, fj)
// of q phi for the node at corner (ca, cb) is q0 hx hy gx(fi, ca) gy(fj, cb)
// with gx(fi, ca) = sum_a w_a exp(-a3 (x_a - xc)^2) phi_ca(xi_a) -- 2 n_q
// exponentials per face and spot instead of n_q^2.
__device__ inline double gauss_line(int nq, const double* gx, const double* gw,
                                    double x0, int f, double h, double c,
                                    double a3, int side) {
  double acc = 0.0;
  for (int qa = 0; qa < nq; ++qa) {
    const double xi = gx[qa];
    const double r = x0 + (f + xi) * h - c;
    acc += gw[qa] * exp(-a3 * r * r) * (side ? xi : 1.0 - xi);
  }
  return acc;
}
// Surface load of one spot at top node (i, j) with the faces of the box
// [fI0, fI1) x [fJ0, fJ1) left out.
__device__ inline double spot_load(const Geo& g, int nq, const double* gx,
                                   const double* gw, const Spot& S, int i,
                                   int j, int fI0, int fI1, int fJ0, int fJ1) {
  // this node is corner (1 - fa, 1 - fb) of face (i - 1 + fa, j - 1 + fb)
  double fx[2] = {0.0, 0.0}, fy[2] = {0.0, 0.0};
  for (int fa = 0; fa < 2; ++fa) {
    const int fi = i - 1 + fa;
    if (fi >= 0 && fi <= g.nx - 2)
      fx[fa] = gauss_line(nq, gx, gw, g.x0, fi, g.hx, S.xc, S.a3, 1 - fa);
    const int fj = j - 1 + fa;
    if (fj >= 0 && fj <= g.ny - 2)
      fy[fa] = gauss_line(nq, gx, gw, g.y0, fj, g.hy, S.yc, S.a3, 1 - fa);
  }
  double fs = 0.0;
  for (int fb = 0; fb < 2; ++fb)
    for (int fa = 0; fa < 2; ++fa) {
      const int fi = i - 1 + fa, fj = j - 1 + fb;
      if (fi >= fI0 && fi < fI1 && fj >= fJ0 && fj < fJ1) continue;
      fs += fx[fa] * fy[fb];
    }
  return (S.q0 * g.hx * g.hy) * fs;
}

__global__ void __launch_bounds__(kBlock)
laser_load_kernel(Geo g, SpotSet sp, int fI0, int fI1, int fJ0, int fJ1,
                  double* __restrict__ F, double* partials) {
  __shared__ double lds[kBlock / 64];
  double acc[1] = {0.0};
  const int ntop = g.nx * g.ny;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntop;
       t += gridDim.x * blockDim.x) {
    const int i = t % g.nx, j = t / g.nx;
    double f = 0.0;
    for (int s = 0; s < sp.n; ++s)
      f += sp.s[s].weight *
           spot_load(g, sp.nq, sp.gx, sp.gw, sp.s[s], i, j, fI0, fI1, fJ0, fJ1);
    F[pidx(g, i, j, g.nz - 1)] = f;
    acc[0] += f;
  }
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) partials[kPartGen * kMaxBlocks + blockIdx.x] = acc[0];
}

void k_laser_load(Launch L, const Geo& g, const SpotSet& spots, int fI0,
                  int fI1, int fJ0, int fJ1, double* F, double ledger_scale,
                  double* ledger_slot, double* partials) {
  const int nb = grid_for((long)g.nx * g.ny);
  hipLaunchKernelGGL(laser_load_kernel, dim3(nb), dim3(kBlock), 0,
                     (hipStream_t)L.stream, g, spots, fI0, fI1, fJ0, fJ1, F,
                     partials);
  if (ledger_slot != nullptr)
    finalize_sum(L, partials + kPartGen * kMaxBlocks, nb, ledger_scale,
                 ledger_slot, 0);
}

// ---------------------------------------------------------------------------
// Volume laser model (paper Section 5.2).  Depths are measured from the top
// node layer (the plate top on both levels): node layer k sits at
// zeta = (k - (nz - 1)) hz <= 0.
// ---------------------------------------------------------------------------
// int over [a, b] of exp(-alpha (x - c)^2) and of x exp(-alpha (x - c)^2)
__device__ inline void gauss_moments(double a, double b, double c, double alpha,
                                     double& m0, double& m1) {
  const double sa = sqrt(alpha);
  m0 = 0.5 * sqrt(M_PI / alpha) * (erf(sa * (b - c)) - erf(sa * (a - c)));
  m1 = c * m0 - (exp(-alpha * (b - c) * (b - c)) -
                 exp(-alpha * (a - c) * (a - c))) / (2.0 * alpha);
}
// int exp(-alpha (x - c)^2) phi_i(x) dx for the hat function of node i of a
// line of n nodes x0 + i h
__device__ inline double hat_gauss(int i, int n, double h, double x0, double c,
                                   double alpha) {
  const double xi = x0 + i * h;
  double G = 0.0, m0, m1;
  if (i > 0) {
    gauss_moments(xi - h, xi, c, alpha, m0, m1);
    G += (m1 - (xi - h) * m0) / h;
  }
  if (i < n - 1) {
    gauss_moments(xi, xi + h, c, alpha, m0, m1);
    G += ((xi + h) * m0 - m1) / h;
  }
  return G;
}

// F_i = int Q- phi_i dV: the Gaussian and the Q1 basis factor by axis, so
// F_i = amp Gx(i) Gy(j) Gz(k) with the closed forms above.
__global__ void __launch_bounds__(kBlock)
volume_load_kernel(Geo g, VolSpot sp, double* __restrict__ F,
                   double* partials) {
  __shared__ double lds[kBlock / 64];
  double acc[1] = {0.0};
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < g.nreal;
       t += gridDim.x * blockDim.x) {
    int i, j, k;
    node_ijk(g, t, i, j, k);
    double f = 0.0;
    if (sp.on) {
      f = sp.amp * hat_gauss(i, g.nx, g.hx, g.x0, sp.xc, sp.a3) *
          hat_gauss(j, g.ny, g.hy, g.y0, sp.yc, sp.a3) *
          hat_gauss(k, g.nz, g.hz, -(g.nz - 1) * g.hz, 0.0, sp.az);
    }
    F[pidx(g, i, j, k)] = f;
    acc[0] += f;
  }
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) partials[kPartGen * kMaxBlocks + blockIdx.x] = acc[0];
}

void k_volume_load(Launch L, const Geo& g, const VolSpot& sp, double* F,
                   double ledger_scale, double* ledger_slot, double* partials) {
  const int nb = grid_for(g.nreal);
  hipLaunchKernelGGL(volume_load_kernel, dim3(nb), dim3(kBlock), 0,
                     (hipStream_t)L.stream, g, sp, F, partials);
  if (ledger_slot != nullptr)
    finalize_sum(L, partials + kPartGen * kMaxBlocks, nb, ledger_scale,
                 ledger_slot, 0);
}

// int over [lo, hi] ∩ [e0, e0 + h] of the falling and the rising 1D basis
// function of the cell [e0, e0 + h]
__device__ inline void hat_box(double lo, double hi, double e0, double h,
                               double& fall, double& rise) {
  const double a = fmin(fmax(lo, e0), e0 + h);
  const double b = fmin(fmax(hi, e0), e0 + h);
  rise = ((b - e0) * (b - e0) - (a - e0) * (a - e0)) / (2.0 * h);
  fall = (b - a) - rise;
}

// F_i = sum over boxes of q int_{box ∩ e} phi_i over the elements e around
// node i that the region keeps: the part of an element inside an
// axis-aligned box is a box, and the trilinear basis integrates over it as
// a product of 1D integrals.
__global__ void __launch_bounds__(kBlock)
box_load_kernel(Geo g, Region rg, BoxSet bs, double* __restrict__ F,
                double* partials) {
  __shared__ double lds[kBlock / 64];
  double acc[1] = {0.0};
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < g.nreal;
       t += gridDim.x * blockDim.x) {
    int i, j, k;
    node_ijk(g, t, i, j, k);
    double f = 0.0;
    for (int e = 0; e < 8; ++e) {
      const int a = e & 1, b = (e >> 1) & 1, c = e >> 2;
      // the element of which this node is corner (a, b, c)
      const int ei = i - a, ej = j - b, ek = k - c;
      if (!elem_active(g, rg, ei, ej, ek)) continue;
      const double ex = g.x0 + ei * g.hx, ey = g.y0 + ej * g.hy;
      const double ez = (ek - (g.nz - 1)) * g.hz;
      for (int q = 0; q < bs.n; ++q) {
        const Box& B = bs.b[q];
        double fx0, fx1, fy0, fy1, fz0, fz1;
        hat_box(B.x_lo, B.x_hi, ex, g.hx, fx0, fx1);
        hat_box(B.y_lo, B.y_hi, ey, g.hy, fy0, fy1);
        hat_box(-B.depth, 0.0, ez, g.hz, fz0, fz1);
        f += B.q * (a ? fx1 : fx0) * (b ? fy1 : fy0) * (c ? fz1 : fz0);
      }
    }
    F[pidx(g, i, j, k)] = f;
    acc[0] += f;
  }
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) partials[kPartGen * kMaxBlocks + blockIdx.x] = acc[0];
}

void k_box_load(Launch L, const Geo& g, const Region& rg, const BoxSet& bs,
                double* F, double ledger_scale, double* ledger_slot,
                double* partials) {
  const int nb = grid_for(g.nreal);
  hipLaunchKernelGGL(box_load_kernel, dim3(nb), dim3(kBlock), 0,
                     (hipStream_t)L.stream, g, rg, bs, F, partials);
  if (ledger_slot != nullptr)
    finalize_sum(L, partials + kPartGen * kMaxBlocks, nb, ledger_scale,
                 ledger_slot, 0);
}

// ---------------------------------------------------------------------------
// Batched per-simulation work around a fine micro step (see MicroItem).
// ---------------------------------------------------------------------------
__device__ inline double prolong(const Geo& gc, const Window& w,
                                 const double* __restrict__ Tc, int fi, int fj,
                                 int fk);
__device__ inline bool fine_gamma(const Geo& gf, const Window& w, int i, int j,
                                  int k);

int micro_blocks(const Geo& gf) {
  return std::max(1, std::min(kMaxMicroBlocks, (gf.nreal + 4 * kBlock - 1) /
                                                   (4 * kBlock)));
}

__global__ void __launch_bounds__(kBlock)
micro_prep_kernel(const MicroItem* __restrict__ items, int per_item) {
  __shared__ double lds[kBlock / 64];
  const MicroItem& it = items[blockIdx.x / per_item];
  const int blk = blockIdx.x % per_item;
  if (blk >= it.nblk) return;   // the whole workgroup
  const Geo& g = it.gf;
  double acc[1] = {0.0};
  for (int t = blk * kBlock + threadIdx.x; t < g.nreal;
       t += it.nblk * kBlock) {
    int i, j, k;
    node_ijk(g, t, i, j, k);
    const int n = pidx(g, i, j, k);
    double v = it.pp != nullptr ? 2.0 * it.prev[n] - it.pp[n] : it.prev[n];
    if (it.w.bottom && k == 0) {
      v = it.T_bottom;
    } else if (fine_gamma(g, it.w, i, j, k)) {
      v = prolong(it.gc, it.w, it.Ta, i, j, k);
      if (it.wb != 0.0)
        v = (1.0 - it.wb) * v + it.wb * prolong(it.gc, it.w, it.Tb, i, j, k);
    }
    it.cur[n] = v;
    double f = 0.0;
    if (it.source == 1) {
      if (it.vs.on)
        f = it.vs.amp * hat_gauss(i, g.nx, g.hx, g.x0, it.vs.xc, it.vs.a3) *
            hat_gauss(j, g.ny, g.hy, g.y0, it.vs.yc, it.vs.a3) *
            hat_gauss(k, g.nz, g.hz, -(g.nz - 1) * g.hz, 0.0, it.vs.az);
      it.F[n] = f;
    } else if (k == g.nz - 1) {
      if (it.spot.weight != 0.0)
        f = spot_load(g, it.nq, it.gx, it.gw, it.spot, i, j, 0, 0, 0, 0);
      it.F[n] = f;
    }
    acc[0] += f;
  }
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) it.part[kPartGen * kMaxBlocks + blk] = acc[0];
}

__global__ void __launch_bounds__(kBlock)
micro_post_kernel(const MicroItem* __restrict__ items, int per_item) {
  __shared__ double lds[2 * kBlock / 64];
  const MicroItem& it = items[blockIdx.x / per_item];
  const int blk = blockIdx.x % per_item;
  if (blk >= it.nblk) return;   // the whole workgroup
  const Geo& g = it.gf;
  const bool surf = it.slot_surf != nullptr && (it.sf.h != 0.0 || it.sf.es != 0.0);
  double acc[2] = {0.0, 0.0};   // bottom reactions, surface loss
  for (int t = blk * kBlock + threadIdx.x; t < g.nreal;
       t += it.nblk * kBlock) {
    int i, j, k;
    node_ijk(g, t, i, j, k);
    const int n = pidx(g, i, j, k);
    if (fine_gamma(g, it.w, i, j, k)) {
      if (it.rho != nullptr) it.rho[n] = it.rho_init ? it.R[n] : it.rho[n] + it.R[n];
    } else if (it.w.bottom && k == 0) {
      acc[0] += it.R[n];
    }
    if (surf && k == g.nz - 1)
      acc[1] += top_area(g, it.rgw, i, j) * surface_flux(it.Tsurf[n], it.sf);
  }
  block_sum<2>(acc, lds);
  if (threadIdx.x == 0) {
    it.part[kPartGen * kMaxBlocks + blk] = acc[0];
    it.part[kPartAux * kMaxBlocks + blk] = acc[1];
  }
}

// One wave per simulation: the nblk partials of region reg times scale,
// added into the slot the item names for that sum.  Lane l adds partials
// l, l + 64, ... in order, then the wave's fixed DPP reduction: the same
// order every time, whatever else the launch holds.
__global__ void __launch_bounds__(64)
micro_finalize_kernel(const MicroItem* __restrict__ items, int post) {
  const MicroItem& it = items[blockIdx.x];
  for (int reg = 0; reg < (post ? 2 : 1); ++reg) {
    double* slot = post ? (reg == 0 ? it.slot_bottom : it.slot_surf) : it.slot_abs;
    const double scale = post ? (reg == 0 ? it.scale_bottom : it.scale_surf)
                              : it.scale_abs;
    if (slot == nullptr) continue;
    if (post && reg == 0 && !it.w.bottom) continue;
    if (post && reg == 1 && it.sf.h == 0.0 && it.sf.es == 0.0) continue;
    double sum = 0.0;
    for (int b = threadIdx.x; b < it.nblk; b += 64)
      sum += it.part[reg * kMaxBlocks + b];
    sum = wave_sum(sum);
    if (threadIdx.x == 0) *slot += scale * sum;
  }
}

void k_micro_prep(Launch L, const MicroItem* items, int n_items, int per_item) {
  if (n_items <= 0) return;
  hipLaunchKernelGGL(micro_prep_kernel, dim3(n_items * per_item),
                     dim3(kBlock), 0, (hipStream_t)L.stream, items, per_item);
  hipLaunchKernelGGL(micro_finalize_kernel, dim3(n_items), dim3(64), 0,
                     (hipStream_t)L.stream, items, 0);
}
void k_micro_post(Launch L, const MicroItem* items, int n_items, int per_item) {
  if (n_items <= 0) return;
  hipLaunchKernelGGL(micro_post_kernel, dim3(n_items * per_item),
                     dim3(kBlock), 0, (hipStream_t)L.stream, items, per_item);
  hipLaunchKernelGGL(micro_finalize_kernel, dim3(n_items), dim3(64), 0,
                     (hipStream_t)L.stream, items, 1);
}

// ---------------------------------------------------------------------------
// K7: Dirichlet data of the fine window.  Bottom nodes of a window that
// reaches the plate bottom get T_bottom; nodes on immersed faces get the
// trilinear interpolant of (1 - wb) Ta + wb Tb (coarse fields), the time
// blend of the paper's local problem (Section 4).
// ---------------------------------------------------------------------------
__device__ inline double prolong(const Geo& gc, const Window& w,
                                 const double* __restrict__ Tc, int fi, int fj,
                                 int fk) {
  // global fine index on each axis, its coarse cell and position in it
  const int gi = w.r * w.I0 + fi, gj = w.r * w.J0 + fj, gk = w.r * w.K0 + fk;
  int ci = gi / w.r, cj = gj / w.r, ck = gk / w.r;
  if (ci > gc.nx - 2) ci = gc.nx - 2;
  if (cj > gc.ny - 2) cj = gc.ny - 2;
  if (ck > gc.nz - 2) ck = gc.nz - 2;
  const double fx = (double)(gi - ci * w.r) / (double)w.r;
  const double fy = (double)(gj - cj * w.r) / (double)w.r;
  const double fz = (double)(gk - ck * w.r) / (double)w.r;
  const int n = pidx(gc, ci, cj, ck);
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int a = c & 1, b = (c >> 1) & 1, e = c >> 2;
    const double wt = ((a ? fx : 1.0 - fx) * (b ? fy : 1.0 - fy)) *
                      (e ? fz : 1.0 - fz);
    acc += wt * Tc[n + a + b * gc.px + e * gc.pxy];
  }
  return acc;
}

__device__ inline bool fine_gamma(const Geo& gf, const Window& w, int i, int j,
                                  int k) {
  if (w.bottom && k == 0) return false;
  return ((w.faces & kFx0) && i == 0) || ((w.faces & kFx1) && i == gf.nx - 1) ||
         ((w.faces & kFy0) && j == 0) || ((w.faces & kFy1) && j == gf.ny - 1) ||
         ((w.faces & kFz0) && k == 0);
}

__global__ void fine_dirichlet_kernel(Geo gf, Geo gc, Window w, double Tb_val,
                                      const double* __restrict__ Ta,
                                      const double* __restrict__ Tb, double wb,
                                      double* __restrict__ Tf) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < gf.nreal;
       t += gridDim.x * blockDim.x) {
    int i, j, k;
    node_ijk(gf, t, i, j, k);
    const int n = pidx(gf, i, j, k);
    if (w.bottom && k == 0) {
      Tf[n] = Tb_val;
    } else if (fine_gamma(gf, w, i, j, k)) {
      double v = prolong(gc, w, Ta, i, j, k);
      if (wb != 0.0) v = (1.0 - wb) * v + wb * prolong(gc, w, Tb, i, j, k);
      Tf[n] = v;
    }
  }
}

void k_fine_dirichlet(Launch L, const Geo& gf, const Geo& gc, const Window& w,
                      double T_bottom, const double* Ta, const double* Tb,
                      double wb, double* Tf) {
  hipLaunchKernelGGL(fine_dirichlet_kernel, dim3(grid_for(gf.nreal)),
                     dim3(kBlock), 0, (hipStream_t)L.stream, gf, gc, w,
                     T_bottom, Ta, Tb, wb, Tf);
}

// ---------------------------------------------------------------------------
// K9 (part 1): accumulate the fine interface reactions over micro steps and
// the heat leaving through the plate bottom inside the window.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
interface_acc_kernel(Geo gf, Window w, const double* __restrict__ R,
                     double* __restrict__ rho, int init, double* partials) {
  __shared__ double lds[kBlock / 64];
  double acc[1] = {0.0};
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < gf.nreal;
       t += gridDim.x * blockDim.x) {
    int i, j, k;
    node_ijk(gf, t, i, j, k);
    const int n = pidx(gf, i, j, k);
    if (fine_gamma(gf, w, i, j, k)) {
      if (rho != nullptr) rho[n] = init ? R[n] : rho[n] + R[n];
    } else if (w.bottom && k == 0) {
      acc[0] += R[n];
    }
  }
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) partials[kPartGen * kMaxBlocks + blockIdx.x] = acc[0];
}

void k_interface_accumulate(Launch L, const Geo& gf, const Window& w,
                            const double* R, double* rho_acc, int init,
                            double bottom_scale, double* ledger_bottom,
                            double* partials) {
  const int nb = grid_for(gf.nreal);
  hipLaunchKernelGGL(interface_acc_kernel, dim3(nb), dim3(kBlock), 0,
                     (hipStream_t)L.stream, gf, w, R, rho_acc, init, partials);
  if (ledger_bottom != nullptr && w.bottom)
    finalize_sum(L, partials + kPartGen * kMaxBlocks, nb, bottom_scale,
                 ledger_bottom, 0);
}

// ---------------------------------------------------------------------------
// K9 (part 2): restriction of the interface reactions onto the coarse
// interface nodes with the transpose of the trilinear prolongation:
//   ext_J = scale * sum_k P_kJ (rho_acc_k + Rm_k)   over fine interface nodes k
// (either array may be null).
// One workgroup per coarse node of the closed window box; nodes of the box
// that are not interface nodes get 0.
// ---------------------------------------------------------------------------
// With `all`, the restriction P^T of rho + Rm over every fine node of the
// window onto every coarse node of the closed window (the consistent
// global problem's load).
__global__ void __launch_bounds__(kBlock)
restrict_kernel(Geo gf, Geo gc, Window w, const double* __restrict__ rho,
                const double* __restrict__ Rm, double scale,
                double* __restrict__ ext, int all) {
  __shared__ double lds[kBlock / 64];
  const int bx = w.wx + 1, by = w.wy + 1;
  const int b = blockIdx.x;
  const int li = b % bx, lj = (b / bx) % by, lk = b / (bx * by);
  const int I = w.I0 + li, J = w.J0 + lj, K = w.K0 + lk;
  Region rg;
  rg.faces = w.faces;
  const bool gamma = all || on_immersed_face(rg, I, J, K, w.I0, w.I0 + w.wx,
                                             w.J0, w.J0 + w.wy, w.K0);
  const int r = w.r;
  const int span = 2 * r - 1;
  const int fi0 = r * li, fj0 = r * lj, fk0 = r * lk;
  double acc[1] = {0.0};
  if (gamma) {
    const int tot = span * span * span;
    for (int t = threadIdx.x; t < tot; t += kBlock) {
      const int di = t % span - (r - 1), dj = (t / span) % span - (r - 1),
                dk = t / (span * span) - (r - 1);
      const int fi = fi0 + di, fj = fj0 + dj, fk = fk0 + dk;
      if (fi < 0 || fj < 0 || fk < 0 || fi > gf.nx - 1 || fj > gf.ny - 1 ||
          fk > gf.nz - 1)
        continue;
      if (!all && !fine_gamma(gf, w, fi, fj, fk)) continue;
      const double wt = ((double)(r - abs(di)) / (double)r) *
                        ((double)(r - abs(dj)) / (double)r) *
                        ((double)(r - abs(dk)) / (double)r);
      const int n = pidx(gf, fi, fj, fk);
      acc[0] += wt * ((rho != nullptr ? rho[n] : 0.0) +
                      (Rm != nullptr ? Rm[n] : 0.0));
    }
  }
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) ext[pidx(gc, I, J, K)] = gamma ? scale * acc[0] : 0.0;
}

void k_restrict(Launch L, const Geo& gf, const Geo& gc, const Window& w,
                const double* rho_acc, const double* Rm, double scale,
                double* ext) {
  const int nb = (w.wx + 1) * (w.wy + 1) * (w.wz + 1);
  hipLaunchKernelGGL(restrict_kernel, dim3(nb), dim3(kBlock), 0,
                     (hipStream_t)L.stream, gf, gc, w, rho_acc, Rm, scale, ext,
                     0);
}
void k_restrict_all(Launch L, const Geo& gf, const Geo& gc, const Window& w,
                    const double* s, double* ext) {
  const int nb = (w.wx + 1) * (w.wy + 1) * (w.wz + 1);
  hipLaunchKernelGGL(restrict_kernel, dim3(nb), dim3(kBlock), 0,
                     (hipStream_t)L.stream, gf, gc, w, (const double*)nullptr,
                     s, 1.0, ext, 1);
}

// ---------------------------------------------------------------------------
// The consistent global problem's load from the local solution (paper
// Section 3: the volume terms inside the local domain and the interface
// jump, rewritten with the local equation): on every fine node of the
// window
//   s = rhoc_f m_k (Tm - T0) / Dt + k_f (K1 Tavg)_k - (rho + Rm)_k / m,
// K1 the unit-conductivity stiffness of the window's elements, Tavg =
// (Tsum + Tm) / m the mean of the m micro-step fields, and the last term --
// the mean of the local reactions -- on the interface nodes only.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
consistent_source_kernel(Geo gf, Window w, const double* __restrict__ Tm,
                         const double* __restrict__ T0,
                         const double* __restrict__ Tsum,
                         const double* __restrict__ rho,
                         const double* __restrict__ Rm, double inv_m,
                         double Dt, double kf, double rhocf,
                         double* __restrict__ src) {
  double wts[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) wts[q] = gf.w[q];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < gf.nreal;
       t += gridDim.x * blockDim.x) {
    int i, j, k;
    node_ijk(gf, t, i, j, k);
    const int n = pidx(gf, i, j, k);
    double v27[27];
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          const int q = n + dz * gf.pxy + dy * gf.px + dx;
          v27[N27(dx, dy, dz)] =
              ((Tsum != nullptr ? Tsum[q] : 0.0) + Tm[q]) * inv_m;
        }
    double k8[8];
    double nact = 0.0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
      const int ei = i - ex, ej = j - ey, ek = k - ez;
      const bool in = ei >= 0 && ej >= 0 && ek >= 0 && ei <= gf.nx - 2 &&
                      ej <= gf.ny - 2 && ek <= gf.nz - 2;
      k8[e] = in ? 1.0 : 0.0;
      nact += k8[e];
    }
    double v = rhocf * gf.vol8 * nact * (Tm[n] - T0[n]) / Dt +
               kf * stencil_apply(v27, k8, wts);
    if (fine_gamma(gf, w, i, j, k))
      v -= ((rho != nullptr ? rho[n] : 0.0) + Rm[n]) * inv_m;
    src[n] = v;
  }
}

void k_consistent_source(Launch L, const Geo& gf, const Window& w,
                         const double* Tm, const double* T0, const double* Tsum,
                         const double* rho, const double* Rm, int m, double Dt,
                         double kf, double rhocf, double* src) {
  hipLaunchKernelGGL(consistent_source_kernel, dim3(grid_for(gf.nreal)),
                     dim3(kBlock), 0, (hipStream_t)L.stream, gf, w, Tm, T0,
                     Tsum, rho, Rm, 1.0 / m, Dt, kf, rhocf, src);
}

__global__ void accumulate_kernel(double* __restrict__ dst,
                                  const double* __restrict__ src, long n,
                                  int assign) {
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n;
       t += (long)gridDim.x * blockDim.x)
    dst[t] = assign ? src[t] : dst[t] + src[t];
}
void k_accumulate(Launch L, double* dst, const double* src, long n, int assign) {
  hipLaunchKernelGGL(accumulate_kernel, dim3(grid_for(n)), dim3(kBlock), 0,
                     (hipStream_t)L.stream, dst, src, n, assign);
}

// ---------------------------------------------------------------------------
// Cost of a device-wide synchronisation (tl_op_sync_probe): `rounds` sweeps
// over n doubles (each entry mixed with one a few thousand entries away, so
// a sweep depends on other workgroups' results of the sweep before), either
// one kernel launch per sweep or all sweeps in one cooperative launch with a
// grid barrier between them.  The barrier: every workgroup arrives with a
// release increment of a counter, the last one resets it and bumps a
// generation word, the others poll it with relaxed loads and take one
// acquire fence; polling is bounded and a timeout sets *err instead of
// hanging.
// ---------------------------------------------------------------------------
constexpr unsigned kSyncSpinMax = 1u << 22;

__device__ inline void grid_barrier(unsigned* cnt, unsigned* gen, int* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned g =
        __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned a = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE,
                                              __HIP_MEMORY_SCOPE_AGENT);
    if (a == gridDim.x - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE,
                             __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(gen, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSyncSpinMax) {
          *err = 1;
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  __syncthreads();
}

template <int kBarrier>
__global__ void __launch_bounds__(kBlock)
sync_probe_kernel(double* __restrict__ data, long n, int rounds,
                  unsigned* cnt, unsigned* gen, int* err) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (int r = 0; r < rounds; ++r) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n;
         i += stride) {
      const long j = i + 4099 < n ? i + 4099 : i + 4099 - n;
      data[i] = 0.5 * data[i] + 0.25 * data[j] + 1.0;
    }
    if (kBarrier) grid_barrier(cnt, gen, err);
  }
}

int sync_probe_resident() {
  static const int res = resident_blocks(sync_probe_kernel<1>);
  return res;
}

int k_sync_probe(Launch L, int blocks, int rounds, int barrier, double* data,
                 long n, unsigned* ctl) {
  if (!barrier) {
    for (int r = 0; r < rounds; ++r)
      hipLaunchKernelGGL(sync_probe_kernel<0>, dim3(blocks), dim3(kBlock), 0,
                         (hipStream_t)L.stream, data, n, 1, ctl, ctl + 64,
                         (int*)(ctl + 128));
    return hipGetLastError();
  }
  unsigned* gen = ctl + 64;
  int* err = (int*)(ctl + 128);
  void* args[] = {&data, &n, &rounds, &ctl, &gen, &err};
  return hipLaunchCooperativeKernel((void*)sync_probe_kernel<1>, dim3(blocks),
                                   dim3(kBlock), args, 0,
                                   (hipStream_t)L.stream);
}

// ---------------------------------------------------------------------------
// K9 (part 3): injection of the fine solution into the coarse nodes of the
// window that are not on an immersed face.
// ---------------------------------------------------------------------------
__global__ void inject_kernel(Geo gf, Geo gc, Window w,
                              const double* __restrict__ Tf,
                              double* __restrict__ Tc) {
  const int bx = w.wx + 1, by = w.wy + 1, bz = w.wz + 1;
  Region rg;
  rg.faces = w.faces;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < bx * by * bz;
       t += gridDim.x * blockDim.x) {
    const int li = t % bx, lj = (t / bx) % by, lk = t / (bx * by);
    const int I = w.I0 + li, J = w.J0 + lj, K = w.K0 + lk;
    if (on_immersed_face(rg, I, J, K, w.I0, w.I0 + w.wx, w.J0, w.J0 + w.wy,
                         w.K0))
      continue;
    if (K == 0) continue;  // plate bottom keeps its fixed value
    Tc[pidx(gc, I, J, K)] = Tf[pidx(gf, w.r * li, w.r * lj, w.r * lk)];
  }
}

void k_inject(Launch L, const Geo& gf, const Geo& gc, const Window& w,
              const double* Tf, double* Tc) {
  const long n = (long)(w.wx + 1) * (w.wy + 1) * (w.wz + 1);
  hipLaunchKernelGGL(inject_kernel, dim3(grid_for(n)), dim3(kBlock), 0,
                     (hipStream_t)L.stream, gf, gc, w, Tf, Tc);
}

// ---------------------------------------------------------------------------
// K8: window move.  Fine nodes inside the old window copy the old fine value;
// newly covered ones take the trilinear interpolant of the coarse field.
// ---------------------------------------------------------------------------
__global__ void window_shift_kernel(Geo gf, Geo gc, Window wn, Window wo,
                                    const double* __restrict__ Tf_old,
                                    const double* __restrict__ Tc,
                                    double* __restrict__ Tf_new) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < gf.nreal;
       t += gridDim.x * blockDim.x) {
    int i, j, k;
    node_ijk(gf, t, i, j, k);
    const int oi = i + wn.r * (wn.I0 - wo.I0), oj = j + wn.r * (wn.J0 - wo.J0);
    double v;
    if (oi >= 0 && oi <= gf.nx - 1 && oj >= 0 && oj <= gf.ny - 1)
      v = Tf_old[pidx(gf, oi, oj, k)];
    else
      v = prolong(gc, wn, Tc, i, j, k);
    Tf_new[pidx(gf, i, j, k)] = v;
  }
}

void k_window_shift(Launch L, const Geo& gf, const Geo& gc, const Window& wn,
                    const Window& wo, const double* Tf_old, const double* Tc,
                    double* Tf_new) {
  hipLaunchKernelGGL(window_shift_kernel, dim3(grid_for(gf.nreal)),
                     dim3(kBlock), 0, (hipStream_t)L.stream, gf, gc, wn, wo,
                     Tf_old, Tc, Tf_new);
}

// ---------------------------------------------------------------------------
// K10: energy sum_i m_i(region) H(T_i) and bottom reaction sums.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock)
energy_kernel(Geo g, Region rg, MatDev m, const double* __restrict__ T,
              double lin, double* partials) {
  __shared__ double lds[kBlock / 64];
  double acc[1] = {0.0};
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < g.nreal;
       t += gridDim.x * blockDim.x) {
    int i, j, k;
    node_ijk(g, t, i, j, k);
    double nact = 0.0, nfict = 0.0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int ex = e & 1, ey = (e >> 1) & 1, ez = e >> 2;
      if (elem_active(g, rg, i - ex, j - ey, k - ez)) {
        if (elem_fictitious(rg, i - ex, j - ey, k - ez))
          nfict += 1.0;
        else
          nact += 1.0;
      }
    }
    const double Tn = T[pidx(g, i, j, k)];
    if (nact > 0.0) acc[0] += g.vol8 * nact * (enthalpy(Tn, m) + lin * Tn);
    if (nfict > 0.0) acc[0] += g.vol8 * nfict * rg.rhocf * Tn;
  }
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) partials[kPartGen * kMaxBlocks + blockIdx.x] = acc[0];
}

void k_energy(Launch L, const Geo& g, const Region& rg, const MatDev& m,
              const double* T, double* slot, int assign, double* partials,
              double lin) {
  const int nb = grid_for(g.nreal);
  hipLaunchKernelGGL(energy_kernel, dim3(nb), dim3(kBlock), 0,
                     (hipStream_t)L.stream, g, rg, m, T, lin, partials);
  finalize_sum(L, partials + kPartGen * kMaxBlocks, nb, 1.0, slot, assign);
}

__global__ void __launch_bounds__(kBlock)
bottom_sum_kernel(Geo g, const double* __restrict__ R, double* partials) {
  __shared__ double lds[kBlock / 64];
  double acc[1] = {0.0};
  const int nb = g.nx * g.ny;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nb;
       t += gridDim.x * blockDim.x)
    acc[0] += R[pidx(g, t % g.nx, t / g.nx, 0)];
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) partials[kPartGen * kMaxBlocks + blockIdx.x] = acc[0];
}

void k_bottom_sum(Launch L, const Geo& g, const double* R, double scale,
                  double* slot, double* partials) {
  const int nb = grid_for((long)g.nx * g.ny);
  hipLaunchKernelGGL(bottom_sum_kernel, dim3(nb), dim3(kBlock), 0,
                     (hipStream_t)L.stream, g, R, partials);
  finalize_sum(L, partials + kPartGen * kMaxBlocks, nb, scale, slot, 0);
}

__global__ void __launch_bounds__(kBlock)
surface_sum_kernel(Geo g, Region rg, SurfDev sf, const double* __restrict__ T,
                   double* partials) {
  __shared__ double lds[kBlock / 64];
  double acc[1] = {0.0};
  const int ntop = g.nx * g.ny;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < ntop;
       t += gridDim.x * blockDim.x) {
    const int i = t % g.nx, j = t / g.nx;
    const double A = top_area(g, rg, i, j);
    if (A > 0.0) acc[0] += A * surface_flux(T[pidx(g, i, j, g.nz - 1)], sf);
  }
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) partials[kPartGen * kMaxBlocks + blockIdx.x] = acc[0];
}

void k_surface_sum(Launch L, const Geo& g, const Region& rg, const SurfDev& sf,
                   const double* T, double scale, double* slot,
                   double* partials) {
  if (sf.h == 0.0 && sf.es == 0.0) return;
  const int nb = grid_for((long)g.nx * g.ny);
  hipLaunchKernelGGL(surface_sum_kernel, dim3(nb), dim3(kBlock), 0,
                     (hipStream_t)L.stream, g, rg, sf, T, partials);
  finalize_sum(L, partials + kPartGen * kMaxBlocks, nb, scale, slot, 0);
}

// ---------------------------------------------------------------------------
// Interface values of the two-level iteration (coarse nodes on the immersed
// window faces), gathered for the host-side relaxation and scattered back.
// ---------------------------------------------------------------------------
__global__ void gamma_gather_kernel(const int* __restrict__ idx, int n,
                                    const double* __restrict__ T,
                                    const double* __restrict__ lam,
                                    double* __restrict__ out) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += gridDim.x * blockDim.x) {
    out[2 * q] = T[idx[q]];
    out[2 * q + 1] = lam[idx[q]];
  }
}
__global__ void gamma_scatter_kernel(const int* __restrict__ idx, int n,
                                     const double* __restrict__ in,
                                     double* __restrict__ lam) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += gridDim.x * blockDim.x)
    lam[idx[q]] = in[q];
}
void k_gamma_gather(Launch L, const int* idx, int n, const double* T,
                    const double* lam, double* out) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gamma_gather_kernel, dim3(grid_for(n)), dim3(kBlock), 0,
                     (hipStream_t)L.stream, idx, n, T, lam, out);
}
void k_gamma_scatter(Launch L, const int* idx, int n, const double* in,
                     double* lam) {
  if (n <= 0) return;
  hipLaunchKernelGGL(gamma_scatter_kernel, dim3(grid_for(n)), dim3(kBlock), 0,
                     (hipStream_t)L.stream, idx, n, in, lam);
}

// ---------------------------------------------------------------------------
// layout conversion
// ---------------------------------------------------------------------------
template <class T>
__global__ void pack_kernel(Geo g, int kind, const T* __restrict__ plain,
                            T* __restrict__ padded, int to_padded) {
  // kind 0: nodes (nx x ny x nz); kind 1: elements ((nx-1) x (ny-1) x (nz-1))
  const int ex = kind ? g.nx - 1 : g.nx, ey = kind ? g.ny - 1 : g.ny,
            ez = kind ? g.nz - 1 : g.nz;
  const long tot = (long)ex * ey * ez;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < tot;
       t += (long)gridDim.x * blockDim.x) {
    const int i = (int)(t % ex), j = (int)((t / ex) % ey), k = (int)(t / ((long)ex * ey));
    const int n = pidx(g, i, j, k);
    if (to_padded)
      padded[n] = plain[t];
    else
      padded[t] = plain[n];  // here `plain` is the padded source
  }
}

void k_pack(Launch L, const Geo& g, int kind, int elem_bytes, const void* plain,
            void* padded) {
  k_zero_bytes(L, padded, (size_t)g.npad * elem_bytes);
  const long tot = (long)g.nreal;
  if (elem_bytes == 8)
    hipLaunchKernelGGL(pack_kernel<double>, dim3(grid_for(tot)), dim3(kBlock),
                       0, (hipStream_t)L.stream, g, kind, (const double*)plain,
                       (double*)padded, 1);
  else
    hipLaunchKernelGGL(pack_kernel<float>, dim3(grid_for(tot)), dim3(kBlock), 0,
                       (hipStream_t)L.stream, g, kind, (const float*)plain,
                       (float*)padded, 1);
}

void k_unpack(Launch L, const Geo& g, int kind, int elem_bytes,
              const void* padded, void* plain) {
  const long tot = (long)g.nreal;
  if (elem_bytes == 8)
    hipLaunchKernelGGL(pack_kernel<double>, dim3(grid_for(tot)), dim3(kBlock),
                       0, (hipStream_t)L.stream, g, kind, (const double*)padded,
                       (double*)plain, 0);
  else
    hipLaunchKernelGGL(pack_kernel<float>, dim3(grid_for(tot)), dim3(kBlock), 0,
                       (hipStream_t)L.stream, g, kind, (const float*)padded,
                       (float*)plain, 0);
}

}  // namespace tl
