// Solver runtime and C interface of the two-level thermal library.
//
// Host-side control of the spatiotemporal two-level method (paper Sections 3
// and 4, Algorithm 1): window placement and moves, the coarse predictor, the
// fine micro steps with time-blended Dirichlet data, the Dirichlet-Neumann
// two-level correction with relaxation, injection, and the FP64 energy
// ledger.  Each implicit step is a frozen-kappa Newton iteration with a
// backtracking line search whose linear systems are solved by
// Jacobi-preconditioned CG in FP64, or in FP32 for the fine level of the
// mixed-precision path.  All arithmetic on fields runs in the HIP kernels of
// tl_kernels.hip; the host reads back a few scalars per Newton iteration, per
// CG chunk and per two-level iteration to steer the loops.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tl.h"
#include "../../include/tl_ops.h"
#include "tl_internal.h"

using namespace tl;

namespace {

thread_local std::string g_last_error;

tl_status fail(tl_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HIP_OK(expr)                                                        \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      return fail(TL_EDEVICE, std::string(#expr) + ": " +                   \
                                  hipGetErrorString(e_));                   \
  } while (0)

struct NoConv {
  std::string msg;
};
struct DevErr {
  std::string msg;
};

inline void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw DevErr{std::string(what) + ": " + hipGetErrorString(e)};
}

constexpr int kLineSearchMax = 12;  // halvings tried before a step is taken anyway
constexpr int kProfPairs = 64;      // event pairs held between host syncs
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Sizes of everything carved out of the caller's workspace.
struct Layout {
  Geo gc, gf;
  size_t off_c[22], off_fd[8], off_fcg[12];
  size_t off_scal, off_ledger, off_partials, off_gidx, off_gbuf;
  int gamma_cap;
  size_t total;
  int cg_bytes;
};

constexpr int kCoarseArrays = 22;  // Tn Tpred cur trial lam dprev R Fall Fout ext | 12 CG arrays
constexpr int kFineD = 8;          // state prev cur trial alt R F rho
constexpr int kFineCG = 12;        // kap d dinv r0 r1 w0 w1 s0 s1 p x0 x1

Layout make_layout(const tl_mesh& me, const tl_options& op) {
  Layout L;
  const double hx = me.lx / me.nx, hy = me.ly / me.ny, hz = me.lz / me.nz;
  L.gc = make_geo(me.nx, me.ny, me.nz, hx, hy, hz, 0.0, 0.0);
  const int r = me.refine;
  L.gf = make_geo(r * me.win_nx, r * me.win_ny, r * me.win_nz, hx / r, hy / r,
                  hz / r, 0.0, 0.0);
  L.cg_bytes = op.precision == TL_MIXED ? 4 : 8;
  size_t off = 0;
  const size_t cbytes = align_up((size_t)L.gc.npad * 8);
  const size_t fbytes = align_up((size_t)L.gf.npad * 8);
  const size_t fcg = align_up((size_t)L.gf.npad * L.cg_bytes);
  for (int a = 0; a < kCoarseArrays; ++a) { L.off_c[a] = off; off += cbytes; }
  for (int a = 0; a < kFineD; ++a) { L.off_fd[a] = off; off += fbytes; }
  for (int a = 0; a < kFineCG; ++a) { L.off_fcg[a] = off; off += fcg; }
  L.off_scal = off; off += align_up(2 * sizeof(LevelScalars));
  L.off_ledger = off; off += align_up(sizeof(LedgerDev));
  L.off_partials = off;
  off += align_up((size_t)kMaxBlocks * kPartRegions * sizeof(double));
  L.gamma_cap = (me.win_nx + 1) * (me.win_ny + 1) * (me.win_nz + 1);
  L.off_gidx = off; off += align_up((size_t)L.gamma_cap * sizeof(int));
  L.off_gbuf = off; off += align_up((size_t)L.gamma_cap * 2 * sizeof(double));
  L.total = off;
  return L;
}

// Buffers of one level's Newton/CG solve.
template <class R>
struct CGBufs {
  R *kap, *d, *dinv, *r[2], *w[2], *s[2], *p, *x[2];
};

}  // namespace

struct tl_sim {
  tl_mesh mesh;
  tl_material mat_in;
  tl_options opts;
  MatDev mat;
  std::vector<TrackH> tracks;
  double t_start;
  Layout lay;
  Geo gc, gf;
  Window win;
  hipStream_t stream;
  Launch L;
  char* ws;
  // coarse fields
  double *Tn, *Tpred, *ccur, *ctrial, *lam, *dprev, *cR, *Fall, *Fout, *ext;
  CGBufs<double> ccg;
  // fine fields
  double *fstate, *fprev, *fcur, *ftrial, *falt, *fR, *fF, *rho;
  CGBufs<double> fcg64;
  CGBufs<float> fcg32;
  LevelScalars *sc_c, *sc_f;
  LedgerDev* led;
  double* partials;
  int* gidx;            // padded indices of the coarse interface nodes
  double* gbuf;         // interface gather/scatter staging
  int n_gamma;
  // host side
  LevelScalars* h_sc;   // pinned
  LedgerDev* h_led;     // pinned
  double* h_gbuf;       // pinned, 2 * gamma_cap doubles
  tl_ledger ledger;     // committed ledger
  tl_stats stats;
  long n_macro;
  double theta0;
  int last_cg_f, last_cg_c;
  // sampled event timing of the fine CG operator kernel (tl_set_profiling)
  int prof_every;
  long prof_count;
  int prof_used;
  hipEvent_t prof_ev[2 * 64];
  int prof_k[64];
};

namespace {

Region region_window(const tl_sim* s) {
  Region rg{};
  rg.mode = kWindow;
  rg.faces = s->win.faces;
  rg.bottom = s->win.bottom;
  return rg;
}
Region region_outside(const tl_sim* s) {
  Region rg{};
  rg.mode = kOutside;
  rg.I0 = s->win.I0;
  rg.I1 = s->win.I0 + s->win.wx;
  rg.J0 = s->win.J0;
  rg.J1 = s->win.J0 + s->win.wy;
  rg.K0 = s->win.K0;
  rg.faces = s->win.faces;
  return rg;
}
Region region_all() {
  Region rg{};
  rg.mode = kAllBottom;
  return rg;
}

// Padded indices of the coarse interface nodes (on an immersed window face),
// in box-scan order, uploaded to the device.
void set_interface(tl_sim* s);

Window make_window(const tl_mesh& me, int I0, int J0) {
  Window w;
  w.I0 = I0;
  w.J0 = J0;
  w.K0 = me.nz - me.win_nz;
  w.wx = me.win_nx;
  w.wy = me.win_ny;
  w.wz = me.win_nz;
  w.r = me.refine;
  w.faces = 0;
  if (I0 > 0) w.faces |= kFx0;
  if (I0 + w.wx < me.nx) w.faces |= kFx1;
  if (J0 > 0) w.faces |= kFy0;
  if (J0 + w.wy < me.ny) w.faces |= kFy1;
  if (w.K0 > 0) w.faces |= kFz0;
  w.bottom = w.K0 == 0 ? 1 : 0;
  return w;
}

// Free fine nodes of the window (not on an immersed face, not on the bottom).
double fine_free_nodes(const Geo& gf, const Window& w) {
  long cnt = 0;
  for (int k = 0; k < gf.nz; ++k)
    for (int j = 0; j < gf.ny; ++j)
      for (int i = 0; i < gf.nx; ++i) {
        bool dir = (w.bottom && k == 0) || ((w.faces & kFx0) && i == 0) ||
                   ((w.faces & kFx1) && i == gf.nx - 1) ||
                   ((w.faces & kFy0) && j == 0) ||
                   ((w.faces & kFy1) && j == gf.ny - 1) ||
                   ((w.faces & kFz0) && k == 0);
        if (!dir) ++cnt;
      }
  return (double)cnt;
}

void set_interface(tl_sim* s) {
  const Window& w = s->win;
  std::vector<int> idx;
  for (int k = w.K0; k <= w.K0 + w.wz; ++k)
    for (int j = w.J0; j <= w.J0 + w.wy; ++j)
      for (int i = w.I0; i <= w.I0 + w.wx; ++i) {
        const bool g = ((w.faces & kFx0) && i == w.I0) ||
                       ((w.faces & kFx1) && i == w.I0 + w.wx) ||
                       ((w.faces & kFy0) && j == w.J0) ||
                       ((w.faces & kFy1) && j == w.J0 + w.wy) ||
                       ((w.faces & kFz0) && k == w.K0);
        if (g) idx.push_back((k + 1) * s->gc.pxy + (j + 1) * s->gc.px + (i + 1));
      }
  s->n_gamma = (int)idx.size();
  if (!idx.empty())
    hip_check(hipMemcpy(s->gidx, idx.data(), idx.size() * sizeof(int),
                        hipMemcpyHostToDevice),
              "hipMemcpy(interface indices)");
}

void sync_read_scalars(tl_sim* s, const LevelScalars* dev) {
  hip_check(hipGetLastError(), "kernel launch");
  hip_check(hipMemcpyAsync(s->h_sc, dev, sizeof(LevelScalars),
                           hipMemcpyDeviceToHost, s->stream),
            "hipMemcpyAsync(scalars)");
  hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
}

// Collect the sampled event timings of fine operator launches after a host
// sync of the CG loop.  Launches of iteration k did work unless the solve has
// finished with k >= iters (those return at once); only working launches are
// counted.
void flush_profile(tl_sim* s, const LevelScalars& sc) {
  for (int q = 0; q < s->prof_used; ++q) {
    if (sc.done && s->prof_k[q] >= sc.iters) continue;
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, s->prof_ev[2 * q], s->prof_ev[2 * q + 1]),
              "hipEventElapsedTime");
    s->stats.fine_op_timed_ms += ms;
    s->stats.fine_op_timed += 1;
  }
  s->prof_used = 0;
}

// One backward-Euler step of one level: frozen-kappa Newton with backtracking
// on |R_free|_2; linear systems by Jacobi-PCG in precision R.  T holds the
// initial guess with the Dirichlet values in place; on return T (possibly
// swapped with Tt) holds the solution and Rout the residual there.
//
// Each round queues, without host synchronisation: the residual at the trial
// T - alpha x (alpha = 0 on the first round), the device-side line-search
// decision with the CG start, and n_launch CG iterations for the next
// direction (they return at once when the trial is rejected, Newton has
// converged, or CG has converged).  The host then reads the outcome once.
template <class R>
void solve_level(tl_sim* s, bool fine, const Geo& g, const Region& rg,
                 double tau, const double* Told, const double* F,
                 const double* Fext, double*& T, double*& Tt, double* Rout,
                 CGBufs<R>& cg, LevelScalars* sc, int& last_cg) {
  const tl_options& op = s->opts;
  const double tol = op.newton_tol;
  double rtol = op.cg_rtol;
  if (sizeof(R) == 4) rtol = std::max(rtol, 1e-5);
  const double rtol2 = rtol * rtol;
  int64_t& n_newton = fine ? s->stats.newton_fine : s->stats.newton_coarse;
  int64_t& n_cg = fine ? s->stats.cg_fine : s->stats.cg_coarse;
  const double op_bytes_per_node = 13.0 * sizeof(R);
  int xi = 0;  // cg.x[xi]: direction being line-searched; CG writes cg.x[1-xi]
  int n_launch = std::min(op.cg_max, std::max(3, last_cg + 2));
  double rn0 = 0.0;

  auto round = [&](bool first, double alpha, int h) {
    k_residual<R, R>(s->L, g, rg, s->mat, tau, T,
                     first ? (const R*)nullptr : cg.x[xi], alpha, Told, F,
                     Fext, Tt, Rout, cg.kap, cg.d, cg.dinv, cg.r[0],
                     s->partials);
    k_cg_start<R>(s->L, g, first ? 1 : 0, alpha, rn0, tol,
                  h == kLineSearchMax - 1 ? 1 : 0, cg.r[0], cg.dinv, cg.d,
                  cg.kap, cg.w[0], sc, s->partials);
    for (int k = 0; k < n_launch; ++k) {
      const bool timed = fine && s->prof_every > 0 &&
                         (s->prof_count++ % s->prof_every) == 0 &&
                         s->prof_used < kProfPairs;
      k_cg_iter<R>(s->L, g, k, cg.r, cg.w, cg.s, cg.p, cg.x[1 - xi], cg.d,
                   cg.kap, cg.dinv, rtol2, sc, s->partials,
                   timed ? (void*)s->prof_ev[2 * s->prof_used] : nullptr,
                   timed ? (void*)s->prof_ev[2 * s->prof_used + 1] : nullptr);
      if (timed) {
        s->prof_k[s->prof_used] = k;
        ++s->prof_used;
      }
    }
  };

  round(true, 0.0, 0);
  int dirs = 0;  // Newton directions computed
  int h = 0;
  for (;;) {
    sync_read_scalars(s, sc);
    const LevelScalars& o = *s->h_sc;
    if (fine && s->prof_used > 0) flush_profile(s, o);
    if (!std::isfinite(o.rnorm2) || !std::isfinite(o.dmax))
      throw NoConv{"non-finite residual or Newton update"};
    if (!o.accepted) {
      ++s->stats.line_search_halvings;
      ++h;
      round(false, std::ldexp(1.0, -h), h);
      continue;
    }
    std::swap(T, Tt);
    rn0 = std::sqrt(o.rnorm2);
    if (o.converged || o.rz0 == 0.0) return;
    // the CG of this round produced the next direction
    if (o.breakdown && o.iters == 0)
      throw NoConv{"CG breakdown (non-positive or non-finite curvature)"};
    if (dirs >= op.newton_max)
      throw NoConv{std::string(fine ? "fine" : "coarse") +
                   " Newton did not converge within newton_max iterations"};
    ++dirs;
    ++n_newton;
    n_cg += o.iters;
    if (fine) {
      s->stats.fine_op_bytes += op_bytes_per_node * g.nreal * o.iters;
      s->stats.fine_op_applies += o.iters;
    }
    const bool cut = !o.done;  // CG stopped by the launch count, not rtol
    last_cg = cut ? n_launch + 2 : o.iters;
    n_launch = std::min(op.cg_max, std::max(3, last_cg + 2));
    xi = 1 - xi;
    h = 0;
    round(false, 1.0, 0);
  }
}

void solve_fine(tl_sim* s, double tau, const double* Told, const double* F) {
  const Region rg = region_window(s);
  if (s->opts.precision == TL_MIXED)
    solve_level<float>(s, true, s->gf, rg, tau, Told, F, nullptr, s->fcur,
                       s->ftrial, s->fR, s->fcg32, s->sc_f, s->last_cg_f);
  else
    solve_level<double>(s, true, s->gf, rg, tau, Told, F, nullptr, s->fcur,
                        s->ftrial, s->fR, s->fcg64, s->sc_f, s->last_cg_f);
  ++s->stats.fine_solves;
}

void solve_coarse(tl_sim* s, const Region& rg, double tau, const double* F,
                  const double* Fext) {
  solve_level<double>(s, false, s->gc, rg, tau, s->Tn, F, Fext, s->ccur,
                      s->ctrial, s->cR, s->ccg, s->sc_c, s->last_cg_c);
  ++s->stats.coarse_solves;
}

SpotSet make_spots(const tl_sim* s, long n, int j0, int j1, double weight) {
  SpotSet sp;
  std::memset(&sp, 0, sizeof(sp));
  sp.nq = s->opts.face_quad;
  gauss01(sp.nq, sp.gx, sp.gw);
  int cnt = 0;
  for (int j = j0; j <= j1; ++j) {
    double t = micro_time(s->t_start, s->opts.dt_coarse, s->opts.m_time, n, j);
    double xc, yc, P, Rr, eta;
    int k;
    if (!laser_at(s->tracks.data(), (int)s->tracks.size(), s->t_start, t, &xc,
                  &yc, &P, &Rr, &eta, &k))
      continue;
    Spot& S = sp.s[cnt++];
    S.xc = xc;
    S.yc = yc;
    S.q0 = 3.0 * eta * P / (M_PI * Rr * Rr);
    S.a3 = 3.0 / (Rr * Rr);
    S.weight = weight;
  }
  sp.n = cnt;
  return sp;
}

void energy_now(tl_sim* s, double* slot) {
  k_energy(s->L, s->gc, region_outside(s), s->mat, s->Tn, slot, 1,
           s->partials);
  k_energy(s->L, s->gf, region_window(s), s->mat, s->fstate, slot, 0,
           s->partials);
}

void read_ledger(tl_sim* s) {
  hip_check(hipGetLastError(), "kernel launch");
  hip_check(hipMemcpyAsync(s->h_led, s->led, sizeof(LedgerDev),
                           hipMemcpyDeviceToHost, s->stream),
            "hipMemcpyAsync(ledger)");
  hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
}

void write_ledger(tl_sim* s) {
  s->h_led->stored = s->ledger.stored;
  s->h_led->stored0 = s->ledger.stored0;
  s->h_led->absorbed = s->ledger.absorbed;
  s->h_led->bottom = s->ledger.bottom;
  s->h_led->remap = s->ledger.remap;
  hip_check(hipMemcpyAsync(s->led, s->h_led, sizeof(LedgerDev),
                           hipMemcpyHostToDevice, s->stream),
            "hipMemcpyAsync(ledger)");
  hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
}

// Relaxation of the two-level (Dirichlet-Neumann) interface iteration
// lambda -> G(lambda), G = fine solve with Dirichlet data P lambda followed
// by the coarse outside solve, read back on the interface nodes.  With a
// fixed theta: lambda <- lambda + theta (G(lambda) - lambda).  Otherwise the
// interface quasi-Newton method with inverse least squares (IQN-ILS): the
// first step is relaxed with theta0; afterwards, with residual r = G(l) - l
// and the differences of successive residuals (columns of V) and of
// successive G values (columns of W),
//   c = argmin |V c + r_k|_2,   lambda_{k+1} = G(lambda_k) + W c.
// The fixed point -- and so the result -- is the same for every relaxation;
// only the number of iterations differs.
struct Interface {
  std::vector<std::vector<double>> V, W;
  std::vector<double> r_prev, g_prev;
  bool has_prev = false;
  static constexpr int kMaxCols = 24;

  void update(const std::vector<double>& lam, const std::vector<double>& g,
              double theta0, bool fixed, std::vector<double>& next) {
    const size_t n = lam.size();
    std::vector<double> r(n);
    for (size_t q = 0; q < n; ++q) r[q] = g[q] - lam[q];
    next.assign(n, 0.0);
    if (fixed || !has_prev) {
      for (size_t q = 0; q < n; ++q) next[q] = lam[q] + theta0 * r[q];
    } else {
      std::vector<double> dv(n), dw(n);
      for (size_t q = 0; q < n; ++q) {
        dv[q] = r[q] - r_prev[q];
        dw[q] = g[q] - g_prev[q];
      }
      V.push_back(dv);
      W.push_back(dw);
      if ((int)V.size() > kMaxCols) {
        V.erase(V.begin());
        W.erase(W.begin());
      }
      // least squares by modified Gram-Schmidt, newest column first; columns
      // that are (numerically) dependent on newer ones are skipped
      const int m = (int)V.size();
      std::vector<std::vector<double>> Q;
      std::vector<int> cols;
      std::vector<std::vector<double>> Rm;  // upper triangle, row per kept col
      for (int c = m - 1; c >= 0; --c) {
        std::vector<double> v = V[c];
        double n0 = 0.0;
        for (double x : v) n0 += x * x;
        n0 = std::sqrt(n0);
        std::vector<double> rc(Q.size() + 1, 0.0);
        for (size_t a = 0; a < Q.size(); ++a) {
          double d = 0.0;
          for (size_t q = 0; q < n; ++q) d += Q[a][q] * v[q];
          rc[a] = d;
          for (size_t q = 0; q < n; ++q) v[q] -= d * Q[a][q];
        }
        double nv = 0.0;
        for (double x : v) nv += x * x;
        nv = std::sqrt(nv);
        if (!(nv > 1e-10 * n0) || n0 == 0.0) continue;
        for (double& x : v) x /= nv;
        rc[Q.size()] = nv;
        Q.push_back(v);
        Rm.push_back(rc);
        cols.push_back(c);
      }
      const int k = (int)Q.size();
      // solve R c = -Q^T r (R upper triangular in the kept-column order)
      std::vector<double> rhs(k), cvec(k, 0.0);
      for (int a = 0; a < k; ++a) {
        double d = 0.0;
        for (size_t q = 0; q < n; ++q) d += Q[a][q] * r[q];
        rhs[a] = -d;
      }
      for (int a = k - 1; a >= 0; --a) {
        double v = rhs[a];
        for (int b = a + 1; b < k; ++b) v -= Rm[b][a] * cvec[b];
        cvec[a] = v / Rm[a][a];
      }
      for (size_t q = 0; q < n; ++q) next[q] = g[q];
      for (int a = 0; a < k; ++a) {
        const std::vector<double>& wc = W[cols[a]];
        for (size_t q = 0; q < n; ++q) next[q] += cvec[a] * wc[q];
      }
    }
    r_prev = r;
    g_prev = g;
    has_prev = true;
  }
};

// One macro step of Algorithm 1.
void macro_step(tl_sim* s) {
  const tl_options& op = s->opts;
  const int m = op.m_time;
  const double Dt = op.dt_coarse, dt = Dt / m;
  const long n = s->n_macro;
  const Launch L = s->L;
  LedgerDev* led = s->led;

  // 1. window placement for the beam at t_{n+1}
  int I0, J0;
  window_origin(s->tracks.data(), (int)s->tracks.size(), s->t_start,
                micro_time(s->t_start, Dt, m, n + 1, 0), s->gc.hx, s->gc.hy,
                s->mesh.nx, s->mesh.ny, s->mesh.win_nx, s->mesh.win_ny, 1,
                s->win.I0, s->win.J0, &I0, &J0);
  if (I0 != s->win.I0 || J0 != s->win.J0) {
    energy_now(s, &led->e_tmp0);
    const Window wo = s->win;
    const Window wn = make_window(s->mesh, I0, J0);
    k_window_shift(L, s->gf, s->gc, wn, wo, s->fstate, s->Tn, s->falt);
    std::swap(s->fstate, s->falt);
    s->win = wn;
    s->gf.x0 = wn.I0 * s->gc.hx;
    s->gf.y0 = wn.J0 * s->gc.hy;
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    set_interface(s);
    k_fill(L, s->ext, 0.0, s->gc.npad);
    energy_now(s, &led->e_tmp1);
    read_ledger(s);
    s->h_led->remap += s->h_led->e_tmp1 - s->h_led->e_tmp0;
    hip_check(hipMemcpyAsync(&led->remap, &s->h_led->remap, sizeof(double),
                             hipMemcpyHostToDevice, s->stream),
              "hipMemcpyAsync(remap)");
    ++s->stats.window_moves;
  }
  const Window& w = s->win;

  // 2. coarse loads averaged over the m micro times; predictor
  SpotSet avg = make_spots(s, n, 1, m, 1.0 / m);
  k_laser_load(L, s->gc, avg, 0, 0, 0, 0, s->Fall, 0.0, nullptr, s->partials);
  k_laser_load(L, s->gc, avg, w.I0, w.I0 + w.wx, w.J0, w.J0 + w.wy, s->Fout,
               Dt, &led->absorbed, s->partials);
  k_copy(L, s->ccur, s->Tn, s->gc.npad);
  solve_coarse(s, region_all(), Dt, s->Fall, nullptr);
  std::swap(s->Tpred, s->ccur);

  // 3. micro steps j = 1..m-1 with blended Dirichlet data
  k_copy(L, s->fprev, s->fstate, s->gf.npad);
  for (int j = 1; j < m; ++j) {
    k_copy(L, s->fcur, s->fprev, s->gf.npad);
    k_fine_dirichlet(L, s->gf, s->gc, w, s->mat_in.T_bottom, s->Tn, s->Tpred,
                     (double)j / m, s->fcur);
    SpotSet sp = make_spots(s, n, j, j, 1.0);
    k_laser_load(L, s->gf, sp, 0, 0, 0, 0, s->fF, dt, &led->absorbed,
                 s->partials);
    solve_fine(s, dt, s->fprev, s->fF);
    k_interface_accumulate(L, s->gf, w, s->fR, s->rho, j == 1 ? 1 : 0, -dt,
                           &led->bottom, s->partials);
    std::swap(s->fprev, s->fcur);
    ++s->stats.micro_steps;
  }

  // 4. two-level correction at t_{n+1}
  {
    SpotSet sp = make_spots(s, n, m, m, 1.0);
    k_laser_load(L, s->gf, sp, 0, 0, 0, 0, s->fF, dt, &led->absorbed,
                 s->partials);
  }
  k_copy(L, s->lam, s->Tpred, s->gc.npad);
  k_copy(L, s->fcur, s->fprev, s->gf.npad);
  k_copy(L, s->ccur, s->Tpred, s->gc.npad);
  const Region rout = region_outside(s);
  Interface iqn;
  std::vector<double> lam_v, lt_v, next;
  int it = 1;
  for (;; ++it) {
    if (it > op.dn_max) throw NoConv{"two-level iteration did not converge"};
    k_fine_dirichlet(L, s->gf, s->gc, w, s->mat_in.T_bottom, s->lam, nullptr,
                     0.0, s->fcur);
    solve_fine(s, dt, s->fprev, s->fF);
    k_restrict(L, s->gf, s->gc, w, m > 1 ? s->rho : nullptr, s->fR, -1.0 / m,
               s->ext);
    k_inject(L, s->gf, s->gc, w, s->fcur, s->ccur);
    solve_coarse(s, rout, Dt, s->Fout, s->ext);
    // interface residual lambda' - lambda on the host
    const int ng = s->n_gamma;
    k_gamma_gather(L, s->gidx, ng, s->ccur, s->lam, s->gbuf);
    if (ng > 0)
      hip_check(hipMemcpyAsync(s->h_gbuf, s->gbuf, 2 * sizeof(double) * ng,
                               hipMemcpyDeviceToHost, s->stream),
                "hipMemcpyAsync(interface)");
    hip_check(hipStreamSynchronize(s->stream), "hipStreamSynchronize");
    lt_v.resize(ng);
    lam_v.resize(ng);
    double diff = 0.0;
    for (int q = 0; q < ng; ++q) {
      lt_v[q] = s->h_gbuf[2 * q];
      lam_v[q] = s->h_gbuf[2 * q + 1];
      diff = std::max(diff, std::fabs(lt_v[q] - lam_v[q]));
    }
    if (!std::isfinite(diff)) throw NoConv{"non-finite interface update"};
    if (diff <= op.dn_tol) break;
    iqn.update(lam_v, lt_v, s->theta0, op.dn_theta > 0.0, next);
    for (int q = 0; q < ng; ++q) s->h_gbuf[q] = next[q];
    hip_check(hipMemcpyAsync(s->gbuf, s->h_gbuf, sizeof(double) * ng,
                             hipMemcpyHostToDevice, s->stream),
              "hipMemcpyAsync(interface)");
    k_gamma_scatter(L, s->gidx, ng, s->gbuf, s->lam);
  }
  s->stats.dn_iters += it;
  ++s->stats.micro_steps;
  // bottom heat flow of the last fine step and of the coarse outside solve
  k_interface_accumulate(L, s->gf, w, s->fR, nullptr, 0, -dt, &led->bottom,
                         s->partials);
  k_bottom_sum(L, s->gc, s->cR, -Dt, &led->bottom, s->partials);
  std::swap(s->Tn, s->ccur);
  std::swap(s->fstate, s->fcur);
  energy_now(s, &led->stored);
  s->stats.fine_dof_steps += fine_free_nodes(s->gf, w) * m;
}

bool finite_all(std::initializer_list<double> v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

tl_status validate(const tl_mesh* me, const tl_material* ma,
                   const tl_scan_path* sp, const tl_options* op) {
  if (!me || !ma || !sp || !op) return fail(TL_EINVAL, "null argument");
  if (!finite_all({me->lx, me->ly, me->lz}) || me->lx <= 0 || me->ly <= 0 ||
      me->lz <= 0)
    return fail(TL_EINVAL, "plate sizes must be positive and finite");
  if (me->nx < 1 || me->ny < 1 || me->nz < 1)
    return fail(TL_EINVAL, "cell counts must be >= 1");
  if (me->refine < 1) return fail(TL_EINVAL, "refine must be >= 1");
  if (me->win_nx < 1 || me->win_ny < 1 || me->win_nz < 1 ||
      me->win_nx > me->nx || me->win_ny > me->ny || me->win_nz > me->nz)
    return fail(TL_EINVAL, "window must fit inside the plate");
  const double nf = (double)(me->refine * me->win_nx + 1) *
                    (me->refine * me->win_ny + 1) * (me->refine * me->win_nz + 1);
  const double nc = (double)(me->nx + 3) * (me->ny + 3) * (me->nz + 3);
  if (nf > 2.0e8 || nc > 2.0e8) return fail(TL_EINVAL, "grid too large");
  if (!finite_all({ma->rho, ma->T_lo, ma->T_hi, ma->c_lo, ma->c_hi, ma->k_lo,
                   ma->k_hi, ma->latent, ma->T_sol, ma->T_liq, ma->sharpness,
                   ma->T_init, ma->T_bottom}))
    return fail(TL_EINVAL, "non-finite material parameter");
  if (ma->rho <= 0 || ma->c_lo <= 0 || ma->c_hi <= 0 || ma->k_lo <= 0 ||
      ma->k_hi <= 0 || ma->latent < 0 || ma->sharpness <= 0)
    return fail(TL_EINVAL, "non-physical material parameter");
  if (!(ma->T_lo < ma->T_hi)) return fail(TL_EINVAL, "need T_lo < T_hi");
  if (!(ma->T_sol < ma->T_liq)) return fail(TL_EINVAL, "need T_sol < T_liq");
  if (ma->pc_kind != 0) return fail(TL_EINVAL, "pc_kind must be 0 (sigmoid)");
  if (sp->n_tracks < 1 || !sp->tracks)
    return fail(TL_EINVAL, "scan path needs at least one track");
  if (!std::isfinite(sp->t_start)) return fail(TL_EINVAL, "non-finite t_start");
  for (int q = 0; q < sp->n_tracks; ++q) {
    const tl_track& t = sp->tracks[q];
    if (!finite_all({t.x0, t.y0, t.x1, t.y1, t.speed, t.power, t.radius,
                     t.absorptivity}) ||
        t.speed <= 0 || t.radius <= 0 || t.power < 0 || t.absorptivity < 0)
      return fail(TL_EINVAL, "invalid track " + std::to_string(q));
  }
  if (!std::isfinite(op->dt_coarse) || op->dt_coarse <= 0)
    return fail(TL_EINVAL, "dt_coarse must be positive");
  if (op->m_time < 1 || op->m_time > kMaxSpots)
    return fail(TL_EINVAL, "m_time must be in 1..32");
  if (op->precision != TL_FP64 && op->precision != TL_MIXED)
    return fail(TL_EINVAL, "unknown precision");
  if (op->face_quad < 1 || op->face_quad > 4)
    return fail(TL_EINVAL, "face_quad must be in 1..4");
  if (!finite_all({op->newton_tol, op->cg_rtol, op->dn_tol, op->dn_theta}) ||
      op->newton_tol <= 0 || op->cg_rtol <= 0 || op->dn_tol <= 0 ||
      op->dn_theta > 2.0)
    return fail(TL_EINVAL, "invalid tolerance or relaxation");
  if (op->newton_max < 1 || op->cg_max < 1 || op->dn_max < 1)
    return fail(TL_EINVAL, "iteration caps must be >= 1");
  return TL_OK;
}

}  // namespace

// ===========================================================================
// C interface
// ===========================================================================
extern "C" {

const char* tl_last_error(void) { return g_last_error.c_str(); }

size_t tl_workspace_bytes(const tl_mesh* mesh, const tl_options* opts) {
  if (!mesh || !opts || mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1 ||
      mesh->refine < 1 || mesh->win_nx < 1 || mesh->win_ny < 1 ||
      mesh->win_nz < 1 || !(mesh->lx > 0) || !(mesh->ly > 0) || !(mesh->lz > 0))
    return 0;
  return make_layout(*mesh, *opts).total;
}

static tl_status init_state(tl_sim* s) {
  const Launch L = s->L;
  k_zero_bytes(L, s->ws, s->lay.total);
  // initial temperatures: T_init everywhere, T_bottom on the bottom face
  std::vector<double> hc;
  k_fill(L, s->Tn, 0.0, s->gc.npad);
  k_fill(L, s->fstate, 0.0, s->gf.npad);
  HIP_OK(hipStreamSynchronize(s->stream));
  // fill the real nodes on the host and upload (once)
  auto upload = [&](double* dst, const Geo& g, bool has_bottom) -> tl_status {
    std::vector<double> h((size_t)g.npad, 0.0);
    for (int k = 0; k < g.nz; ++k)
      for (int j = 0; j < g.ny; ++j)
        for (int i = 0; i < g.nx; ++i)
          h[(size_t)(k + 1) * g.pxy + (size_t)(j + 1) * g.px + (i + 1)] =
              (has_bottom && k == 0) ? s->mat_in.T_bottom : s->mat_in.T_init;
    HIP_OK(hipMemcpy(dst, h.data(), h.size() * sizeof(double),
                     hipMemcpyHostToDevice));
    return TL_OK;
  };
  tl_status st = upload(s->Tn, s->gc, true);
  if (st != TL_OK) return st;
  st = upload(s->fstate, s->gf, s->win.bottom != 0);
  if (st != TL_OK) return st;
  energy_now(s, &s->led->stored);
  read_ledger(s);
  s->ledger.stored = s->h_led->stored;
  s->ledger.stored0 = s->h_led->stored;
  s->ledger.absorbed = s->ledger.bottom = s->ledger.remap = 0.0;
  write_ledger(s);
  return TL_OK;
}

tl_status tl_create(const tl_mesh* mesh, const tl_material* material,
                    const tl_scan_path* scan, const tl_options* opts,
                    void* dev_workspace, size_t ws_bytes, void* hip_stream,
                    tl_sim** out) {
  if (!out) return fail(TL_EINVAL, "out is null");
  *out = nullptr;
  tl_status st = validate(mesh, material, scan, opts);
  if (st != TL_OK) return st;
  Layout lay = make_layout(*mesh, *opts);
  if (!dev_workspace) return fail(TL_EINVAL, "workspace is null");
  if (((uintptr_t)dev_workspace) % kAlign != 0)
    return fail(TL_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < lay.total)
    return fail(TL_ENOMEM, "workspace too small: need " +
                               std::to_string(lay.total) + " bytes");
  tl_sim* s = new tl_sim();
  s->mesh = *mesh;
  s->mat_in = *material;
  s->opts = *opts;
  s->t_start = scan->t_start;
  for (int q = 0; q < scan->n_tracks; ++q) {
    const tl_track& t = scan->tracks[q];
    s->tracks.push_back(TrackH{t.x0, t.y0, t.x1, t.y1, t.speed, t.power,
                               t.radius, t.absorptivity});
  }
  MatDev& m = s->mat;
  m.rho = material->rho;
  m.T_lo = material->T_lo;
  m.T_hi = material->T_hi;
  m.c_lo = material->c_lo;
  m.c_hi = material->c_hi;
  m.k_lo = material->k_lo;
  m.k_hi = material->k_hi;
  m.latent = material->latent;
  m.Tm = 0.5 * (material->T_sol + material->T_liq);
  m.S = material->sharpness;
  m.cslope = (m.c_hi - m.c_lo) / (m.T_hi - m.T_lo);
  m.kslope = (m.k_hi - m.k_lo) / (m.T_hi - m.T_lo);
  m.sens_full = 0.5 * (m.c_lo + m.c_hi) * (m.T_hi - m.T_lo);
  s->lay = lay;
  s->gc = lay.gc;
  s->gf = lay.gf;
  s->stream = (hipStream_t)hip_stream;
  s->L.stream = hip_stream;
  s->ws = (char*)dev_workspace;
  auto C = [&](int a) { return (double*)(s->ws + lay.off_c[a]); };
  s->Tn = C(0); s->Tpred = C(1); s->ccur = C(2); s->ctrial = C(3);
  s->lam = C(4); s->dprev = C(5); s->cR = C(6); s->Fall = C(7);
  s->Fout = C(8); s->ext = C(9);
  auto cgb64 = [&](auto A) {
    return CGBufs<double>{(double*)A(0), (double*)A(1), (double*)A(2),
                          {(double*)A(3), (double*)A(4)},
                          {(double*)A(5), (double*)A(6)},
                          {(double*)A(7), (double*)A(8)}, (double*)A(9),
                          {(double*)A(10), (double*)A(11)}};
  };
  s->ccg = cgb64([&](int a) { return (void*)C(10 + a); });
  auto FD = [&](int a) { return (double*)(s->ws + lay.off_fd[a]); };
  s->fstate = FD(0); s->fprev = FD(1); s->fcur = FD(2); s->ftrial = FD(3);
  s->falt = FD(4); s->fR = FD(5); s->fF = FD(6); s->rho = FD(7);
  auto FC = [&](int a) { return (void*)(s->ws + lay.off_fcg[a]); };
  s->fcg64 = cgb64(FC);
  s->fcg32 = CGBufs<float>{(float*)FC(0), (float*)FC(1), (float*)FC(2),
                           {(float*)FC(3), (float*)FC(4)},
                           {(float*)FC(5), (float*)FC(6)},
                           {(float*)FC(7), (float*)FC(8)}, (float*)FC(9),
                           {(float*)FC(10), (float*)FC(11)}};
  s->sc_c = (LevelScalars*)(s->ws + lay.off_scal);
  s->sc_f = s->sc_c + 1;
  s->led = (LedgerDev*)(s->ws + lay.off_ledger);
  s->partials = (double*)(s->ws + lay.off_partials);
  s->gidx = (int*)(s->ws + lay.off_gidx);
  s->gbuf = (double*)(s->ws + lay.off_gbuf);
  if (hipHostMalloc((void**)&s->h_sc, sizeof(LevelScalars), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&s->h_led, sizeof(LedgerDev), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&s->h_gbuf, 2 * sizeof(double) * lay.gamma_cap,
                    hipHostMallocDefault) != hipSuccess) {
    delete s;
    return fail(TL_EDEVICE, "hipHostMalloc failed");
  }
  std::memset(&s->stats, 0, sizeof(s->stats));
  s->stats.fine_nodes[0] = s->gf.nx;
  s->stats.fine_nodes[1] = s->gf.ny;
  s->stats.fine_nodes[2] = s->gf.nz;
  s->stats.coarse_nodes[0] = s->gc.nx;
  s->stats.coarse_nodes[1] = s->gc.ny;
  s->stats.coarse_nodes[2] = s->gc.nz;
  s->n_macro = 0;
  s->theta0 = opts->dn_theta > 0 ? opts->dn_theta
                                 : mesh->refine / (mesh->refine + 1.0);
  s->last_cg_f = s->last_cg_c = 8;
  int I0, J0;
  window_origin(s->tracks.data(), (int)s->tracks.size(), s->t_start,
                micro_time(s->t_start, opts->dt_coarse, opts->m_time, 1, 0),
                s->gc.hx, s->gc.hy, mesh->nx, mesh->ny, mesh->win_nx,
                mesh->win_ny, 0, 0, 0, &I0, &J0);
  s->win = make_window(*mesh, I0, J0);
  s->gf.x0 = I0 * s->gc.hx;
  s->gf.y0 = J0 * s->gc.hy;
  try {
    st = init_state(s);  // zero-fills the whole workspace first
    if (st == TL_OK) set_interface(s);
  } catch (const DevErr& e) {
    st = fail(TL_EDEVICE, e.msg);
  }
  if (st != TL_OK) {
    tl_destroy(s);
    return st;
  }
  *out = s;
  return TL_OK;
}

tl_status tl_step(tl_sim* s, int n_macro) {
  if (!s) return fail(TL_EINVAL, "null handle");
  if (n_macro < 0) return fail(TL_EINVAL, "n_macro must be >= 0");
  auto t0 = std::chrono::steady_clock::now();
  tl_status st = TL_OK;
  for (int q = 0; q < n_macro; ++q) {
    const Window w_saved = s->win;
    const Geo gf_saved = s->gf;
    double* state_saved = s->fstate;
    double* alt_saved = s->falt;
    const tl_stats stats_saved = s->stats;
    try {
      macro_step(s);
      read_ledger(s);
      s->ledger.stored = s->h_led->stored;
      s->ledger.absorbed = s->h_led->absorbed;
      s->ledger.bottom = s->h_led->bottom;
      s->ledger.remap = s->h_led->remap;
      ++s->n_macro;
      ++s->stats.macro_steps;
    } catch (const NoConv& e) {
      st = fail(TL_ENOCONV, "macro step " + std::to_string(s->n_macro) + ": " + e.msg);
    } catch (const DevErr& e) {
      st = fail(TL_EDEVICE, e.msg);
    }
    if (st != TL_OK) {
      // roll back to the last completed macro step: the committed coarse
      // field Tn is only replaced at the end of a step; the fine state may
      // have been remapped by a window move
      (void)hipStreamSynchronize(s->stream);
      s->win = w_saved;
      s->gf = gf_saved;
      s->fstate = state_saved;
      s->falt = alt_saved;
      s->stats = stats_saved;
      try {
        set_interface(s);
        k_fill(s->L, s->ext, 0.0, s->gc.npad);
        write_ledger(s);
      } catch (const DevErr& e) {
        st = fail(TL_EDEVICE, e.msg);
      }
      break;
    }
  }
  auto t1 = std::chrono::steady_clock::now();
  s->stats.step_ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
  return st;
}

tl_status tl_get_temperature(tl_sim* s, int level, double* host_out,
                             size_t cap, int dims_out[3],
                             int fine_origin_out[3]) {
  if (!s || !host_out || !dims_out) return fail(TL_EINVAL, "null argument");
  if (level != 0 && level != 1) return fail(TL_EINVAL, "level must be 0 or 1");
  const Geo& g = level == 0 ? s->gc : s->gf;
  if (cap < (size_t)g.nreal) return fail(TL_ENOMEM, "host buffer too small");
  double* scratch = level == 0 ? s->ctrial : s->falt;
  const double* src = level == 0 ? s->Tn : s->fstate;
  k_unpack(s->L, g, 0, 8, src, scratch);
  HIP_OK(hipMemcpyAsync(host_out, scratch, (size_t)g.nreal * sizeof(double),
                        hipMemcpyDeviceToHost, s->stream));
  HIP_OK(hipStreamSynchronize(s->stream));
  dims_out[0] = g.nx;
  dims_out[1] = g.ny;
  dims_out[2] = g.nz;
  if (fine_origin_out) {
    fine_origin_out[0] = s->win.r * s->win.I0;
    fine_origin_out[1] = s->win.r * s->win.J0;
    fine_origin_out[2] = s->win.r * s->win.K0;
  }
  return TL_OK;
}

tl_status tl_get_ledger(tl_sim* s, tl_ledger* out) {
  if (!s || !out) return fail(TL_EINVAL, "null argument");
  *out = s->ledger;
  return TL_OK;
}

tl_status tl_get_stats(tl_sim* s, tl_stats* out) {
  if (!s || !out) return fail(TL_EINVAL, "null argument");
  *out = s->stats;
  return TL_OK;
}

tl_status tl_get_time(tl_sim* s, double* t, int64_t* n) {
  if (!s) return fail(TL_EINVAL, "null handle");
  if (t) *t = s->t_start + (double)s->n_macro * s->opts.dt_coarse;
  if (n) *n = s->n_macro;
  return TL_OK;
}

namespace {
struct CkptHeader {
  char magic[8];
  int32_t version;
  int32_t I0, J0;
  int32_t gc_n, gf_n;
  int64_t n_macro;
  tl_ledger ledger;
  tl_stats stats;
};
}  // namespace

tl_status tl_save(tl_sim* s, void* host, size_t cap, size_t* used) {
  if (!s || !used) return fail(TL_EINVAL, "null argument");
  const size_t need = sizeof(CkptHeader) +
                      ((size_t)s->gc.nreal + s->gf.nreal) * sizeof(double);
  *used = need;
  if (!host) return TL_OK;
  if (cap < need) return fail(TL_ENOMEM, "checkpoint buffer too small");
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, "TLCKPT1", 8);
  h.version = 1;
  h.I0 = s->win.I0;
  h.J0 = s->win.J0;
  h.gc_n = s->gc.nreal;
  h.gf_n = s->gf.nreal;
  h.n_macro = s->n_macro;
  h.ledger = s->ledger;
  h.stats = s->stats;
  char* p = (char*)host;
  std::memcpy(p, &h, sizeof(h));
  int dims[3];
  tl_status st = tl_get_temperature(s, 0, (double*)(p + sizeof(h)),
                                    (size_t)s->gc.nreal, dims, nullptr);
  if (st != TL_OK) return st;
  return tl_get_temperature(
      s, 1, (double*)(p + sizeof(h) + (size_t)s->gc.nreal * sizeof(double)),
      (size_t)s->gf.nreal, dims, nullptr);
}

tl_status tl_load(tl_sim* s, const void* host, size_t n) {
  if (!s || !host) return fail(TL_EINVAL, "null argument");
  if (n < sizeof(CkptHeader)) return fail(TL_EINVAL, "checkpoint too short");
  CkptHeader h;
  std::memcpy(&h, host, sizeof(h));
  if (std::memcmp(h.magic, "TLCKPT1", 8) != 0 || h.version != 1)
    return fail(TL_EINVAL, "not a checkpoint of this library");
  if (h.gc_n != s->gc.nreal || h.gf_n != s->gf.nreal)
    return fail(TL_EINVAL, "checkpoint grid sizes differ from this handle");
  const size_t need = sizeof(CkptHeader) +
                      ((size_t)s->gc.nreal + s->gf.nreal) * sizeof(double);
  if (n < need) return fail(TL_EINVAL, "checkpoint truncated");
  if (h.I0 < 0 || h.J0 < 0 || h.I0 + s->mesh.win_nx > s->mesh.nx ||
      h.J0 + s->mesh.win_ny > s->mesh.ny)
    return fail(TL_EINVAL, "checkpoint window outside the plate");
  const char* p = (const char*)host + sizeof(h);
  try {
    s->win = make_window(s->mesh, h.I0, h.J0);
    s->gf.x0 = h.I0 * s->gc.hx;
    s->gf.y0 = h.J0 * s->gc.hy;
    set_interface(s);
    HIP_OK(hipMemcpyAsync(s->ctrial, p, (size_t)s->gc.nreal * sizeof(double),
                          hipMemcpyHostToDevice, s->stream));
    k_pack(s->L, s->gc, 0, 8, s->ctrial, s->Tn);
    HIP_OK(hipMemcpyAsync(s->falt, p + (size_t)s->gc.nreal * sizeof(double),
                          (size_t)s->gf.nreal * sizeof(double),
                          hipMemcpyHostToDevice, s->stream));
    k_pack(s->L, s->gf, 0, 8, s->falt, s->fstate);
    k_fill(s->L, s->ext, 0.0, s->gc.npad);
    s->n_macro = h.n_macro;
    s->ledger = h.ledger;
    s->stats = h.stats;
    write_ledger(s);
  } catch (const DevErr& e) {
    return fail(TL_EDEVICE, e.msg);
  }
  return TL_OK;
}

tl_status tl_set_profiling(tl_sim* s, int sample_every) {
  if (!s) return fail(TL_EINVAL, "null handle");
  if (sample_every < 0) return fail(TL_EINVAL, "sample_every must be >= 0");
  if (sample_every > 0 && !s->prof_ev[0]) {
    for (int q = 0; q < 2 * kProfPairs; ++q)
      HIP_OK(hipEventCreate(&s->prof_ev[q]));
  }
  s->prof_every = sample_every;
  s->prof_count = 0;
  return TL_OK;
}

void tl_destroy(tl_sim* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  else (void)hipDeviceSynchronize();
  if (s->prof_ev[0])
    for (int q = 0; q < 2 * kProfPairs; ++q) (void)hipEventDestroy(s->prof_ev[q]);
  if (s->h_sc) (void)hipHostFree(s->h_sc);
  if (s->h_led) (void)hipHostFree(s->h_led);
  if (s->h_gbuf) (void)hipHostFree(s->h_gbuf);
  delete s;
}

// ---- operator-level entry points (tl_ops.h) --------------------------------
static Geo geo_of(const tl_grid* g) {
  return make_geo(g->nx, g->ny, g->nz, g->hx, g->hy, g->hz, 0.0, 0.0);
}
static tl_status check_grid(const tl_grid* g) {
  if (!g) return fail(TL_EINVAL, "null grid");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1)
    return fail(TL_EINVAL, "cell counts must be >= 1");
  if (!(g->hx > 0) || !(g->hy > 0) || !(g->hz > 0) || !std::isfinite(g->hx) ||
      !std::isfinite(g->hy) || !std::isfinite(g->hz))
    return fail(TL_EINVAL, "spacings must be positive and finite");
  if ((double)(g->nx + 3) * (g->ny + 3) * (g->nz + 3) > 2.0e9)
    return fail(TL_EINVAL, "grid too large");
  return TL_OK;
}

size_t tl_op_padded_size(const tl_grid* grid) {
  if (check_grid(grid) != TL_OK) return 0;
  return (size_t)geo_of(grid).npad;
}

tl_status tl_op_pack(const tl_grid* grid, int kind, int elem_bytes,
                     const void* plain, void* padded, void* hip_stream) {
  tl_status st = check_grid(grid);
  if (st != TL_OK) return st;
  if ((kind != 0 && kind != 1) || (elem_bytes != 4 && elem_bytes != 8) ||
      !plain || !padded)
    return fail(TL_EINVAL, "bad pack arguments");
  Launch L{hip_stream};
  k_pack(L, geo_of(grid), kind, elem_bytes, plain, padded);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize((hipStream_t)hip_stream));
  return TL_OK;
}

tl_status tl_op_unpack(const tl_grid* grid, int kind, int elem_bytes,
                       const void* padded, void* plain, void* hip_stream) {
  tl_status st = check_grid(grid);
  if (st != TL_OK) return st;
  if ((kind != 0 && kind != 1) || (elem_bytes != 4 && elem_bytes != 8) ||
      !plain || !padded)
    return fail(TL_EINVAL, "bad unpack arguments");
  Launch L{hip_stream};
  k_unpack(L, geo_of(grid), kind, elem_bytes, padded, plain);
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize((hipStream_t)hip_stream));
  return TL_OK;
}

tl_status tl_op_apply(const tl_grid* grid, int precision, const void* d,
                      const void* kappa, const void* v, void* y, int repeat,
                      void* hip_stream) {
  tl_status st = check_grid(grid);
  if (st != TL_OK) return st;
  if (!d || !kappa || !v || !y || repeat < 1)
    return fail(TL_EINVAL, "bad operator arguments");
  if (precision != TL_FP64 && precision != TL_MIXED)
    return fail(TL_EINVAL, "unknown precision");
  Launch L{hip_stream};
  const Geo g = geo_of(grid);
  for (int q = 0; q < repeat; ++q) {
    if (precision == TL_FP64)
      k_op_apply<double>(L, g, (const double*)d, (const double*)kappa,
                         (const double*)v, (double*)y);
    else
      k_op_apply<float>(L, g, (const float*)d, (const float*)kappa,
                        (const float*)v, (float*)y);
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize((hipStream_t)hip_stream));
  return TL_OK;
}

}  // extern "C"
