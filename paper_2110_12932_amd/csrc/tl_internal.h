// Internal declarations shared by the HIP kernels (tl_kernels.hip), the
// solver runtime (tl_runtime.cpp) and the host-side geometry and scan-path
// logic (tl_host.cpp).  Not part of the public interface.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace tl {

constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts of 64)
constexpr int kMaxBlocks = 2048; // grid cap for grid-stride kernels
constexpr int kMaxSpots = 32;    // laser positions averaged by one load call

// Structured Q1 grid in the padded layout: node (i,j,k) at
// (k+1)*pxy + (j+1)*px + (i+1); the element whose lowest corner is node
// (i,j,k) is stored at that node's index.
struct Geo {
  int nx, ny, nz;        // nodes per axis
  int px, pxy;           // padded strides: px = nx+2 rounded up to a
                         // multiple of 32 (rows start on 128-byte lines),
                         // pxy = px*(ny+2)
  int nreal;             // nx*ny*nz
  long npad;             // pxy*(nz+2)
  double hx, hy, hz;     // spacing
  double x0, y0;         // coordinates of node (0,0,*)
  double vol8;           // element volume / 8
  double w[8];           // element stiffness K_e[a][b] by the xor pattern a^b
};

// Which elements are active and which nodes are Dirichlet, as index rules.
enum RegionMode {
  kAllBottom = 0,   // all elements; Dirichlet on k = 0 (coarse predictor)
  kOutside = 1,     // coarse elements outside the window box; Dirichlet on
                    // k = 0 and on window nodes not on an immersed face
  kWindow = 2,      // fine window: all elements; Dirichlet on immersed faces
                    // and, when the window reaches the plate bottom, k = 0
  kFictitious = 3   // coarse plate, all elements, Dirichlet on k = 0; the
                    // elements of the window box [I0,I1) x [J0,J1) x [K0,..)
                    // carry the constant coefficients kf, rhocf (the
                    // consistent global problem); top-surface loss outside
                    // the window only
};
enum FaceBits { kFx0 = 1, kFx1 = 2, kFy0 = 4, kFy1 = 8, kFz0 = 16 };

struct Region {
  int mode;
  int I0, I1, J0, J1, K0;  // kOutside: coarse window box in cells [I0,I1) ...
  int faces;               // immersed faces (FaceBits) for kOutside/kWindow
  int bottom;              // kWindow: 1 if node layer k = 0 is on the plate bottom
  double kf, rhocf;        // kFictitious: conductivity and volumetric heat
                           // capacity of the window box's elements
};

struct MatDev {
  double rho, T_lo, T_hi, c_lo, c_hi, k_lo, k_hi, latent, Tm, S;
  double cslope, kslope, sens_full;  // derived on the host
};

// Top-surface heat loss of one level: q(T) = h (T - T_amb) + es (T^4 -
// T_amb^4), es = sigma * emissivity (0 on the coarse level).
struct SurfDev {
  double h, es, T_amb;
};
constexpr double kSigmaSB = 5.670374419e-8;   // W / (m^2 K^4)

// One laser position with its flux parameters q0 = 3 eta P / (pi R^2) and
// a3 = 3 / R^2, and the weight of this position in a time average.
struct Spot { double xc, yc, q0, a3, weight; };

// Volume laser model (paper Section 5.2).  Local level: the volumetric
// Gaussian amp * exp(-a3 ((x-xc)^2 + (y-yc)^2) - az (z - z_top)^2) of one
// spot; global level: constant sources q in axis-aligned boxes (the path the
// beam sweeps in a macro step), z given as depth below the top surface.
struct VolSpot { double xc, yc, amp, a3, az; int on; };
constexpr int kMaxBoxes = 8;
struct Box { double x_lo, x_hi, y_lo, y_hi, depth, q; };
struct BoxSet {
  int n;
  Box b[kMaxBoxes];
};

struct SpotSet {
  int n;
  int nq;                  // Gauss points per face direction
  double gx[4], gw[4];     // Gauss points and weights on [0, 1]
  Spot s[kMaxSpots];
};

// Newton state of one implicit solve, kept on the device so that the host
// can queue several Newton rounds between synchronisations.  Round r reads
// ns[r & 1]; only workgroup 0 of round r's CG-start kernel writes, into
// ns[(r + 1) & 1], which no kernel of round r reads before that.
constexpr int kLineSearchMax = 12;  // halvings tried before a step is taken anyway
enum NewtonStatus {
  kRunning = 0,
  kConverged = 1,
  kFailNonFinite = 2,   // non-finite residual or update
  kFailBreakdown = 3,   // CG broke down before its first iteration
  kFailNewtonMax = 4    // no convergence within newton_max directions
};
struct NewtonState {
  double alpha;       // step of the trial evaluated in this round
  double rn0;         // |R_free| at the accepted temperature
  double dmax_last;   // max |alpha dx| of the last accepted step
  double dmax_prev;   // the same for the accepted step before it
  int cur;            // Tb[cur] holds the accepted temperature
  int xi;             // xb[xi] holds the direction being line-searched
  int h;              // halvings of the current direction
  int first;          // no accepted evaluation yet (trial = T, no direction)
  int pending;        // the direction was produced by the previous round's CG
  int status;         // NewtonStatus
  int budget;         // CG iterations a round may run (fixed per solve, so
                      // that a solve does not depend on the others of its
                      // batch)
  int cg_need;        // most CG iterations a direction took (+2 if cut)
  int n_newton;       // directions taken
  int n_cg;           // CG iterations summed over the solve
  int n_halvings;     // line-search halvings summed over the solve
  int dir_cut;        // the direction being line-searched comes from a CG
                      // that its budget stopped before it reached cg_rtol
};
// CG scalars of one round, double-buffered by round parity: round r's CG
// kernels use cg[r & 1] and the next round's CG-start reads its outcome.
struct CGScalars {
  double rz0;        // r.z at the start of the CG solve
  double gbuf[2];    // gamma_k = r_k.u_k in gbuf[k & 1]
  double abuf[2];    // alpha_k in abuf[k & 1]
  int iters, done, breakdown, pad;
};
constexpr int kRoundLog = 32;   // rounds whose CG iteration counts are kept
struct LevelScalars {
  NewtonState ns[2];
  CGScalars cg[2];
  double rnorm2;     // |R_free|^2 at the last evaluated trial
  double dmax;       // max |alpha dx| of the last evaluated trial
  int cg_log[kRoundLog];   // CG iterations of round r at [r % kRoundLog]
};

// Per-workgroup partial sums of the generic reductions (loads, energy,
// bottom reactions): kMaxBlocks doubles, summed by a one-workgroup kernel.
enum PartialRegion { kPartGen = 0, kPartAux = 1, kPartRegions = 2 };

// Per-tile partial sums of the batched Newton/CG kernels: regions of
// `tstride` doubles indexed by tile.  A consumer sums an item's tiles in
// tile order, so the result does not depend on how many workgroups shared
// the tiles.  The CG iteration kernels alternate between two region pairs
// by parity, since a kernel never writes a region it reads (a grid larger
// than the resident capacity has workgroups that start only after others
// have finished).
enum TilePartial {
  kTRes = 0,    // residual kernel: |R_free|^2, max |alpha dx|, r.(Dinv r)
  kTCG = 3,     // CG gamma/delta, written by CG start and odd iterations
  kTCG2 = 5,    // CG gamma/delta, written by even iterations
  kTileRegions = 7
};

// Energy ledger slots on the device.
struct LedgerDev {
  double stored, stored0, absorbed, bottom, remap, surface;
  double e_tmp0, e_tmp1;
};

// Fine window placement on the coarse plate and its transfer parameters.
struct Window {
  int I0, J0, K0;           // lowest coarse node of the window
  int wx, wy, wz;           // window size in coarse cells
  int r;                    // refinement
  int faces;                // immersed faces
  int bottom;               // window reaches the plate bottom
};

// ---- kernels launched from the runtime (tl_kernels.hip) -------------------
struct Launch { void* stream; };

void k_fill(Launch L, double* a, double v, long n);
void k_zero_bytes(Launch L, void* a, size_t bytes);
void k_copy(Launch L, double* dst, const double* src, long n);
// dst = 2 a - b (a linear extrapolation in time)
void k_extrapolate(Launch L, double* dst, const double* a, const double* b,
                   long n);

// Bare operator kernels: chosen by grid size, 3D LDS tiles, z-marching
// columns.  blocks > 0 (a multiple of 8) overrides the workgroup count.
enum OpKernel { kOpAuto = 0, kOpTiled = 1, kOpZmarch = 2 };
template <class R>
void k_op_apply(Launch L, const Geo& g, int kernel, int blocks, const R* d,
                const R* kap, const R* v, R* y);

// Composite-grid coupling: the two-level correction solved as one system
// over the free fine nodes and the coarse nodes outside the window interior,
// with the fine interface values slaved to the coarse ones (T-_gamma =
// P T+_Gamma) and the fine rows scaled by 1/m so that the frozen-kappa
// Jacobian is symmetric.  The pair is a fine item and a coarse item that
// share one Newton/CG state; every launch of a round runs the fine side, a
// gather kernel (P^T of the fine interface rows onto the coarse interface
// nodes), then the coarse side.  The fine side reads its interface values
// as prolonged from the coarse arrays; the coarse side adds the gathered
// rows on its interface nodes.  Both sides sum the pair's tile partials in the same
// order (fine tiles, then coarse tiles), so they take the same decisions.
// Before each fine launch a prolongation kernel writes the coarse values
// onto the fine side's interface nodes.
// kFineSide forms its interface values inside its own kernels (fewest
// launches: the choice for one or a few simulations); kFineSideP reads them
// as written by the prolongation kernel before it (cheaper kernels: the
// choice for large batches).  Both give bitwise the same values.
enum CoupleSide { kAlone = 0, kFineSide = 1, kCoarseSide = 2, kFineSideP = 3 };
struct Couple {
  Window w;              // window placement
  Geo go;                // the other level's grid
  double rscale;         // scale of this side's rows (1/m fine, 1 coarse)
  // fine side: the coarse arrays its interface values come from
  const double* oT[2];   // temperatures (Tb)
  const void* ox[2];     // Newton directions (xb)
  const void* odinv;     // Jacobi preconditioner
  const void* orr[2];    // CG residuals
  const void* ow[2];     // J u
  const void* os[2];     // J p
  // coarse side: the fine arrays the gather kernel restricts, and where
  // the gathered rows go (coarse-indexed, read on interface nodes only)
  const double* fR;      // fine residual (rows scaled by 1/m)
  const void* fdiag;     // fine Jacobian diagonal on interface rows (the
                         // fine preconditioner array holds it there)
  const void* fw[2];     // fine J u
  double* gR;            // gathered residual rows
  void* gDW;             // gathered diagonal (double, residual phase), then
                         // gathered J u rows (CG precision, CG phases)
  const int* gidx;       // padded indices of the coarse interface nodes
  int ngamma;
  // the pair's per-tile partials: fine tiles (A), then coarse tiles (B);
  // an item alone has only A (its own)
  int ntA, ntB, tsA, tsB;
  const double* tpA;
  const double* tpB;
};

// One level solve in a batched Newton/CG launch (device-resident table).
// CG-precision arrays are untyped; the launch's precision decides.
struct SolveItem {
  Geo g;
  Region rg;
  MatDev m;
  SurfDev sf;        // top-surface loss of this level
  double tau;
  double tol;        // Newton tolerance on max |alpha dx| [K]
  double rtol2;      // CG: stop when r.u <= rtol2 * r0.u0
  int newton_max;    // Newton directions allowed
  int cg_max;        // CG iterations allowed per direction
  int ntx, nty, ntiles;     // tiles of this item
  int tstride;              // entries per region of tpart (>= ntiles)
  double* Tb[2];       // the accepted and the trial temperature (see ns.cur)
  const double* Told;  // temperature at the previous time level
  double* Hold;        // H(Told): written in a solve's first round, then read
  const double* F;     // surface load at the new time level
  const double* Fext;  // interface load (null if none)
  double* R;           // residual at the trial
  void* xb[2];         // CG solutions: the direction being line-searched
                       // and the next one (see ns.xi)
  void* kap;           // element conductivity
  void* d;             // m H'(T) / tau
  void* dinv;          // Jacobi preconditioner, 0 on Dirichlet rows
  void* r[2];          // CG residual (double-buffered by parity)
  void* w[2];          // J u (double-buffered)
  void* s[2];          // J p (double-buffered)
  void* p;             // search direction
  LevelScalars* sc;    // per-item scalars (shared by a composite pair)
  double* tpart;       // per-tile partial sums, kTileRegions * tstride
  Couple cp;           // composite-grid coupling (cp side kAlone: none)
};

// Tiles of a grid in the batched kernels.
int grid_tiles(const Geo& g, int& ntx, int& nty);
// Workgroups every item of a batched tiled launch gets (a multiple of 8),
// for a largest item of ntiles tiles and a kernel of which the device holds
// `resident` workgroups at once: one per tile up to kResidentShare times
// that residency when alone, a share of it in larger batches but at least
// 64 (each workgroup then walks several tiles, the next tile's loads in
// flight during the current one; an item with fewer tiles leaves some
// workgroups without work).  A launch larger than the device holds would
// run its last workgroups as a partly filled second wave.
constexpr double kResidentShare = 1.0;
int item_tile_blocks(int ntiles, int n_items, int resident);

// Stacks of two tiles along z on grid g (work units of the CG kernels on
// large items).
int cg_stacks(const Geo& g);

// Batched launches of Newton round `round` over a device table of n_items
// items whose largest has ntiles tiles and nstacks stacks of two
// (cg_stacks); the grid follows item_tile_blocks.
// ev_start/ev_stop (hipEvent_t, may be null) are recorded with the CG
// dispatch itself.
template <class R>
void k_residual_batched(Launch L, const SolveItem* items, int n_items,
                        int ntiles, int round);
template <class R>
void k_cg_start_batched(Launch L, const SolveItem* items, int n_items,
                        int ntiles, int nstacks, int round);
template <class R>
void k_cg_iter_batched(Launch L, const SolveItem* items, int n_items,
                       int ntiles, int nstacks, int round, int kit,
                       void* ev_start, void* ev_stop);
// The same launches for the two sides of composite pairs (side =
// kFineSide or kCoarseSide), and the gather between them over the coarse
// sides' table: phase 0 after the residual, 1 after the CG start, 2 after
// CG iteration kit.
template <class R>
void k_residual_pair(Launch L, const SolveItem* items, int n_items,
                     int ntiles, int round, int side);
template <class R>
void k_cg_start_pair(Launch L, const SolveItem* items, int n_items,
                     int ntiles, int nstacks, int round, int side);
template <class R>
void k_cg_iter_pair(Launch L, const SolveItem* items, int n_items,
                    int ntiles, int nstacks, int round, int kit, int side,
                    void* ev_start, void* ev_stop);
template <class R>
void k_couple_gather(Launch L, const SolveItem* coarse_items, int n_items,
                     int max_gamma, int round, int phase, int kit);
// The prolongation onto the fine sides' interface nodes before each fine
// launch of composite pairs (same phases), per_item workgroups per pair.
template <class R>
void k_couple_prolong(Launch L, const SolveItem* fine_items, int n_items,
                      int per_item, int round, int phase, int kit);

void k_laser_load(Launch L, const Geo& g, const SpotSet& spots, int fI0,
                  int fI1, int fJ0, int fJ1, double* F, double ledger_scale,
                  double* ledger_slot, double* partials);

// Volume model loads: F = int Q- phi_i over the grid (its top layer on the
// plate top), and F = sum over boxes of q int_{box} phi_i over the elements
// the region keeps (kOutside: outside the window); each adds
// ledger_scale * sum(F) into *ledger_slot when that is not null.
void k_volume_load(Launch L, const Geo& g, const VolSpot& sp, double* F,
                   double ledger_scale, double* ledger_slot, double* partials);
void k_box_load(Launch L, const Geo& g, const Region& rg, const BoxSet& bs,
                double* F, double ledger_scale, double* ledger_slot,
                double* partials);

// The per-simulation work around one fine micro step, for many
// simulations in one launch: before the solve, the initial guess (prev, or
// 2 prev - pp), the Dirichlet data (T_bottom on the plate bottom, the
// prolonged blend (1 - wb) P Ta + wb P Tb on immersed faces) and the laser
// load F with its absorbed energy; after it, the interface reactions into
// rho and the bottom and top-surface heat flows.  A simulation's
// workgroup count `nblk` follows from its own size only (micro_blocks), so
// its sums do not depend on the others.  Ledger slots may be null (nothing
// booked).
constexpr int kMaxMicroBlocks = 256;
int micro_blocks(const Geo& gf);
struct MicroItem {
  int nblk;
  Geo gf, gc;
  Window w;
  double T_bottom, wb;
  const double* Ta;
  const double* Tb;
  const double* prev;
  const double* pp;        // null: the guess is prev
  double* cur;
  int source;              // 0 surface Gaussian, 1 volumetric Gaussian
  int nq;                  // surface model: Gauss rule on [0, 1]
  double gx[4], gw[4];
  Spot spot;               // surface model (weight 0: beam off)
  VolSpot vs;              // volume model
  double* F;
  double* part;            // the simulation's partials, kPartRegions regions
  double* slot_abs;
  double scale_abs;
  const double* R;         // after the solve: residual at the solution
  double* rho;             // reaction accumulator (null: none)
  int rho_init;
  double* slot_bottom;
  double scale_bottom;
  Region rgw;              // region for the top-surface areas
  SurfDev sf;
  const double* Tsurf;     // temperature for the surface loss
  double* slot_surf;
  double scale_surf;
};
// per_item: the launch's workgroups per item, at least every item's nblk
void k_micro_prep(Launch L, const MicroItem* items, int n_items, int per_item);
void k_micro_post(Launch L, const MicroItem* items, int n_items, int per_item);

void k_fine_dirichlet(Launch L, const Geo& gf, const Geo& gc, const Window& w,
                      double T_bottom, const double* Ta, const double* Tb,
                      double wb, double* Tf);

void k_interface_accumulate(Launch L, const Geo& gf, const Window& w,
                            const double* R, double* rho_acc, int init,
                            double bottom_scale, double* ledger_bottom,
                            double* partials);

void k_restrict(Launch L, const Geo& gf, const Geo& gc, const Window& w,
                const double* rho_acc, const double* Rm, double scale,
                double* ext);

// ext = P^T s over every fine node of the window, on every coarse node of
// the closed window (other coarse entries untouched).
void k_restrict_all(Launch L, const Geo& gf, const Geo& gc, const Window& w,
                    const double* s, double* ext);
// The consistent global problem's load from the local solution, on the
// fine window: src = rhocf m_k (Tm - T0)/Dt + kf (K1 Tavg)_k - (rho + Rm)_k/m
// (the last term on interface nodes), Tavg = (Tsum + Tm)/m; Tsum and rho
// may be null (m = 1).
void k_consistent_source(Launch L, const Geo& gf, const Window& w,
                         const double* Tm, const double* T0, const double* Tsum,
                         const double* rho, const double* Rm, int m, double Dt,
                         double kf, double rhocf, double* src);
// Synchronisation-cost probe: `rounds` dependent sweeps over n doubles on
// `blocks` workgroups, one launch per sweep (barrier = 0) or one cooperative
// launch with a grid barrier between sweeps (barrier = 1; blocks must not
// exceed sync_probe_resident()).  ctl: >= 1 KiB of zeroed device memory
// (counter, generation word, timeout flag at ctl[128]).
int sync_probe_resident();
int k_sync_probe(Launch L, int blocks, int rounds, int barrier, double* data,
                 long n, unsigned* ctl);   // returns a hipError_t
// dst = src (assign) or dst += src, over n entries.
void k_accumulate(Launch L, double* dst, const double* src, long n, int assign);

void k_inject(Launch L, const Geo& gf, const Geo& gc, const Window& w,
              const double* Tf, double* Tc);

void k_window_shift(Launch L, const Geo& gf, const Geo& gc, const Window& wn,
                    const Window& wo, const double* Tf_old, const double* Tc,
                    double* Tf_new);

// Sum over nodes of mass(region) * H(T) (+ into slot, or = when assign).
void k_energy(Launch L, const Geo& g, const Region& rg, const MatDev& m,
              const double* T, double* slot, int assign, double* partials,
              double lin = 0.0);

// Sum over nodes with k = 0 of R (scaled, added into slot).
void k_bottom_sum(Launch L, const Geo& g, const double* R, double scale,
                  double* slot, double* partials);

// Heat flow out of the top surface, sum over top nodes of A_i q(T_i) with
// A_i the lumped area of the top faces the region keeps (scaled, added into
// slot).  Nothing is launched when the level has no loss.
void k_surface_sum(Launch L, const Geo& g, const Region& rg, const SurfDev& sf,
                   const double* T, double scale, double* slot,
                   double* partials);

// Interface values: out[2q] = T[idx[q]], out[2q+1] = lam[idx[q]] for the
// n coarse interface nodes listed in idx (padded indices); and the inverse
// scatter lam[idx[q]] = in[q].
void k_gamma_gather(Launch L, const int* idx, int n, const double* T,
                    const double* lam, double* out);
void k_gamma_scatter(Launch L, const int* idx, int n, const double* in,
                     double* lam);

void k_pack(Launch L, const Geo& g, int kind, int elem_bytes, const void* plain,
            void* padded);
void k_unpack(Launch L, const Geo& g, int kind, int elem_bytes,
              const void* padded, void* plain);

// ---- host-side geometry and scan path (tl_host.cpp) -----------------------
struct TrackH {
  double x0, y0, x1, y1, speed, power, radius, absorptivity, depth;
};

// Beam state at time t: returns 0 when off, else 1 and fills the fields.
int laser_at(const TrackH* tr, int n, double t_start, double t, double* xc,
             double* yc, double* P, double* R, double* eta, int* k);
void window_origin(const TrackH* tr, int n, double t_start, double t,
                   double hx, double hy, int nx, int ny, int wx, int wy,
                   int have_current, int cur_I0, int cur_J0, int* I0, int* J0);
double micro_time(double t_start, double dt, int m, long n, int j);
// Boxes of the global volume source for the step [t0, t1]: one per piece of
// track the beam covers, of length v tau along it, width R across it, depth
// d, with density eta P / (R d v (t1 - t0)).  Tracks run along x or y.
// Returns the box count, or -1 when the step covers more than kMaxBoxes
// pieces.
int swept_boxes(const TrackH* tr, int n, double t_start, double t0, double t1,
                BoxSet* out);
void gauss01(int nq, double* x, double* w);

Geo make_geo(int ncx, int ncy, int ncz, double hx, double hy, double hz,
             double x0, double y0);

}  // namespace tl
