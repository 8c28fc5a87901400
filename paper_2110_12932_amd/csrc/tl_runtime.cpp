// Solver runtime and C interface of the two-level thermal library.
//
// Host-side control of the spatiotemporal two-level method (paper Sections 3
// and 4, Algorithm 1): window placement and moves, the coarse predictor, the
// fine micro steps with time-blended Dirichlet data, the two-level
// correction (one composite-grid solve, the Dirichlet-Neumann iteration with
// interface quasi-Newton relaxation, the consistent global formulation, or
// the alternate one), injection, and the FP64 energy ledger.  Each implicit
// step is a frozen-kappa Newton iteration with a backtracking line search
// whose linear systems are solved by Jacobi-preconditioned CG in FP64, or in
// FP32 for the fine level of the mixed-precision path.  All arithmetic on fields runs in the HIP kernels of
// tl_kernels.hip.  Newton, its line search and the CG control run on the
// device (a state machine in the CG-start kernel); the host queues several
// Newton rounds at a time and reads the solvers' states back once per group
// of rounds, and once per iteration of the Dirichlet-Neumann correction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <functional>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tl.h"
#include "../../include/tl_ops.h"
#include "tl_internal.h"
#include "tl_runtime_internal.h"

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

constexpr int kProfPairs = 64;
constexpr int kProlongBatch = 4;   // composite pairs per batch from which the
                                   // prolongation gets a kernel of its own      // event pairs held between host syncs
constexpr int kMaxRoundsPerSync = 8;  // Newton rounds queued between syncs
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Sizes of everything carved out of the caller's workspace.
struct Layout {
  Geo gc, gf;
  size_t off_c[23], off_fd[10], off_fcg[12];
  size_t off_ccg32[12];   // FP32 coarse CG arrays (the mixed path)
  bool ccg32 = false;
  size_t off_fx[2];       // consistent formulation: micro-step field sum,
  bool fx = false;        // load from the local solution (fine)
  size_t off_scal, off_items, off_micro, off_ledger, off_partials, off_tpart,
      off_tpart2, off_gidx, off_gbuf;
  int tstride;   // per-tile partial slots per region (both levels)
  int gamma_cap;
  size_t total;
  int cg_bytes;
};

constexpr int kCoarseArrays = 23;  // Tn Tpred cur trial lam gdw R Fall Fout ext | 12 CG arrays | Hold
constexpr int kFineD = 10;         // state prev cur trial alt R F rho Hold pp
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
  // The mixed-precision path runs the coarse predictor's CG and the
  // composite solve's coarse side in FP32 too; they get arrays of their
  // own, since the stencils rely on zero ghost entries that an FP32 view of
  // the FP64 arrays would not keep.
  L.ccg32 = op.precision == TL_MIXED;
  for (int a = 0; a < kFineCG; ++a) {
    L.off_ccg32[a] = off;
    if (L.ccg32) off += align_up((size_t)L.gc.npad * 4);
  }
  L.fx = op.coupling == TL_COUPLE_CONSISTENT;
  for (int a = 0; a < 2; ++a) {
    L.off_fx[a] = off;
    if (L.fx) off += fbytes;
  }
  L.off_scal = off; off += align_up(2 * sizeof(LevelScalars));
  L.off_items = off; off += align_up(2 * sizeof(SolveItem));
  L.off_micro = off; off += align_up(2 * sizeof(MicroItem));
  L.off_ledger = off; off += align_up(sizeof(LedgerDev));
  L.off_partials = off;
  off += align_up((size_t)kMaxBlocks * kPartRegions * sizeof(double));
  int ntx, nty;
  const int nt = std::max(grid_tiles(L.gc, ntx, nty), grid_tiles(L.gf, ntx, nty));
  L.tstride = (nt + 63) / 64 * 64;
  L.off_tpart = off;
  off += align_up((size_t)L.tstride * kTileRegions * sizeof(double));
  // the coarse side of a composite pair keeps its own tile partials
  L.off_tpart2 = off;
  off += align_up((size_t)L.tstride * kTileRegions * sizeof(double));
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

// Sampled event timing of the fine CG iteration kernel.  Each timed launch
// keeps its round and iteration index; after the host synchronises, only
// launches that did work for some item are counted.
// With profiling on, events at the phase boundaries of every macro step
// give its GPU time per phase: window and coarse loads with the predictor,
// the micro steps, the two-level correction, ledger and commit.
constexpr int kPhases = 4;
struct Profiler {
  int every = 0;
  long count = 0;
  int used = 0;
  hipEvent_t ev[2 * kProfPairs] = {};
  int k[kProfPairs] = {};
  int round[kProfPairs] = {};
  tl_stats* stats = nullptr;
  hipEvent_t pev[kPhases + 1] = {};
  bool phases_pending = false;
};
// the boundary before phase q (q = kPhases: the end of the macro step)
void phase_mark(Profiler* pr, int q, void* stream) {
  if (pr == nullptr || pr->every <= 0 || pr->pev[0] == nullptr) return;
  hip_check(hipEventRecord(pr->pev[q], (hipStream_t)stream), "hipEventRecord(phase)");
  if (q == kPhases) pr->phases_pending = true;
}
// after the host has synchronised with the macro step: add its phase times
void phase_flush(Profiler* pr, double* ms) {
  if (pr == nullptr || !pr->phases_pending) return;
  pr->phases_pending = false;
  for (int q = 0; q < kPhases; ++q) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, pr->pev[q], pr->pev[q + 1]) == hipSuccess && ms)
      ms[q] += t;
  }
}
void phase_events(Profiler* pr, bool create) {
  for (int q = 0; q <= kPhases; ++q) {
    if (create && pr->pev[q] == nullptr)
      hip_check(hipEventCreateWithFlags(&pr->pev[q], hipEventDisableSystemFence),
                "hipEventCreate(phase)");
    if (!create && pr->pev[q] != nullptr) {
      (void)hipEventDestroy(pr->pev[q]);
      pr->pev[q] = nullptr;
    }
  }
}

// Device/pinned tables of one batch context: solve items and scalars.
struct BatchCtx {
  SolveItem* d_items = nullptr;
  SolveItem* h_items = nullptr;
  LevelScalars* d_sc = nullptr;
  LevelScalars* h_sc = nullptr;
  MicroItem* d_micro = nullptr;   // per-simulation micro-step work: two
  MicroItem* h_micro = nullptr;   // halves of micro_cap (before / after)
  int micro_cap = 0;
  int cap = 0;        // solves (scalar sets), simulations
  int item_cap = 0;   // items (a composite pair takes two)
  hipStream_t stream = nullptr;
  Launch L{nullptr};
};

// One implicit step of one level inside a batch: the problem (grid, region,
// step, old field, loads, buffers); the Newton state lives on the device.
template <class R>
struct Job {
  Geo g;
  Region rg;
  MatDev m;
  SurfDev sf{};
  double tau = 0.0;
  const double* Told = nullptr;
  const double* F = nullptr;
  const double* Fext = nullptr;
  double** T = nullptr;   // accepted temperature (swapped with *Tt)
  double** Tt = nullptr;  // trial temperature
  double* Rout = nullptr;
  CGBufs<R>* cg = nullptr;
  double* partials = nullptr;   // generic per-workgroup partials
  double* tpart = nullptr;      // per-tile partials of the Newton/CG kernels
  double* Hold = nullptr;       // H(T_old), formed in the first round
  int tstride = 0;
  int* last_cg = nullptr;   // most CG iterations the level's last solve needed
  int64_t* n_newton = nullptr;
  int64_t* n_cg = nullptr;
  int64_t* n_newton_x = nullptr;   // also counted here when set
  int64_t* n_cg_x = nullptr;
  tl_stats* stats = nullptr;   // line-search count; op bytes if `fine`
  bool fine = false;
  double tol = 0.0, rtol2 = 0.0;
  int newton_max = 0, cg_max = 0;
  const char* what = "";
  bool failed = false;
  bool finished = false;
  std::string err;
  int rounds_hint = 2;   // rounds to queue before the next host sync
  // composite pairs: the caller's part of the coupling (window, row scale;
  // on the coarse side the gather targets and interface list); the solver
  // fills in the partner's arrays
  Couple cpl{};
};

// Count the timed launches that did work: round r's launch k worked when
// some item ran more than k CG iterations in that round.
void flush_profile(Profiler* pr, int r0, const std::vector<int>& iters) {
  for (int q = 0; q < pr->used; ++q) {
    const int r = pr->round[q] - r0;
    if (r < 0 || r >= (int)iters.size() || pr->k[q] >= iters[r]) continue;
    float ms = 0.0f;
    hip_check(hipEventElapsedTime(&ms, pr->ev[2 * q], pr->ev[2 * q + 1]),
              "hipEventElapsedTime");
    pr->stats->fine_op_timed_ms += ms;
    pr->stats->fine_op_timed += 1;
  }
  pr->used = 0;
}

// Rounds a running solve is expected to need: two while the Newton steps
// are irregular (start, line search), else the count at which the observed
// linear rate of the accepted steps brings them within tol.
int predict_rounds(const NewtonState& st, double tol) {
  if (st.first || st.n_newton < 2 || st.h > 0 || st.dmax_prev <= 0.0 ||
      st.dmax_last <= tol)
    return 2;
  const double rate = st.dmax_last / st.dmax_prev;
  if (!(rate > 0.0) || rate >= 0.5) return 2;
  const double q = std::ceil(std::log(tol / st.dmax_last) / std::log(rate));
  return std::max(1, std::min(kMaxRoundsPerSync, (int)q));
}

// Batched implicit steps: frozen-kappa Newton with backtracking on
// |R_free|_2 for every job, linear systems by Jacobi-PCG in precision R.
// A Newton round is three kinds of launch over all unfinished jobs at once:
// the residual at each job's trial, the device-side Newton state machine
// with the CG start, and the CG iterations for the next direction (they
// return at once for a job whose trial was rejected, whose Newton iteration
// converged or failed, or whose CG converged or used its budget).  The host
// queues several rounds without synchronising -- as many as the slowest job
// is predicted to need -- then reads every job's state with one copy.  On
// return each job's *T holds its solution and Rout the residual there.
//
// With `paired`, jobs come as (fine, coarse) composite pairs (jobs[2u],
// jobs[2u+1]) that share one Newton/CG state: every launch of a round runs
// over the fine sides, then the gather of the fine interface rows, then the
// coarse sides (see Couple).  Counts and the CG budget go to the fine job.
template <class R>
void fill_item(SolveItem& it, const Job<R>& j) {
  it.g = j.g;
  it.rg = j.rg;
  it.m = j.m;
  it.sf = j.sf;
  it.tau = j.tau;
  it.tol = j.tol;
  it.rtol2 = j.rtol2;
  it.newton_max = j.newton_max;
  it.cg_max = j.cg_max;
  it.ntiles = grid_tiles(j.g, it.ntx, it.nty);
  it.tstride = j.tstride;
  it.Tb[0] = *j.T;
  it.Tb[1] = *j.Tt;
  it.Told = j.Told;
  it.Hold = j.Hold;
  it.F = j.F;
  it.Fext = j.Fext;
  it.R = j.Rout;
  it.xb[0] = j.cg->x[0];
  it.xb[1] = j.cg->x[1];
  it.kap = j.cg->kap;
  it.d = j.cg->d;
  it.dinv = j.cg->dinv;
  it.r[0] = j.cg->r[0];
  it.r[1] = j.cg->r[1];
  it.w[0] = j.cg->w[0];
  it.w[1] = j.cg->w[1];
  it.s[0] = j.cg->s[0];
  it.s[1] = j.cg->s[1];
  it.p = j.cg->p;
  it.tpart = j.tpart;
  it.cp = j.cpl;
  it.cp.ntA = it.ntiles;
  it.cp.tsA = j.tstride;
  it.cp.tpA = j.tpart;
  it.cp.ntB = 0;
  it.cp.tsB = 0;
  it.cp.tpB = nullptr;
}

// The pair's cross references: the fine side reads the coarse arrays, the
// coarse side gathers from the fine ones; both sum fine then coarse tiles.
template <class R>
void link_pair(SolveItem& f, SolveItem& c, const Job<R>& fj, const Job<R>& cj) {
  f.cp.go = cj.g;
  f.cp.oT[0] = *cj.T;
  f.cp.oT[1] = *cj.Tt;
  f.cp.ox[0] = cj.cg->x[0];
  f.cp.ox[1] = cj.cg->x[1];
  f.cp.odinv = cj.cg->dinv;
  for (int b = 0; b < 2; ++b) {
    f.cp.orr[b] = cj.cg->r[b];
    f.cp.ow[b] = cj.cg->w[b];
    f.cp.os[b] = cj.cg->s[b];
  }
  c.cp.go = fj.g;
  c.cp.fR = fj.Rout;
  c.cp.fdiag = fj.cg->dinv;
  c.cp.fw[0] = fj.cg->w[0];
  c.cp.fw[1] = fj.cg->w[1];
  f.cp.ntB = c.cp.ntA;
  f.cp.tsB = c.cp.tsA;
  f.cp.tpB = c.cp.tpA;
  c.cp.ntB = c.cp.ntA;
  c.cp.tsB = c.cp.tsA;
  c.cp.tpB = c.cp.tpA;
  c.cp.ntA = f.cp.ntA;
  c.cp.tsA = f.cp.tsA;
  c.cp.tpA = f.cp.tpA;
}

template <class R>
void solve_batch(BatchCtx& B, std::vector<Job<R>*>& jobs, Profiler* prof,
                 bool paired = false) {
  const int nj = (int)jobs.size();
  const int nu = paired ? nj / 2 : nj;   // solves: jobs, or pairs
  if (nu > B.cap || nj > B.item_cap)
    throw DevErr{"batch larger than its context"};
  if (nj == 0) return;
  for (int q = 0; q < nj; ++q) {
    jobs[q]->finished = false;
    jobs[q]->failed = false;
    jobs[q]->rounds_hint = 2;
  }
  for (int u = 0; u < nu; ++u) {
    Job<R>& j = *jobs[paired ? 2 * u : u];
    LevelScalars& h = B.h_sc[u];
    std::memset(&h, 0, sizeof(LevelScalars));
    NewtonState& st = h.ns[0];
    st.first = 1;
    st.status = kRunning;
    // CG budget: 1 more than the most the level's last solve needed
    st.budget = std::min(j.cg_max, std::max(3, *j.last_cg + 1));
  }
  hip_check(hipMemcpyAsync(B.d_sc, B.h_sc, sizeof(LevelScalars) * nu,
                           hipMemcpyHostToDevice, B.stream),
            "hipMemcpyAsync(scalars)");
  std::vector<int> act, built, round_iters;
  int round = 0, tiles_a = 0, tiles_c = 0, stacks_a = 0, stacks_c = 0;
  int per_p = 0, max_gamma = 0;
  for (;;) {
    act.clear();
    for (int u = 0; u < nu; ++u)
      if (!jobs[paired ? 2 * u : u]->finished) act.push_back(u);
    if (act.empty()) return;
    const int na = (int)act.size();
    if (act != built) {
      int most = 1, most_c = 1;
      stacks_a = stacks_c = 1;
      max_gamma = 0;
      for (int u : act) {
        int ntx, nty;
        const Geo& ga = jobs[paired ? 2 * u : u]->g;
        most = std::max(most, grid_tiles(ga, ntx, nty));
        stacks_a = std::max(stacks_a, cg_stacks(ga));
        if (paired) {
          const Geo& gc = jobs[2 * u + 1]->g;
          most_c = std::max(most_c, grid_tiles(gc, ntx, nty));
          stacks_c = std::max(stacks_c, cg_stacks(gc));
          max_gamma = std::max(max_gamma, jobs[2 * u + 1]->cpl.ngamma);
        }
      }
      tiles_a = most;     // tiles of the largest item: each kernel sizes
      tiles_c = most_c;   // its grid from its own residency
      // the prolongation: about four interface nodes per thread
      long most_face = 1;
      if (paired)
        for (int u : act) {
          const Geo& g = jobs[2 * u]->g;
          most_face = std::max(most_face, 2l * g.ny * g.nz + 2l * g.nx * g.nz +
                                              (long)g.nx * g.ny);
        }
      per_p = (int)std::max(1l, std::min(256l, most_face / (4 * kBlock) + 1));
      for (int a = 0; a < na; ++a) {
        const int u = act[a];
        if (!paired) {
          fill_item(B.h_items[a], *jobs[u]);
          B.h_items[a].sc = B.d_sc + u;
        } else {
          SolveItem& f = B.h_items[a];
          SolveItem& c = B.h_items[na + a];
          fill_item(f, *jobs[2 * u]);
          fill_item(c, *jobs[2 * u + 1]);
          link_pair(f, c, *jobs[2 * u], *jobs[2 * u + 1]);
          f.sc = c.sc = B.d_sc + u;
        }
      }
      hip_check(hipMemcpyAsync(B.d_items, B.h_items,
                               sizeof(SolveItem) * na * (paired ? 2 : 1),
                               hipMemcpyHostToDevice, B.stream),
                "hipMemcpyAsync(items)");
      built = act;
    }
    // CG launches per round: the largest budget
    int n_launch = 0, n_rounds = 1;
    for (int u : act) {
      n_launch = std::max(n_launch, B.h_sc[u].ns[round & 1].budget);
      n_rounds = std::max(n_rounds, jobs[paired ? 2 * u : u]->rounds_hint);
    }
    const int r0 = round;
    // composite pairs: interface values prolonged by a kernel of their own
    // in large batches (cheaper fine kernels), inside the fine kernels for
    // a few simulations (fewer launches); the values are the same
    const bool prolong = paired && na >= kProlongBatch;
    const int fside = prolong ? kFineSideP : kFineSide;
    const SolveItem* fi = B.d_items;
    const SolveItem* ci = B.d_items + na;
    for (int rr = 0; rr < n_rounds; ++rr, ++round) {
      if (!paired) {
        k_residual_batched<R>(B.L, fi, na, tiles_a, round);
        k_cg_start_batched<R>(B.L, fi, na, tiles_a, stacks_a, round);
      } else {
        if (prolong) k_couple_prolong<R>(B.L, fi, na, per_p, round, 0, 0);
        k_residual_pair<R>(B.L, fi, na, tiles_a, round, fside);
        k_couple_gather<R>(B.L, ci, na, max_gamma, round, 0, 0);
        k_residual_pair<R>(B.L, ci, na, tiles_c, round, kCoarseSide);
        if (prolong) k_couple_prolong<R>(B.L, fi, na, per_p, round, 1, 0);
        k_cg_start_pair<R>(B.L, fi, na, tiles_a, stacks_a, round, fside);
        k_couple_gather<R>(B.L, ci, na, max_gamma, round, 1, 0);
        k_cg_start_pair<R>(B.L, ci, na, tiles_c, stacks_c, round,
                           kCoarseSide);
      }
      for (int k = 0; k < n_launch; ++k) {
        // sampled event timing covers the plain CG kernel (not the pairs'),
        // iterations after the first (those read and write all 13 arrays)
        const bool timed = !paired && k > 0 && prof != nullptr &&
                           prof->every > 0 &&
                           (prof->count++ % prof->every) == 0 &&
                           prof->used < kProfPairs;
        void* e0 = timed ? (void*)prof->ev[2 * prof->used] : nullptr;
        void* e1 = timed ? (void*)prof->ev[2 * prof->used + 1] : nullptr;
        if (!paired) {
          k_cg_iter_batched<R>(B.L, fi, na, tiles_a, stacks_a, round, k, e0,
                               e1);
        } else {
          if (prolong) k_couple_prolong<R>(B.L, fi, na, per_p, round, 2, k);
          k_cg_iter_pair<R>(B.L, fi, na, tiles_a, stacks_a, round, k, fside,
                            nullptr, nullptr);
          k_couple_gather<R>(B.L, ci, na, max_gamma, round, 2, k);
          k_cg_iter_pair<R>(B.L, ci, na, tiles_c, stacks_c, round, k,
                            kCoarseSide, nullptr, nullptr);
        }
        if (timed) {
          prof->k[prof->used] = k;
          prof->round[prof->used] = round;
          ++prof->used;
        }
      }
    }
    hip_check(hipGetLastError(), "kernel launch");
    hip_check(hipMemcpyAsync(B.h_sc, B.d_sc, sizeof(LevelScalars) * nu,
                             hipMemcpyDeviceToHost, B.stream),
              "hipMemcpyAsync(scalars)");
    hip_check(hipStreamSynchronize(B.stream), "hipStreamSynchronize");
    if (prof != nullptr && prof->used > 0) {
      // CG iterations per queued round, most over the jobs: rounds before
      // the last from the log, the last from its CG scalars
      round_iters.assign(n_rounds, 0);
      for (int u : act) {
        const LevelScalars& h = B.h_sc[u];
        for (int rr = 0; rr < n_rounds; ++rr) {
          const int r = r0 + rr;
          const int n = r + 1 < round ? h.cg_log[r % kRoundLog]
                                      : h.cg[r & 1].iters;
          round_iters[rr] = std::max(round_iters[rr], n);
        }
      }
      flush_profile(prof, r0, round_iters);
    }
    for (int u : act) {
      Job<R>& j = *jobs[paired ? 2 * u : u];
      Job<R>* partner = paired ? jobs[2 * u + 1] : nullptr;
      const NewtonState& st = B.h_sc[u].ns[round & 1];
      if (st.status == kRunning) {
        j.rounds_hint = predict_rounds(st, j.tol);
        continue;
      }
      j.finished = true;
      *j.n_newton += st.n_newton;
      *j.n_cg += st.n_cg;
      if (j.n_newton_x) *j.n_newton_x += st.n_newton;
      if (j.n_cg_x) *j.n_cg_x += st.n_cg;
      j.stats->line_search_halvings += st.n_halvings;
      if (j.fine) {
        j.stats->fine_op_bytes += 13.0 * sizeof(R) * j.g.nreal * st.n_cg;
        j.stats->fine_op_applies += st.n_cg;
      }
      if (st.cg_need > 0) *j.last_cg = st.cg_need;
      if (st.cur == 1) {
        std::swap(*j.T, *j.Tt);
        if (partner) std::swap(*partner->T, *partner->Tt);
      }
      if (partner) partner->finished = true;
      if (st.status == kConverged) continue;
      j.failed = true;
      j.err = std::string(j.what);
      switch (st.status) {
        case kFailNonFinite:
          j.err += ": non-finite residual or Newton update";
          break;
        case kFailBreakdown:
          j.err += ": CG breakdown (non-positive or non-finite curvature)";
          break;
        default:
          j.err += " Newton did not converge within newton_max iterations";
      }
      if (partner) {
        partner->failed = true;
        partner->err = j.err;
      }
    }
  }
}

// Interface quasi-Newton (IQN-ILS) for the two-level iteration: lambda is
// the coarse interface trace, g(lambda) the coarse solution there after the
// fine and outside solves, r = g - lambda.  Secant pairs (differences of r
// and of g between iterations) approximate the inverse Jacobian of r by
// least squares.  The pairs are kept across macro steps while the interface
// keeps its nodes (the problem changes little from one step to the next),
// so a step's first update is already a quasi-Newton one; the oldest pairs
// drop out beyond kMaxCols, and a window move or a restored state clears
// them.
struct Interface {
  std::vector<std::vector<double>> V, W;
  std::vector<double> r_prev, g_prev;
  bool has_prev = false;
  static constexpr int kMaxCols = 24;

  void clear() {
    V.clear();
    W.clear();
    has_prev = false;
  }
  // a new macro step: the last iterate of the previous step is no partner
  // for a new secant pair
  void begin_step() { has_prev = false; }

  void update(const std::vector<double>& lam, const std::vector<double>& g,
              double theta0, bool fixed, std::vector<double>& next) {
    const size_t n = lam.size();
    std::vector<double> r(n);
    for (size_t q = 0; q < n; ++q) r[q] = g[q] - lam[q];
    next.assign(n, 0.0);
    if (!fixed && has_prev) {
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
    }
    if (fixed || V.empty() || (V[0].size() != n)) {
      if (!V.empty() && V[0].size() != n) clear();
      for (size_t q = 0; q < n; ++q) next[q] = lam[q] + theta0 * r[q];
    } else {
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

}  // namespace

struct tl_sim {
  tl_mesh mesh;
  tl_material mat_in;
  tl_options opts;
  MatDev mat;
  MatDev mat_global;   // the coarse level's law (no latent heat with the
                       // alternate global formulation)
  std::vector<TrackH> tracks;
  double t_start;
  Interface iqn;   // two-level secant pairs, kept across macro steps
  Layout lay;
  Geo gc, gf;
  Window win;
  hipStream_t stream;
  Launch L;
  char* ws;
  // coarse fields
  // lam: interface values of the Dirichlet-Neumann iteration, or the
  // gathered fine residual rows of a composite solve; gdw: the gathered
  // fine diagonal and J u rows of a composite solve
  double *Tn, *Tpred, *ccur, *ctrial, *lam, *gdw, *cR, *Fall, *Fout, *ext;
  CGBufs<double> ccg;
  CGBufs<float> ccg32;   // coarse CG arrays of the mixed path
  // fine fields
  // fpp: the micro step before fprev (extrapolated initial guesses)
  double *fstate, *fprev, *fcur, *ftrial, *falt, *fR, *fF, *rho, *fpp;
  double *cHold, *fHold;   // H(T_old) of the level's current solve
  // consistent formulation: sum of the micro-step fields of the macro step,
  // the load from the local solution, and the global problem's constant
  // coefficients inside the window
  double *fsum = nullptr, *fsrc = nullptr;
  double kf = 0.0, rhocf = 0.0;
  CGBufs<double> fcg64;
  CGBufs<float> fcg32;
  LevelScalars *sc_c, *sc_f;
  LedgerDev* led;
  double* partials;
  double* tpart;
  double* tpart2;       // tile partials of a composite pair's coarse side
  int* gidx;            // padded indices of the coarse interface nodes
  double* gbuf;         // interface gather/scatter staging
  int n_gamma;
  // host side: pinned (hipHostMalloc), or plain heap memory for a handle
  // of tl_create_static, which calls no HIP allocator
  LevelScalars* h_sc;
  LedgerDev* h_led;
  double* h_gbuf;       // 2 * gamma_cap doubles
  bool pinned_host = true;
  int static_dev = -1;  // device whose static workspace the handle holds
  tl_ledger ledger;     // committed ledger
  tl_stats stats;
  long n_macro;
  double theta0;
  int last_cg_f, last_cg_c, last_cg_x;   // fine, coarse, composite solves
  Profiler prof;   // sampled event timing of the fine CG kernel
  BatchCtx batch;  // one-item batches for this simulation's solves
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
// the consistent global problem: every coarse element, the window's with
// the global problem's own coefficients
Region region_fict(const tl_sim* s) {
  Region rg = region_outside(s);
  rg.mode = kFictitious;
  rg.kf = s->kf;
  rg.rhocf = s->rhocf;
  return rg;
}
bool consistent(const tl_sim* s) {
  return s->opts.coupling == TL_COUPLE_CONSISTENT;
}
// top-surface loss: convection and radiation on the fine level, convection
// only on the coarse one (paper Section 2)
SurfDev surf_fine(const tl_sim* s) {
  return SurfDev{s->mat_in.h_conv, kSigmaSB * s->mat_in.emissivity,
                 s->mat_in.T_amb};
}
SurfDev surf_coarse(const tl_sim* s) {
  return SurfDev{s->mat_in.h_conv, 0.0, s->mat_in.T_amb};
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

// The coarse interface nodes of window w (padded indices on the coarse
// grid gc), in the order of the interface vectors.
std::vector<int> interface_nodes(const Geo& gc, const Window& w) {
  std::vector<int> idx;
  for (int k = w.K0; k <= w.K0 + w.wz; ++k)
    for (int j = w.J0; j <= w.J0 + w.wy; ++j)
      for (int i = w.I0; i <= w.I0 + w.wx; ++i) {
        const bool g = ((w.faces & kFx0) && i == w.I0) ||
                       ((w.faces & kFx1) && i == w.I0 + w.wx) ||
                       ((w.faces & kFy0) && j == w.J0) ||
                       ((w.faces & kFy1) && j == w.J0 + w.wy) ||
                       ((w.faces & kFz0) && k == w.K0);
        if (g) idx.push_back((k + 1) * gc.pxy + (j + 1) * gc.px + (i + 1));
      }
  return idx;
}

void set_interface(tl_sim* s) {
  s->iqn.clear();   // secant pairs belong to the previous interface
  const std::vector<int> idx = interface_nodes(s->gc, s->win);
  s->n_gamma = (int)idx.size();
  if (!idx.empty())
    hip_check(hipMemcpy(s->gidx, idx.data(), idx.size() * sizeof(int),
                        hipMemcpyHostToDevice),
              "hipMemcpy(interface indices)");
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

bool alternate(const tl_sim* s) {
  return s->opts.coupling == TL_COUPLE_ALTERNATE;
}

// The volume model's local source at micro time j of macro step n.
VolSpot vol_spot(const tl_sim* s, long n, int j) {
  VolSpot v{};
  const double t =
      micro_time(s->t_start, s->opts.dt_coarse, s->opts.m_time, n, j);
  double xc, yc, P, Rr, eta;
  int k;
  if (!laser_at(s->tracks.data(), (int)s->tracks.size(), s->t_start, t, &xc,
                &yc, &P, &Rr, &eta, &k))
    return v;
  const double d = s->tracks[k].depth;
  v.xc = xc;
  v.yc = yc;
  v.amp = 6.0 * std::sqrt(3.0) * eta * P / (std::pow(M_PI, 1.5) * Rr * Rr * d);
  v.a3 = 3.0 / (Rr * Rr);
  v.az = 3.0 / (d * d);
  v.on = 1;
  return v;
}

// Fine load at micro time j of macro step n into fF, booked as absorbed
// over dt: the surface Gaussian, or the volume model's Gaussian.
void fine_load(tl_sim* s, long n, int j, double dt) {
  // the alternate formulation's ledger is the global problem's
  double* slot = alternate(s) ? nullptr : &s->led->absorbed;
  if (s->opts.source == TL_SOURCE_VOLUME) {
    k_volume_load(s->L, s->gf, vol_spot(s, n, j), s->fF, dt, slot,
                  s->partials);
  } else {
    SpotSet sp = make_spots(s, n, j, j, 1.0);
    k_laser_load(s->L, s->gf, sp, 0, 0, 0, 0, s->fF, dt, slot, s->partials);
  }
}

// Coarse loads of macro step n: Fall over all elements (the predictor) and
// Fout outside the window (the correction, booked as absorbed over Dt) --
// the time average of the surface loads at the micro times, or the volume
// model's swept boxes.  Returns false when the step covers more track
// pieces than a box set holds.
bool coarse_loads(tl_sim* s, long n, int m, double Dt) {
  const Window& w = s->win;
  // the alternate formulation books the global load itself
  const bool alt = alternate(s);
  if (s->opts.source == TL_SOURCE_VOLUME) {
    BoxSet bs;
    const double t0 = micro_time(s->t_start, Dt, m, n, 0);
    const double t1 = micro_time(s->t_start, Dt, m, n, m);
    if (swept_boxes(s->tracks.data(), (int)s->tracks.size(), s->t_start, t0,
                    t1, &bs) < 0)
      return false;
    k_box_load(s->L, s->gc, region_all(), bs, s->Fall, alt ? Dt : 0.0,
               alt ? &s->led->absorbed : nullptr, s->partials);
    if (!alt)
      k_box_load(s->L, s->gc, region_outside(s), bs, s->Fout, Dt,
                 &s->led->absorbed, s->partials);
    return true;
  }
  SpotSet avg = make_spots(s, n, 1, m, 1.0 / m);
  k_laser_load(s->L, s->gc, avg, 0, 0, 0, 0, s->Fall, alt ? Dt : 0.0,
               alt ? &s->led->absorbed : nullptr, s->partials);
  if (!alt)
    k_laser_load(s->L, s->gc, avg, w.I0, w.I0 + w.wx, w.J0, w.J0 + w.wy,
                 s->Fout, Dt, &s->led->absorbed, s->partials);
  return true;
}

void energy_now(tl_sim* s, double* slot) {
  if (alternate(s)) {   // the global problem's own energy
    k_energy(s->L, s->gc, region_all(), s->mat_global, s->Tn, slot, 1,
             s->partials);
    return;
  }
  if (consistent(s)) {
    // plus the energy the global coefficients hold inside the window beyond
    // the local field's: rhoc_f (sum m_in T+ - sum m_k T-)
    k_energy(s->L, s->gc, region_fict(s), s->mat, s->Tn, slot, 1, s->partials);
    k_energy(s->L, s->gf, region_window(s), s->mat, s->fstate, slot, 0,
             s->partials, -s->rhocf);
    return;
  }
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
  s->h_led->surface = s->ledger.surface;
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

// Per-simulation state of one macro step run in lockstep with others.
struct StepState {
  tl_sim* s = nullptr;
  bool failed = false;
  std::string err;
  int m = 1;
  double Dt = 0.0, dt = 0.0;
  long n = 0;
  bool dn_done = false;
  int it = 0;
  std::vector<double> lam_v, lt_v, next;
};

void fail_step(StepState& st, const std::string& msg) {
  if (!st.failed) {
    st.failed = true;
    st.err = "macro step " + std::to_string(st.n) + ": " + msg;
  }
}

template <class R>
Job<R> make_job(tl_sim* s, bool fine, const Region& rg, double tau,
                const double* Told, const double* F, const double* Fext) {
  Job<R> j;
  j.g = fine ? s->gf : s->gc;
  j.rg = rg;
  j.m = fine ? s->mat : s->mat_global;
  j.sf = fine ? surf_fine(s) : surf_coarse(s);
  j.tau = tau;
  j.Told = Told;
  j.F = F;
  j.Fext = Fext;
  j.T = fine ? &s->fcur : &s->ccur;
  j.Tt = fine ? &s->ftrial : &s->ctrial;
  j.Rout = fine ? s->fR : s->cR;
  j.partials = s->partials;
  j.tpart = s->tpart;
  j.Hold = fine ? s->fHold : s->cHold;
  j.tstride = s->lay.tstride;
  j.last_cg = fine ? &s->last_cg_f : &s->last_cg_c;
  j.n_newton = fine ? &s->stats.newton_fine : &s->stats.newton_coarse;
  j.n_cg = fine ? &s->stats.cg_fine : &s->stats.cg_coarse;
  j.stats = &s->stats;
  j.fine = fine;
  j.tol = s->opts.newton_tol;
  const double rtol =
      sizeof(R) == 4 ? std::max(s->opts.cg_rtol, 1e-5) : s->opts.cg_rtol;
  j.rtol2 = rtol * rtol;
  j.newton_max = s->opts.newton_max;
  j.cg_max = s->opts.cg_max;
  j.what = fine ? "fine" : "coarse";
  return j;
}

template <class R>
CGBufs<R>& cg_of(tl_sim* s, bool fine);
template <>
CGBufs<double>& cg_of<double>(tl_sim* s, bool fine) {
  return fine ? s->fcg64 : s->ccg;
}
template <>
CGBufs<float>& cg_of<float>(tl_sim* s, bool fine) {
  return fine ? s->fcg32 : s->ccg32;
}

// Solve one fine (fine = true) or coarse step for every listed simulation
// in batched launches; `setup` supplies region, step, old field, loads.
// Simulations whose solve fails are marked failed.
template <class R>
void batch_solve(BatchCtx& B, std::vector<StepState*>& list, bool fine,
                 const std::function<Job<R>(StepState&)>& setup,
                 Profiler* prof) {
  std::vector<Job<R>> jobs;
  jobs.reserve(list.size());
  for (StepState* st : list) {
    jobs.push_back(setup(*st));
    jobs.back().cg = &cg_of<R>(st->s, fine);
  }
  std::vector<Job<R>*> ptrs;
  for (Job<R>& j : jobs) ptrs.push_back(&j);
  if (!ptrs.empty()) solve_batch<R>(B, ptrs, prof);
  for (size_t q = 0; q < list.size(); ++q) {
    tl_sim* s = list[q]->s;
    if (jobs[q].failed) fail_step(*list[q], jobs[q].err);
    if (fine)
      ++s->stats.fine_solves;
    else
      ++s->stats.coarse_solves;
  }
}

template <class R>
CGBufs<R>& coarse_cg(tl_sim* s);
template <>
CGBufs<double>& coarse_cg<double>(tl_sim* s) { return s->ccg; }
template <>
CGBufs<float>& coarse_cg<float>(tl_sim* s) { return s->ccg32; }

// Composite-grid two-level corrections of the listed simulations (one
// precision) in batched launches: per simulation a fine job on the window
// (rows scaled by 1/m, the interface values slaved to the coarse ones) and a
// coarse job outside the window interior loaded by the reactions of micro
// steps 1..m-1 (ext), sharing one Newton/CG state.
template <class R>
void batch_composite(BatchCtx& B, std::vector<StepState*>& list,
                     Profiler* prof) {
  if (list.empty()) return;
  std::vector<Job<R>> jobs;
  jobs.reserve(2 * list.size());
  for (StepState* st : list) {
    tl_sim* s = st->s;
    Job<R> f = make_job<R>(s, true, region_window(s), st->dt, s->fprev, s->fF,
                           nullptr);
    f.cg = &cg_of<R>(s, true);
    f.last_cg = &s->last_cg_x;
    f.what = "composite two-level correction";
    f.n_newton_x = &s->stats.newton_corr;
    f.n_cg_x = &s->stats.cg_corr;
    f.cpl.w = s->win;
    f.cpl.rscale = 1.0 / st->m;
    Job<R> c = make_job<R>(s, false, region_outside(s), st->Dt, s->Tn, s->Fout,
                           s->ext);
    c.cg = &coarse_cg<R>(s);
    c.tpart = s->tpart2;
    c.cpl.w = s->win;
    c.cpl.rscale = 1.0;
    c.cpl.gR = s->lam;
    c.cpl.gDW = s->gdw;
    c.cpl.gidx = s->gidx;
    c.cpl.ngamma = s->n_gamma;
    jobs.push_back(f);
    jobs.push_back(c);
  }
  std::vector<Job<R>*> ptrs;
  for (Job<R>& j : jobs) ptrs.push_back(&j);
  solve_batch<R>(B, ptrs, prof, true);
  for (size_t q = 0; q < list.size(); ++q) {
    if (jobs[2 * q].failed) fail_step(*list[q], jobs[2 * q].err);
    ++list[q]->s->stats.fine_solves;
  }
}

// Fine solves of the listed simulations, grouped by the precision of their
// linear solves.
// `corr`: solves of the two-level correction (also counted there).
void batch_fine(BatchCtx& B, std::vector<StepState*>& list,
                const std::function<void(StepState&, Region&, double&,
                                         const double*&)>& told,
                Profiler* prof, bool corr = false) {
  std::vector<StepState*> f64, f32;
  for (StepState* st : list)
    (st->s->opts.precision == TL_MIXED ? f32 : f64).push_back(st);
  auto mk = [&](StepState& st, auto j) {
    if (corr) {
      j.n_newton_x = &st.s->stats.newton_corr;
      j.n_cg_x = &st.s->stats.cg_corr;
    }
    return j;
  };
  auto mk64 = [&](StepState& st) {
    Region rg;
    double tau;
    const double* Told;
    told(st, rg, tau, Told);
    return mk(st, make_job<double>(st.s, true, rg, tau, Told, st.s->fF, nullptr));
  };
  auto mk32 = [&](StepState& st) {
    Region rg;
    double tau;
    const double* Told;
    told(st, rg, tau, Told);
    return mk(st, make_job<float>(st.s, true, rg, tau, Told, st.s->fF, nullptr));
  };
  batch_solve<double>(B, f64, true, mk64, prof);
  batch_solve<float>(B, f32, true, mk32, prof);
}

std::vector<StepState*> live(std::vector<StepState>& steps) {
  std::vector<StepState*> out;
  for (StepState& st : steps)
    if (!st.failed) out.push_back(&st);
  return out;
}

// The micro-step work of one simulation (see MicroItem) before the solve
// of micro step j ...
void micro_prep_item(const StepState& st, int j, MicroItem& mi) {
  tl_sim* s = st.s;
  std::memset(&mi, 0, sizeof(mi));
  mi.nblk = micro_blocks(s->gf);
  mi.gf = s->gf;
  mi.gc = s->gc;
  mi.w = s->win;
  mi.T_bottom = s->mat_in.T_bottom;
  mi.wb = (double)j / st.m;
  mi.Ta = s->Tn;
  mi.Tb = s->Tpred;
  mi.prev = s->fprev;
  mi.pp = j >= 2 ? s->fpp : nullptr;
  mi.cur = s->fcur;
  mi.source = s->opts.source == TL_SOURCE_VOLUME ? 1 : 0;
  if (mi.source == 1) {
    mi.vs = vol_spot(s, st.n, j);
  } else {
    const SpotSet sp = make_spots(s, st.n, j, j, 1.0);
    mi.nq = sp.nq;
    for (int q = 0; q < 4; ++q) {
      mi.gx[q] = sp.gx[q];
      mi.gw[q] = sp.gw[q];
    }
    if (sp.n > 0) mi.spot = sp.s[0];   // weight 0 (zeroed) when off
  }
  mi.F = s->fF;
  mi.part = s->partials;
  // the alternate formulation's ledger is the global problem's
  mi.slot_abs = alternate(s) ? nullptr : &s->led->absorbed;
  mi.scale_abs = st.dt;
}

// ... and after it: reactions on the interface into rho, the bottom and
// top-surface heat flows of the solution.
void micro_post_item(const StepState& st, int j, MicroItem& mi) {
  tl_sim* s = st.s;
  const bool alt = alternate(s);
  std::memset(&mi, 0, sizeof(mi));
  mi.nblk = micro_blocks(s->gf);
  mi.gf = s->gf;
  mi.gc = s->gc;
  mi.w = s->win;
  mi.part = s->partials;
  mi.R = s->fR;
  mi.rho = alt ? nullptr : s->rho;
  mi.rho_init = j == 1 ? 1 : 0;
  mi.slot_bottom = alt ? nullptr : &s->led->bottom;
  mi.scale_bottom = -st.dt;
  mi.rgw = region_window(s);
  mi.sf = surf_fine(s);
  mi.Tsurf = s->fcur;
  mi.slot_surf = alt ? nullptr : &s->led->surface;
  mi.scale_surf = st.dt;
}

// One macro step of Algorithm 1 for several simulations in lockstep: the
// per-simulation work (window, loads, Dirichlet data, transfers, ledger) is
// queued simulation by simulation, and every fine or coarse implicit step of
// a phase is one batched Newton/CG solve over all simulations.  The
// two-level iteration drops each simulation once its interface has
// converged.  A simulation that fails is marked and left out of the rest of
// the step; the caller restores its state.
void macro_step_batch(std::vector<StepState>& steps, BatchCtx& B,
                      Profiler* prof) {
  for (StepState& st : steps) {
    tl_sim* s = st.s;
    st.m = s->opts.m_time;
    st.Dt = s->opts.dt_coarse;
    st.dt = st.Dt / st.m;
    st.n = s->n_macro;
    st.dn_done = false;
    s->iqn.begin_step();
    st.it = 0;
  }
  phase_mark(prof, 0, B.stream);
  // 1. window placement for the beam at t_{n+1}; 2. coarse loads
  for (StepState& st : steps) {
    tl_sim* s = st.s;
    const Launch L = s->L;
    LedgerDev* led = s->led;
    int I0, J0;
    window_origin(s->tracks.data(), (int)s->tracks.size(), s->t_start,
                  micro_time(s->t_start, st.Dt, st.m, st.n + 1, 0), s->gc.hx,
                  s->gc.hy, s->mesh.nx, s->mesh.ny, s->mesh.win_nx,
                  s->mesh.win_ny, 1, s->win.I0, s->win.J0, &I0, &J0);
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
    if (!coarse_loads(s, st.n, st.m, st.Dt))
      fail_step(st, "more track pieces in one macro step than the volume "
                    "source holds");
    k_copy(L, s->ccur, s->Tn, s->gc.npad);
  }
  // coarse predictor over the whole plate: FP64 residual and Newton, the
  // CG in the path's precision
  {
    std::vector<StepState*> p64, p32;
    for (StepState* st : live(steps))
      (st->s->opts.precision == TL_MIXED ? p32 : p64).push_back(st);
    batch_solve<double>(
        B, p64, false,
        [](StepState& st) {
          return make_job<double>(st.s, false, region_all(), st.Dt, st.s->Tn,
                                  st.s->Fall, nullptr);
        },
        nullptr);
    batch_solve<float>(
        B, p32, false,
        [](StepState& st) {
          return make_job<float>(st.s, false, region_all(), st.Dt, st.s->Tn,
                                 st.s->Fall, nullptr);
        },
        nullptr);
  }
  for (StepState* st : live(steps)) {
    tl_sim* s = st->s;
    std::swap(s->Tpred, s->ccur);
    k_copy(s->L, s->fprev, s->fstate, s->gf.npad);
  }
  phase_mark(prof, 1, B.stream);
  // 3. micro steps j = 1..m-1 with blended Dirichlet data (j = 1..m with
  // the alternate formulation, which has no correction to iterate)
  auto last_micro = [](const StepState* st) {
    return alternate(st->s) ? st->m : st->m - 1;
  };
  int jmax = 0;
  for (StepState* st : live(steps)) jmax = std::max(jmax, last_micro(st));
  for (int j = 1; j <= jmax; ++j) {
    std::vector<StepState*> list;
    for (StepState* st : live(steps))
      if (j <= last_micro(st)) list.push_back(st);
    // before the solve, for all listed simulations in one launch: the
    // initial guess (the previous micro step; from the second micro step
    // on its linear extrapolation 2 T_{j-1} - T_{j-2}), the Dirichlet data
    // and the laser load
    if ((int)list.size() > B.micro_cap)
      throw DevErr{"batch larger than its context"};
    int per_micro = 1;
    for (size_t q = 0; q < list.size(); ++q) {
      micro_prep_item(*list[q], j, B.h_micro[q]);
      per_micro = std::max(per_micro, B.h_micro[q].nblk);
    }
    if (!list.empty()) {
      hip_check(hipMemcpyAsync(B.d_micro, B.h_micro,
                               sizeof(MicroItem) * list.size(),
                               hipMemcpyHostToDevice, B.stream),
                "hipMemcpyAsync(micro items)");
      k_micro_prep(B.L, B.d_micro, (int)list.size(), per_micro);
    }
    batch_fine(
        B, list,
        [](StepState& st, Region& rg, double& tau, const double*& Told) {
          rg = region_window(st.s);
          tau = st.dt;
          Told = st.s->fprev;
        },
        prof);
    // the consistent formulation's sum of the micro-step fields
    for (StepState* st : list)
      if (!st->failed && consistent(st->s))
        k_accumulate(st->s->L, st->s->fsum, st->s->fcur, st->s->gf.npad, j == 1);
    // after it, in one launch: reactions on the interface, bottom and
    // top-surface heat flows (the second half of the item table: its first
    // half may still be in flight to the device)
    {
      MicroItem* hp = B.h_micro + B.micro_cap;
      int n = 0, per = 1;
      for (StepState* st : list)
        if (!st->failed) {
          micro_post_item(*st, j, hp[n]);
          per = std::max(per, hp[n++].nblk);
        }
      if (n > 0) {
        hip_check(hipMemcpyAsync(B.d_micro + B.micro_cap, hp,
                                 sizeof(MicroItem) * n, hipMemcpyHostToDevice,
                                 B.stream),
                  "hipMemcpyAsync(micro items)");
        k_micro_post(B.L, B.d_micro + B.micro_cap, n, per);
      }
    }
    for (StepState* st : list) {
      if (st->failed) continue;
      tl_sim* s = st->s;
      // (pp, prev, cur) <- (prev, cur, spare)
      double* spare = s->fpp;
      s->fpp = s->fprev;
      s->fprev = s->fcur;
      s->fcur = spare;
      ++s->stats.micro_steps;
    }
  }
  // the alternate formulation: the predictor is the global step, the last
  // micro step the local one; the global problem's ledger
  for (StepState* st : live(steps)) {
    tl_sim* s = st->s;
    if (!alternate(s)) continue;
    st->dn_done = true;
    k_bottom_sum(s->L, s->gc, s->cR, -st->Dt, &s->led->bottom, s->partials);
    k_surface_sum(s->L, s->gc, region_all(), surf_coarse(s), s->Tpred, st->Dt,
                  &s->led->surface, s->partials);
    std::swap(s->Tn, s->Tpred);
    std::swap(s->fstate, s->fprev);
    energy_now(s, &s->led->stored);
    s->stats.fine_dof_steps += fine_free_nodes(s->gf, s->win) * st->m;
  }
  phase_mark(prof, 2, B.stream);
  // 4. two-level correction at t_{n+1}
  for (StepState* st : live(steps)) {
    tl_sim* s = st->s;
    if (alternate(s)) continue;
    fine_load(s, st->n, st->m, st->dt);
    if (s->opts.coupling == TL_COUPLE_DN || consistent(s))   // interface trace
      k_copy(s->L, s->lam, s->Tpred, s->gc.npad);
    if (st->m >= 2)   // extrapolated from the last two micro steps
      k_extrapolate(s->L, s->fcur, s->fprev, s->fpp, s->gf.npad);
    else
      k_copy(s->L, s->fcur, s->fprev, s->gf.npad);
    k_copy(s->L, s->ccur, s->Tpred, s->gc.npad);
  }
  // the composite-grid form: one solve; the reactions of micro steps
  // 1..m-1 restricted by P^T are its fixed interface load
  {
    std::vector<StepState*> c64, c32;
    for (StepState* st : live(steps)) {
      tl_sim* s = st->s;
      if (s->opts.coupling != TL_COUPLE_COMPOSITE) continue;
      (s->opts.precision == TL_MIXED ? c32 : c64).push_back(st);
      if (st->m > 1)
        k_restrict(s->L, s->gf, s->gc, s->win, s->rho, nullptr, -1.0 / st->m,
                   s->ext);
      else
        k_fill(s->L, s->ext, 0.0, s->gc.npad);
      st->dn_done = true;
    }
    batch_composite<double>(B, c64, prof);
    batch_composite<float>(B, c32, prof);
    for (StepState* st : live(steps)) {
      tl_sim* s = st->s;
      if (s->opts.coupling != TL_COUPLE_COMPOSITE) continue;
      k_inject(s->L, s->gf, s->gc, s->win, s->fcur, s->ccur);
      st->it = 1;
    }
  }
  for (;;) {
    std::vector<StepState*> list;
    for (StepState* st : live(steps))
      if (!st->dn_done) list.push_back(st);
    if (list.empty()) break;
    for (StepState* st : list) {
      tl_sim* s = st->s;
      if (++st->it > s->opts.dn_max) {
        fail_step(*st, "two-level iteration did not converge");
        continue;
      }
      k_fine_dirichlet(s->L, s->gf, s->gc, s->win, s->mat_in.T_bottom, s->lam,
                       nullptr, 0.0, s->fcur);
    }
    list.clear();
    for (StepState* st : live(steps))
      if (!st->dn_done) list.push_back(st);
    batch_fine(
        B, list,
        [](StepState& st, Region& rg, double& tau, const double*& Told) {
          rg = region_window(st.s);
          tau = st.dt;
          Told = st.s->fprev;
        },
        prof, true);
    std::vector<StepState*> clist;
    for (StepState* st : list) {
      if (st->failed) continue;
      tl_sim* s = st->s;
      if (consistent(s)) {
        // the global problem on the whole plate, loaded inside the window
        // by P^T of the load from the local solution; no injection
        k_consistent_source(s->L, s->gf, s->win, s->fcur, s->fstate,
                            st->m > 1 ? s->fsum : nullptr,
                            st->m > 1 ? s->rho : nullptr, s->fR, st->m, st->Dt,
                            s->kf, s->rhocf, s->fsrc);
        k_fill(s->L, s->ext, 0.0, s->gc.npad);
        k_restrict_all(s->L, s->gf, s->gc, s->win, s->fsrc, s->ext);
      } else {
        k_restrict(s->L, s->gf, s->gc, s->win, st->m > 1 ? s->rho : nullptr,
                   s->fR, -1.0 / st->m, s->ext);
        k_inject(s->L, s->gf, s->gc, s->win, s->fcur, s->ccur);
      }
      clist.push_back(st);
    }
    // the coarse solves, the CG in the path's precision
    std::vector<StepState*> c64, c32;
    for (StepState* st : clist)
      (st->s->opts.precision == TL_MIXED ? c32 : c64).push_back(st);
    batch_solve<double>(
        B, c64, false,
        [](StepState& st) {
          return make_job<double>(
              st.s, false,
              consistent(st.s) ? region_fict(st.s) : region_outside(st.s),
              st.Dt, st.s->Tn, st.s->Fout, st.s->ext);
        },
        nullptr);
    batch_solve<float>(
        B, c32, false,
        [](StepState& st) {
          return make_job<float>(
              st.s, false,
              consistent(st.s) ? region_fict(st.s) : region_outside(st.s),
              st.Dt, st.s->Tn, st.s->Fout, st.s->ext);
        },
        nullptr);
    // interface residuals lambda' - lambda, read back for all at once
    std::vector<StepState*> glist;
    for (StepState* st : clist) {
      if (st->failed) continue;
      tl_sim* s = st->s;
      const int ng = s->n_gamma;
      k_gamma_gather(s->L, s->gidx, ng, s->ccur, s->lam, s->gbuf);
      if (ng > 0)
        hip_check(hipMemcpyAsync(s->h_gbuf, s->gbuf, 2 * sizeof(double) * ng,
                                 hipMemcpyDeviceToHost, s->stream),
                  "hipMemcpyAsync(interface)");
      glist.push_back(st);
    }
    for (StepState* st : glist)
      hip_check(hipStreamSynchronize(st->s->stream), "hipStreamSynchronize");
    for (StepState* st : glist) {
      tl_sim* s = st->s;
      const int ng = s->n_gamma;
      st->lt_v.resize(ng);
      st->lam_v.resize(ng);
      double diff = 0.0;
      for (int q = 0; q < ng; ++q) {
        st->lt_v[q] = s->h_gbuf[2 * q];
        st->lam_v[q] = s->h_gbuf[2 * q + 1];
        diff = std::max(diff, std::fabs(st->lt_v[q] - st->lam_v[q]));
      }
      if (!std::isfinite(diff)) {
        fail_step(*st, "non-finite interface update");
        continue;
      }
      if (diff <= s->opts.dn_tol) {
        st->dn_done = true;
        continue;
      }
      s->iqn.update(st->lam_v, st->lt_v, s->theta0, s->opts.dn_theta > 0.0,
                     st->next);
      for (int q = 0; q < ng; ++q) s->h_gbuf[q] = st->next[q];
      hip_check(hipMemcpyAsync(s->gbuf, s->h_gbuf, sizeof(double) * ng,
                               hipMemcpyHostToDevice, s->stream),
                "hipMemcpyAsync(interface)");
      k_gamma_scatter(s->L, s->gidx, ng, s->gbuf, s->lam);
    }
  }
  phase_mark(prof, 3, B.stream);
  // 5. ledger and commit of the new state
  for (StepState* st : live(steps)) {
    tl_sim* s = st->s;
    if (alternate(s)) continue;   // committed above
    const Launch L = s->L;
    s->stats.dn_iters += st->it;
    ++s->stats.micro_steps;
    // bottom heat flow of the last fine step and of the coarse outside solve
    // (a composite solve keeps the fine rows scaled by 1/m)
    const bool comp = s->opts.coupling == TL_COUPLE_COMPOSITE;
    k_interface_accumulate(L, s->gf, s->win, s->fR, nullptr, 0,
                           comp ? -st->Dt : -st->dt, &s->led->bottom,
                           s->partials);
    k_bottom_sum(L, s->gc, s->cR, -st->Dt, &s->led->bottom, s->partials);
    // heat lost through the top by the last fine step and the outside solve
    k_surface_sum(L, s->gf, region_window(s), surf_fine(s), s->fcur, st->dt,
                  &s->led->surface, s->partials);
    k_surface_sum(L, s->gc, region_outside(s), surf_coarse(s), s->ccur, st->Dt,
                  &s->led->surface, s->partials);
    std::swap(s->Tn, s->ccur);
    std::swap(s->fstate, s->fcur);
    energy_now(s, &s->led->stored);
    s->stats.fine_dof_steps += fine_free_nodes(s->gf, s->win) * st->m;
  }
  phase_mark(prof, kPhases, B.stream);
}

// After a successful macro step: read the device ledger, count the step.
void commit_step(tl_sim* s) {
  read_ledger(s);
  s->ledger.stored = s->h_led->stored;
  s->ledger.absorbed = s->h_led->absorbed;
  s->ledger.bottom = s->h_led->bottom;
  s->ledger.remap = s->h_led->remap;
  s->ledger.surface = s->h_led->surface;
  ++s->n_macro;
  ++s->stats.macro_steps;
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
  // padded node counts in floating point (no integer overflow for any
  // input); every index of a grid below the limit fits an int, and every
  // byte offset into one of its FP64 arrays fits the 32-bit offsets the
  // batched kernels address their arrays with (2e8 x 8 B < 2^32)
  auto padded = [](double nx, double ny, double nz) {
    return (std::floor((nx + 34.0) / 32.0) * 32.0) * (ny + 3.0) * (nz + 3.0);
  };
  const double r = me->refine;
  const double nf = padded(r * me->win_nx, r * me->win_ny, r * me->win_nz);
  const double nc = padded(me->nx, me->ny, me->nz);
  if (nf > 2.0e8 || nc > 2.0e8) return fail(TL_EINVAL, "grid too large");
  if (!finite_all({ma->rho, ma->T_lo, ma->T_hi, ma->c_lo, ma->c_hi, ma->k_lo,
                   ma->k_hi, ma->latent, ma->T_sol, ma->T_liq, ma->sharpness,
                   ma->T_init, ma->T_bottom, ma->h_conv, ma->emissivity,
                   ma->T_amb}))
    return fail(TL_EINVAL, "non-finite material parameter");
  if (ma->h_conv < 0 || ma->emissivity < 0 || ma->emissivity > 1 ||
      ma->T_amb <= 0)
    return fail(TL_EINVAL,
                "surface loss needs h_conv >= 0, 0 <= emissivity <= 1, T_amb > 0");
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
                     t.absorptivity, t.depth}) ||
        t.speed <= 0 || t.radius <= 0 || t.power < 0 || t.absorptivity < 0)
      return fail(TL_EINVAL, "invalid track " + std::to_string(q));
    if (op->source == TL_SOURCE_VOLUME &&
        (t.depth <= 0 || (t.x0 != t.x1 && t.y0 != t.y1)))
      return fail(TL_EINVAL, "the volume source needs depth > 0 and tracks "
                             "along x or y (track " + std::to_string(q) + ")");
  }
  if (op->source != TL_SOURCE_SURFACE && op->source != TL_SOURCE_VOLUME)
    return fail(TL_EINVAL, "unknown source model");
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
  if (op->coupling != TL_COUPLE_DN && op->coupling != TL_COUPLE_COMPOSITE &&
      op->coupling != TL_COUPLE_ALTERNATE && op->coupling != TL_COUPLE_CONSISTENT)
    return fail(TL_EINVAL, "unknown coupling");
  if (!finite_all({ma->k_fict, ma->rhoc_fict}) || ma->k_fict < 0 ||
      ma->rhoc_fict < 0)
    return fail(TL_EINVAL, "k_fict and rhoc_fict must be finite and >= 0");
  return TL_OK;
}

}  // namespace

// ===========================================================================
// Internal interface for the serving loop
// ===========================================================================
namespace tl {

struct BatchImpl {
  BatchCtx ctx;
  Profiler prof;
  tl_stats pstats{};  // only the timing and op-byte fields are used
};

// Items for 2 * max_slots (composite pairs take two), scalars and
// micro-step items for max_slots.
size_t batch_tables_bytes(int max_slots) {
  return align_up(sizeof(SolveItem) * 2 * (size_t)max_slots) +
         align_up(sizeof(LevelScalars) * (size_t)max_slots) +
         align_up(sizeof(MicroItem) * 2 * (size_t)max_slots);
}

tl_status batch_tables_init(BatchTables* bt, void* dev_area, int max_slots,
                            void* hip_stream) {
  BatchImpl* b = new BatchImpl();
  b->prof.stats = &b->pstats;
  char* p = (char*)dev_area;
  b->ctx.d_items = (SolveItem*)p;
  b->ctx.d_sc =
      (LevelScalars*)(p + align_up(sizeof(SolveItem) * 2 * (size_t)max_slots));
  b->ctx.d_micro =
      (MicroItem*)(p + align_up(sizeof(SolveItem) * 2 * (size_t)max_slots) +
                   align_up(sizeof(LevelScalars) * (size_t)max_slots));
  b->ctx.cap = max_slots;
  b->ctx.item_cap = 2 * max_slots;
  b->ctx.micro_cap = max_slots;
  b->ctx.stream = (hipStream_t)hip_stream;
  b->ctx.L.stream = hip_stream;
  if (hipHostMalloc((void**)&b->ctx.h_items, sizeof(SolveItem) * 2 * max_slots,
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&b->ctx.h_sc, sizeof(LevelScalars) * max_slots,
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&b->ctx.h_micro, sizeof(MicroItem) * 2 * max_slots,
                    hipHostMallocDefault) != hipSuccess) {
    batch_tables_free(&(bt->impl = b, *bt));
    return fail(TL_EDEVICE, "hipHostMalloc failed");
  }
  bt->impl = b;
  return TL_OK;
}

void batch_tables_free(BatchTables* bt) {
  BatchImpl* b = (BatchImpl*)bt->impl;
  if (!b) return;
  if (b->ctx.h_items) (void)hipHostFree(b->ctx.h_items);
  if (b->ctx.h_sc) (void)hipHostFree(b->ctx.h_sc);
  if (b->ctx.h_micro) (void)hipHostFree(b->ctx.h_micro);
  if (b->prof.ev[0])
    for (int q = 0; q < 2 * kProfPairs; ++q) (void)hipEventDestroy(b->prof.ev[q]);
  delete b;
  bt->impl = nullptr;
}

tl_status step_many(const std::vector<tl_sim*>& sims, BatchTables* bt,
                    std::vector<std::string>& errs) {
  BatchImpl* b = (BatchImpl*)bt->impl;
  errs.assign(sims.size(), std::string());
  std::vector<StepState> steps(sims.size());
  for (size_t q = 0; q < sims.size(); ++q) steps[q].s = sims[q];
  try {
    macro_step_batch(steps, b->ctx, b->prof.every > 0 ? &b->prof : nullptr);
    for (size_t q = 0; q < sims.size(); ++q) {
      if (steps[q].failed)
        errs[q] = steps[q].err;
      else
        commit_step(sims[q]);
    }
  } catch (const NoConv& e) {
    return fail(TL_ENOCONV, e.msg);
  } catch (const DevErr& e) {
    return fail(TL_EDEVICE, e.msg);
  }
  return TL_OK;
}

tl_status validate_request(const tl_mesh* mesh, const tl_material* material,
                           const tl_scan_path* scan, const tl_options* opts) {
  return validate(mesh, material, scan, opts);
}

tl_status batch_set_profiling(BatchTables* bt, int sample_every) {
  BatchImpl* b = (BatchImpl*)bt->impl;
  if (sample_every < 0) return fail(TL_EINVAL, "sample_every must be >= 0");
  if (sample_every > 0 && !b->prof.ev[0]) {
    for (int q = 0; q < 2 * kProfPairs; ++q)
      HIP_OK(hipEventCreateWithFlags(&b->prof.ev[q], hipEventDisableSystemFence));
  }
  b->prof.every = sample_every;
  b->prof.count = 0;
  return TL_OK;
}

void batch_get_profile(BatchTables* bt, int64_t* launches, double* ms,
                       double* bytes) {
  BatchImpl* b = (BatchImpl*)bt->impl;
  if (launches) *launches = b->pstats.fine_op_timed;
  if (ms) *ms = b->pstats.fine_op_timed_ms;
  if (bytes) *bytes = b->pstats.fine_op_bytes;
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

size_t tl_sim_nodes(tl_sim* s, int level) {
  return (size_t)(level == 0 ? s->gc.nreal : s->gf.nreal);
}

}  // namespace tl

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

static tl_status create_sim(const tl_mesh* mesh, const tl_material* material,
                            const tl_scan_path* scan, const tl_options* opts,
                            void* dev_workspace, size_t ws_bytes,
                            void* hip_stream, bool pinned_host, int static_dev,
                            tl_sim** out);

tl_status tl_create(const tl_mesh* mesh, const tl_material* material,
                    const tl_scan_path* scan, const tl_options* opts,
                    void* dev_workspace, size_t ws_bytes, void* hip_stream,
                    tl_sim** out) {
  if (!out) return fail(TL_EINVAL, "out is null");
  *out = nullptr;
  return create_sim(mesh, material, scan, opts, dev_workspace, ws_bytes,
                    hip_stream, true, -1, out);
}

static tl_status create_sim(const tl_mesh* mesh, const tl_material* material,
                            const tl_scan_path* scan, const tl_options* opts,
                            void* dev_workspace, size_t ws_bytes,
                            void* hip_stream, bool pinned_host, int static_dev,
                            tl_sim** out) {
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
                               t.radius, t.absorptivity, t.depth});
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
  s->mat_global = m;
  if (opts->coupling == TL_COUPLE_ALTERNATE) s->mat_global.latent = 0.0;
  {
    // the consistent formulation's coefficients inside the window: given,
    // or the law's conductivity and rho c at T_init
    const double Ti = std::min(std::max(material->T_init, m.T_lo), m.T_hi);
    s->kf = material->k_fict > 0 ? material->k_fict
                                 : m.k_lo + m.kslope * (Ti - m.T_lo);
    s->rhocf = material->rhoc_fict > 0
                   ? material->rhoc_fict
                   : m.rho * (m.c_lo + m.cslope * (Ti - m.T_lo));
  }
  s->lay = lay;
  s->gc = lay.gc;
  s->gf = lay.gf;
  s->stream = (hipStream_t)hip_stream;
  s->L.stream = hip_stream;
  s->ws = (char*)dev_workspace;
  auto C = [&](int a) { return (double*)(s->ws + lay.off_c[a]); };
  s->Tn = C(0); s->Tpred = C(1); s->ccur = C(2); s->ctrial = C(3);
  s->lam = C(4); s->gdw = C(5); s->cR = C(6); s->Fall = C(7);
  s->Fout = C(8); s->ext = C(9);
  auto cgb64 = [&](auto A) {
    return CGBufs<double>{(double*)A(0), (double*)A(1), (double*)A(2),
                          {(double*)A(3), (double*)A(4)},
                          {(double*)A(5), (double*)A(6)},
                          {(double*)A(7), (double*)A(8)}, (double*)A(9),
                          {(double*)A(10), (double*)A(11)}};
  };
  s->ccg = cgb64([&](int a) { return (void*)C(10 + a); });
  s->cHold = C(22);
  if (lay.ccg32) {
    auto A = [&](int a) { return (float*)(s->ws + lay.off_ccg32[a]); };
    s->ccg32 = CGBufs<float>{A(0), A(1), A(2), {A(3), A(4)}, {A(5), A(6)},
                             {A(7), A(8)}, A(9), {A(10), A(11)}};
  } else {
    s->ccg32 = CGBufs<float>{};
  }
  auto FD = [&](int a) { return (double*)(s->ws + lay.off_fd[a]); };
  s->fstate = FD(0); s->fprev = FD(1); s->fcur = FD(2); s->ftrial = FD(3);
  s->falt = FD(4); s->fR = FD(5); s->fF = FD(6); s->rho = FD(7);
  s->fpp = FD(9);
  s->fHold = FD(8);
  if (lay.fx) {
    s->fsum = (double*)(s->ws + lay.off_fx[0]);
    s->fsrc = (double*)(s->ws + lay.off_fx[1]);
  }
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
  s->tpart = (double*)(s->ws + lay.off_tpart);
  s->tpart2 = (double*)(s->ws + lay.off_tpart2);
  s->gidx = (int*)(s->ws + lay.off_gidx);
  s->gbuf = (double*)(s->ws + lay.off_gbuf);
  s->pinned_host = pinned_host;
  s->static_dev = static_dev;
  s->h_sc = nullptr;
  s->h_led = nullptr;
  s->h_gbuf = nullptr;
  auto halloc = [&](void** p, size_t n) {
    if (pinned_host) return hipHostMalloc(p, n, hipHostMallocDefault) == hipSuccess;
    *p = std::calloc(1, n);
    return *p != nullptr;
  };
  if (!halloc((void**)&s->h_sc, 2 * sizeof(LevelScalars)) ||
      !halloc((void**)&s->batch.h_items, 2 * sizeof(SolveItem)) ||
      !halloc((void**)&s->batch.h_micro, 2 * sizeof(MicroItem)) ||
      !halloc((void**)&s->h_led, sizeof(LedgerDev)) ||
      !halloc((void**)&s->h_gbuf, 2 * sizeof(double) * lay.gamma_cap)) {
    s->static_dev = -1;   // the caller keeps its claim on the device's array
    tl_destroy(s);
    return fail(TL_EDEVICE, pinned_host ? "hipHostMalloc failed"
                                        : "host memory allocation failed");
  }
  s->batch.d_items = (SolveItem*)(s->ws + lay.off_items);
  s->batch.d_micro = (MicroItem*)(s->ws + lay.off_micro);
  s->batch.d_sc = s->sc_c;
  s->batch.h_sc = s->h_sc;
  s->batch.cap = 2;
  s->batch.item_cap = 2;
  s->batch.micro_cap = 1;
  s->batch.stream = s->stream;
  s->batch.L = s->L;
  std::memset(&s->stats, 0, sizeof(s->stats));
  s->prof.stats = &s->stats;
  s->stats.fine_nodes[0] = s->gf.nx;
  s->stats.fine_nodes[1] = s->gf.ny;
  s->stats.fine_nodes[2] = s->gf.nz;
  s->stats.coarse_nodes[0] = s->gc.nx;
  s->stats.coarse_nodes[1] = s->gc.ny;
  s->stats.coarse_nodes[2] = s->gc.nz;
  s->n_macro = 0;
  s->theta0 = opts->dn_theta > 0 ? opts->dn_theta
                                 : mesh->refine / (mesh->refine + 1.0);
  s->last_cg_f = s->last_cg_c = s->last_cg_x = 8;
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
    s->static_dev = -1;   // the caller keeps its claim on the device's array
    tl_destroy(s);
    return st;
  }
  *out = s;
  return TL_OK;
}

// ---- allocation-free creation (tl_create_static) ---------------------------
// The workspace of a handle made by tl_create_static is this device array:
// every GPU the library runs on holds its own copy until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory; the
// device address comes from hipGetSymbolAddress, once per device with that
// device current, and only that address is ever passed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[TL_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxStaticDevices];   // device address of `scratch`
bool g_static_held[kMaxStaticDevices];   // a live handle holds the array

void release_static(int dev) {
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (dev >= 0 && dev < kMaxStaticDevices) g_static_held[dev] = false;
}
}  // namespace

tl_status tl_create_static(const tl_mesh* mesh, const tl_material* material,
                           const tl_scan_path* scan, const tl_options* opts,
                           void* hip_stream, tl_sim** out) {
  if (!out) return fail(TL_EINVAL, "out is null");
  *out = nullptr;
  tl_status st = validate(mesh, material, scan, opts);
  if (st != TL_OK) return st;
  const size_t need = make_layout(*mesh, *opts).total;
  if (need > (size_t)TL_STATIC_WORKSPACE_BYTES)
    return fail(TL_ENOMEM, "tl_create_static: the problem needs " +
                               std::to_string(need) +
                               " bytes of workspace, more than the static "
                               "workspace's " +
                               std::to_string((size_t)TL_STATIC_WORKSPACE_BYTES) +
                               "; use tl_create with a caller-owned workspace");
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (hip_stream != nullptr) {
    int sdev = -1;
    HIP_OK(hipStreamGetDevice((hipStream_t)hip_stream, &sdev));
    if (sdev != dev)
      return fail(TL_EINVAL,
                  "tl_create_static: the stream belongs to another device "
                  "than the current one");
  }
  if (dev < 0 || dev >= kMaxStaticDevices)
    return fail(TL_EDEVICE, "tl_create_static: device index out of range");
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_ptr[dev] == nullptr) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || p == nullptr)
        return fail(TL_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                    hipGetErrorString(e));
      g_static_ptr[dev] = p;
    }
    if (g_static_held[dev])
      return fail(TL_EBUSY,
                  "tl_create_static: a live handle already holds this "
                  "device's static workspace (destroy it first)");
    g_static_held[dev] = true;
    ws = g_static_ptr[dev];
  }
  // create_sim zero-fills the whole workspace before use, so nothing of the
  // previous handle's contents survives
  st = create_sim(mesh, material, scan, opts, ws,
                  (size_t)TL_STATIC_WORKSPACE_BYTES, hip_stream, false, dev, out);
  if (st != TL_OK) release_static(dev);
  return st;
}

tl_status tl_step(tl_sim* s, int n_macro) {
  if (!s) return fail(TL_EINVAL, "null handle");
  if (n_macro < 0) return fail(TL_EINVAL, "n_macro must be >= 0");
  auto t0 = std::chrono::steady_clock::now();
  tl_status st = TL_OK;
  for (int q = 0; q < n_macro; ++q) {
    const Window w_saved = s->win;
    const Geo gf_saved = s->gf;
    // every field pointer a macro step permutes (window moves, solves,
    // micro-step rotation, commit), so that a failure at any point restores
    // the committed buffers and a set of distinct work buffers
    double** const perm[] = {&s->Tn,     &s->Tpred, &s->ccur,  &s->ctrial,
                             &s->fstate, &s->fprev, &s->fcur,  &s->ftrial,
                             &s->falt,   &s->fpp};
    constexpr int kPerm = (int)(sizeof(perm) / sizeof(perm[0]));
    double* perm_saved[kPerm];
    for (int q2 = 0; q2 < kPerm; ++q2) perm_saved[q2] = *perm[q2];
    const tl_stats stats_saved = s->stats;
    // solver history later steps depend on: CG budgets, secant pairs
    const int cg_saved[3] = {s->last_cg_f, s->last_cg_c, s->last_cg_x};
    const Interface iqn_saved = s->iqn;
    try {
      std::vector<StepState> steps(1);
      steps[0].s = s;
      macro_step_batch(steps, s->batch, &s->prof);
      if (steps[0].failed) throw NoConv{steps[0].err};
      commit_step(s);   // synchronises with the stream
      phase_flush(&s->prof, s->stats.phase_ms);
    } catch (const NoConv& e) {
      st = fail(TL_ENOCONV, e.msg);
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
      for (int q2 = 0; q2 < kPerm; ++q2) *perm[q2] = perm_saved[q2];
      s->stats = stats_saved;
      s->last_cg_f = cg_saved[0];
      s->last_cg_c = cg_saved[1];
      s->last_cg_x = cg_saved[2];
      try {
        set_interface(s);
        s->iqn = iqn_saved;
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
// Checkpoint: header, coarse and fine fields (plain layout), then the
// solver history that later steps depend on -- the two-level secant pairs
// (ncols columns of V, then of W, n_gamma values each) -- so that a restored
// run continues exactly as the saved one would have.
struct CkptHeader {
  char magic[8];
  int32_t version;
  int32_t I0, J0;
  int32_t gc_n, gf_n;
  int32_t n_gamma, ncols;
  int32_t last_cg_f, last_cg_c, last_cg_x, pad;
  int64_t n_macro;
  tl_ledger ledger;
  tl_stats stats;
};
size_t ckpt_bytes(const tl_sim* s) {
  const size_t ng = s->iqn.V.empty() ? 0 : s->iqn.V[0].size();
  return sizeof(CkptHeader) +
         ((size_t)s->gc.nreal + s->gf.nreal) * sizeof(double) +
         2 * s->iqn.V.size() * ng * sizeof(double);
}
}  // namespace

tl_status tl_save(tl_sim* s, void* host, size_t cap, size_t* used) {
  if (!s || !used) return fail(TL_EINVAL, "null argument");
  const size_t need = ckpt_bytes(s);
  *used = need;
  if (!host) return TL_OK;
  if (cap < need) return fail(TL_ENOMEM, "checkpoint buffer too small");
  CkptHeader h;
  std::memset(&h, 0, sizeof(h));
  std::memcpy(h.magic, "TLCKPT3", 8);
  h.version = 3;
  h.I0 = s->win.I0;
  h.J0 = s->win.J0;
  h.gc_n = s->gc.nreal;
  h.gf_n = s->gf.nreal;
  h.ncols = (int32_t)s->iqn.V.size();
  h.n_gamma = h.ncols ? (int32_t)s->iqn.V[0].size() : 0;
  h.last_cg_f = s->last_cg_f;
  h.last_cg_c = s->last_cg_c;
  h.last_cg_x = s->last_cg_x;
  h.n_macro = s->n_macro;
  h.ledger = s->ledger;
  h.stats = s->stats;
  char* p = (char*)host;
  std::memcpy(p, &h, sizeof(h));
  int dims[3];
  tl_status st = tl_get_temperature(s, 0, (double*)(p + sizeof(h)),
                                    (size_t)s->gc.nreal, dims, nullptr);
  if (st != TL_OK) return st;
  st = tl_get_temperature(
      s, 1, (double*)(p + sizeof(h) + (size_t)s->gc.nreal * sizeof(double)),
      (size_t)s->gf.nreal, dims, nullptr);
  if (st != TL_OK) return st;
  char* q = p + sizeof(h) + ((size_t)s->gc.nreal + s->gf.nreal) * sizeof(double);
  const size_t col = (size_t)h.n_gamma * sizeof(double);
  for (const auto& v : s->iqn.V) { std::memcpy(q, v.data(), col); q += col; }
  for (const auto& w : s->iqn.W) { std::memcpy(q, w.data(), col); q += col; }
  return TL_OK;
}

tl_status tl_load(tl_sim* s, const void* host, size_t n) {
  if (!s || !host) return fail(TL_EINVAL, "null argument");
  if (n < sizeof(CkptHeader)) return fail(TL_EINVAL, "checkpoint too short");
  CkptHeader h;
  std::memcpy(&h, host, sizeof(h));
  if (std::memcmp(h.magic, "TLCKPT3", 8) != 0 || h.version != 3)
    return fail(TL_EINVAL, "not a checkpoint of this library");
  if (h.gc_n != s->gc.nreal || h.gf_n != s->gf.nreal)
    return fail(TL_EINVAL, "checkpoint grid sizes differ from this handle");
  if (h.ncols < 0 || h.ncols > Interface::kMaxCols || h.n_gamma < 0 ||
      (h.ncols > 0 && h.n_gamma == 0))
    return fail(TL_EINVAL, "checkpoint interface history is malformed");
  const size_t need = sizeof(CkptHeader) +
                      ((size_t)s->gc.nreal + s->gf.nreal) * sizeof(double) +
                      2 * (size_t)h.ncols * h.n_gamma * sizeof(double);
  if (n < need) return fail(TL_EINVAL, "checkpoint truncated");
  if (h.I0 < 0 || h.J0 < 0 || h.I0 + s->mesh.win_nx > s->mesh.nx ||
      h.J0 + s->mesh.win_ny > s->mesh.ny)
    return fail(TL_EINVAL, "checkpoint window outside the plate");
  // the secant pairs must have the length of the restored window's
  // interface (checked before anything of the handle changes)
  if (h.ncols > 0 &&
      (size_t)h.n_gamma != interface_nodes(s->gc, make_window(s->mesh, h.I0, h.J0)).size())
    return fail(TL_EINVAL, "checkpoint interface history does not fit its window");
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
    s->last_cg_f = h.last_cg_f;
    s->last_cg_c = h.last_cg_c;
    s->last_cg_x = h.last_cg_x;
    // the secant pairs (set_interface above cleared the old ones)
    const double* q = (const double*)(p + ((size_t)s->gc.nreal + s->gf.nreal) * sizeof(double));
    for (int c = 0; c < h.ncols; ++c, q += h.n_gamma)
      s->iqn.V.emplace_back(q, q + h.n_gamma);
    for (int c = 0; c < h.ncols; ++c, q += h.n_gamma)
      s->iqn.W.emplace_back(q, q + h.n_gamma);
    write_ledger(s);
  } catch (const DevErr& e) {
    return fail(TL_EDEVICE, e.msg);
  }
  return TL_OK;
}

tl_status tl_set_profiling(tl_sim* s, int sample_every) {
  if (!s) return fail(TL_EINVAL, "null handle");
  if (sample_every < 0) return fail(TL_EINVAL, "sample_every must be >= 0");
  if (sample_every > 0 && !s->prof.ev[0]) {
    for (int q = 0; q < 2 * kProfPairs; ++q)
      HIP_OK(hipEventCreateWithFlags(&s->prof.ev[q], hipEventDisableSystemFence));
    try {
      phase_events(&s->prof, true);
    } catch (const DevErr& e) {
      return fail(TL_EDEVICE, e.msg);
    }
  }
  s->prof.every = sample_every;
  s->prof.count = 0;
  return TL_OK;
}

void tl_destroy(tl_sim* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  else (void)hipDeviceSynchronize();
  if (s->prof.ev[0])
    for (int q = 0; q < 2 * kProfPairs; ++q) (void)hipEventDestroy(s->prof.ev[q]);
  phase_events(&s->prof, false);
  auto hfree = [&](void* p) {
    if (!p) return;
    if (s->pinned_host) (void)hipHostFree(p);
    else std::free(p);
  };
  hfree(s->batch.h_items);
  hfree(s->batch.h_micro);
  hfree(s->h_sc);
  hfree(s->h_led);
  hfree(s->h_gbuf);
  // the stream has drained: the device's static workspace is free again
  if (s->static_dev >= 0) release_static(s->static_dev);
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
  // in floating point: no integer overflow for any input
  if (std::floor((g->nx + 34.0) / 32.0) * 32.0 * (g->ny + 3.0) * (g->nz + 3.0) > 2.0e9)
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

tl_status tl_op_sync_probe(int blocks, int rounds, int barrier, double* data,
                           size_t n, void* ctl, double* us_out,
                           void* hip_stream) {
  if (!data || !ctl || !us_out) return fail(TL_EINVAL, "null argument");
  if (n < 1 || rounds < 1 || blocks < 1)
    return fail(TL_EINVAL, "n, rounds and blocks must be >= 1");
  if (barrier && blocks > sync_probe_resident())
    return fail(TL_EINVAL, "a barrier run needs all workgroups resident: at most " +
                               std::to_string(sync_probe_resident()));
  const Launch L{hip_stream};
  hipStream_t st = (hipStream_t)hip_stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_OK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(TL_EDEVICE, "hipEventCreate failed");
  }
  tl_status res = TL_OK;
  int err = 0;
  float ms = 0.0f;
  k_zero_bytes(L, ctl, 1024);
  hipError_t e = hipEventRecord(e0, st);
  if (e == hipSuccess)
    e = (hipError_t)k_sync_probe(L, blocks, rounds, barrier, data, (long)n,
                                 (unsigned*)ctl);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess)
    e = hipMemcpy(&err, (char*)ctl + 128 * sizeof(unsigned), sizeof(int),
                  hipMemcpyDeviceToHost);
  if (e != hipSuccess)
    res = fail(TL_EDEVICE, std::string("sync probe: ") + hipGetErrorString(e));
  else if (err)
    res = fail(TL_EDEVICE, "sync probe: the barrier's bounded wait ran out");
  *us_out = 1e3 * ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return res;
}

tl_status tl_op_apply(const tl_grid* grid, int precision, int kernel,
                      int blocks, const void* d, const void* kappa,
                      const void* v, void* y, int repeat, void* hip_stream) {
  tl_status st = check_grid(grid);
  if (st != TL_OK) return st;
  if (!d || !kappa || !v || !y || repeat < 1)
    return fail(TL_EINVAL, "bad operator arguments");
  if (precision != TL_FP64 && precision != TL_MIXED)
    return fail(TL_EINVAL, "unknown precision");
  if (kernel != kOpAuto && kernel != kOpTiled && kernel != kOpZmarch)
    return fail(TL_EINVAL, "unknown operator kernel");
  if (blocks < 0 || blocks % 8 != 0 || blocks > (1 << 20))
    return fail(TL_EINVAL, "workgroup count must be 0 or a positive multiple "
                           "of 8 up to 2^20");
  Launch L{hip_stream};
  const Geo g = geo_of(grid);
  for (int q = 0; q < repeat; ++q) {
    if (precision == TL_FP64)
      k_op_apply<double>(L, g, kernel, blocks, (const double*)d,
                         (const double*)kappa, (const double*)v, (double*)y);
    else
      k_op_apply<float>(L, g, kernel, blocks, (const float*)d,
                        (const float*)kappa, (const float*)v, (float*)y);
  }
  HIP_OK(hipGetLastError());
  HIP_OK(hipStreamSynchronize((hipStream_t)hip_stream));
  return TL_OK;
}

}  // extern "C"
