/*
 * tl.h -- C interface of the MI355X (gfx950) spatiotemporal two-level thermal
 * solver for laser powder-bed fusion (arXiv 2110.12932).
 *
 * The library advances a global (coarse) temperature field on the whole plate
 * and a local (fine) field on a window that follows the laser, with m implicit
 * micro steps of the fine level per coarse macro step (the paper's
 * Algorithm 1, Section 4).  Every step of the path runs in the library's HIP
 * kernels; the caller supplies device memory and a HIP stream.
 *
 * Units are SI throughout (m, s, K, W, J, kg).  All calls return a tl_status;
 * a description of the last failure on the calling thread is available from
 * tl_last_error().  Calls are synchronous with respect to the host: they return
 * after the work they queued on the caller's stream has finished.  A handle
 * must not be used from two host threads at once.
 */
#ifndef TL_H
#define TL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TL_OK = 0,
  TL_EINVAL = -1,   /* invalid argument; nothing was queued on the device    */
  TL_ENOMEM = -2,   /* workspace or host buffer too small                    */
  TL_EDEVICE = -3,  /* a HIP runtime call failed                             */
  TL_ENOCONV = -4,  /* Newton, CG or the two-level iteration did not converge
                       within its cap; the state is rolled back to the last
                       completed macro step                                  */
  TL_ESTATE = -5,   /* call not valid in the handle's current state          */
  TL_EBUSY = -6     /* server queue or slots are full                        */
} tl_status;

/* Arithmetic of the linear solves inside each Newton iteration (TL_MIXED:
 * FP32 CG on both levels).  The nonlinear residual, the Newton iteration,
 * the Dirichlet data, the fields and the energy ledger are always FP64. */
typedef enum { TL_FP64 = 0, TL_MIXED = 1 } tl_precision;

/* Coarse plate [0,lx]x[0,ly]x[0,lz] with nx x ny x nz Q1 cells (spacing
 * lx/nx, ly/ny, lz/nz; z up, laser on z = lz, Dirichlet T_bottom on z = 0,
 * insulated elsewhere).  The fine window covers win_nx x win_ny x win_nz
 * coarse cells, flush with the top surface, each refined `refine` times per
 * axis (refine >= 1).  Requires 1 <= win_* <= n*. */
typedef struct {
  double lx, ly, lz;
  int nx, ny, nz;
  int refine;
  int win_nx, win_ny, win_nz;
} tl_mesh;

/* Material law (paper Section 2): constant density rho; heat capacity c and
 * conductivity kappa linear between (T_lo, c_lo / k_lo) and (T_hi, c_hi /
 * k_hi) and constant outside; latent heat `latent` [J/kg] released by the
 * sigmoid f_pc = (1 + tanh(sharpness (T - (T_sol + T_liq)/2))) / 2.
 * pc_kind must be 0 (the sigmoid).  T_init is the initial temperature of the
 * plate, T_bottom the fixed temperature of its bottom face.
 * Top-surface heat loss (paper Section 2, boundary conditions): the flux
 * h_conv (T - T_amb) [W/m^2] leaves through the top faces of both levels and
 * sigma emissivity (T^4 - T_amb^4) through the fine window's top faces
 * (sigma = 5.670374419e-8); both are lumped onto the faces' corner nodes.
 * h_conv >= 0, 0 <= emissivity <= 1, T_amb > 0; zero h_conv and emissivity
 * give an adiabatic top.
 * k_fict [W/m/K] and rhoc_fict [J/m^3/K] are the global problem's own
 * constant conductivity and volumetric heat capacity inside the window in
 * the consistent global formulation (TL_COUPLE_CONSISTENT, paper Section 3:
 * the global coefficients kappa+, c+ rho+ inside the local domain); 0
 * selects kappa(T_init) and rho c(T_init); both finite and >= 0. */
typedef struct {
  double rho, T_lo, T_hi, c_lo, c_hi, k_lo, k_hi;
  double latent, T_sol, T_liq, sharpness;
  int pc_kind;
  double T_init, T_bottom;
  double h_conv, emissivity, T_amb;
  double k_fict, rhoc_fict;
} tl_material;

/* One straight laser pass from (x0,y0) to (x1,y1) on the top surface at
 * `speed`.  Surface model (TL_SOURCE_SURFACE): the absorbed flux is the
 * surface Gaussian
 *   q = 3 absorptivity power / (pi radius^2) exp(-3 r^2 / radius^2)
 * (the exponent convention of the paper's source terms, Section 5.2).
 * Volume model (TL_SOURCE_VOLUME, the paper's Section 5.2 sources): the
 * fine level takes the volumetric Gaussian
 *   A exp(-3 r^2 / radius^2 - 3 (z - z_top)^2 / depth^2),
 *   A = 6 sqrt(3) absorptivity power / (pi^(3/2) radius^2 depth),
 * normalised so that the half-space below the surface absorbs
 * absorptivity * power; the coarse level takes absorptivity power /
 * (radius depth speed dt_coarse) in the box the beam sweeps during the
 * macro step (speed dt_coarse along the track, radius across it, depth
 * below the top).  depth [m] is used by the volume model only. */
typedef struct {
  double x0, y0, x1, y1, speed, power, radius, absorptivity;
  double depth;
} tl_track;

/* Tracks are run back to back starting at t_start; the beam is off before
 * t_start and after the last track ends.  The array is copied at creation. */
typedef struct {
  int n_tracks;
  const tl_track* tracks;
  double t_start;
} tl_scan_path;

/* How the two-level correction at the end of a macro step is solved (paper
 * Section 3).  TL_COUPLE_DN: the Dirichlet-Neumann iteration -- fine solve
 * with the coarse interface trace, coarse solve outside the window loaded by
 * the restricted fine reactions -- relaxed until the trace settles.
 * TL_COUPLE_COMPOSITE: one Newton solve of the equations that iteration
 * holds at its fixed point, over the free fine nodes and the coarse nodes
 * outside the window interior, the fine interface values slaved to the
 * coarse ones by the trilinear prolongation.  Both give the same discrete
 * solution (to the tolerances).  TL_COUPLE_ALTERNATE: the paper's alternate
 * global formulation -- the global problem over the whole plate keeps only
 * the interface jump term, zero here since both levels share kappa(T), and
 * (as in the paper) no latent heat; the local problem takes all m micro
 * steps with the blended global data and does not feed back.  It is a
 * different discrete problem; its ledger (tl_get_ledger) is the global
 * problem's: stored = sum over coarse nodes of the lumped mass times H(T+)
 * without latent heat, absorbed / bottom / surface of the global solve.
 * TL_COUPLE_CONSISTENT: the paper's consistent global formulation -- the
 * global problem over every coarse element, the window's with the constant
 * coefficients k_fict, rhoc_fict (tl_material), loaded inside the window by
 * the local solution: P^T s with s = rhoc_fict m_k (T-_m - T-_0)/dt_coarse
 * + k_fict (K1 Tavg)_k - (mean local reaction on the interface)_k, which is
 * Section 3's volume and interface-jump terms after the local equation is
 * used (K1: unit-conductivity fine stiffness, Tavg: mean of the m micro-step
 * fields).  It is iterated with the last micro step on the interface
 * values like TL_COUPLE_DN (dn_tol, dn_theta, dn_max apply).  The coarse
 * field keeps its own values inside the window (no injection); the stored
 * energy adds rhoc_fict (sum m_in T+ - sum m_k T-), the energy the global
 * coefficients hold inside the window beyond the local field's. */
typedef enum {
  TL_COUPLE_DN = 0,
  TL_COUPLE_COMPOSITE = 1,
  TL_COUPLE_ALTERNATE = 2,
  TL_COUPLE_CONSISTENT = 3
} tl_coupling;

/* Laser model (see tl_track).  The volume model needs depth > 0 on every
 * track and tracks along x or along y (its boxes are axis-aligned), and at
 * most 8 track pieces per macro step. */
typedef enum { TL_SOURCE_SURFACE = 0, TL_SOURCE_VOLUME = 1 } tl_source;

/* dt_coarse: macro step; m_time: micro steps per macro step (1..32);
 * face_quad: Gauss points per direction for the surface load (1..4);
 * newton_tol [K]: stop when the applied Newton step has max-norm <= tol;
 * cg_rtol: relative reduction of the preconditioned residual norm in each
 * linear solve; dn_tol [K]: two-level iteration stops when the interface
 * update has max-norm <= dn_tol; dn_theta: fixed relaxation when > 0, else
 * interface quasi-Newton (IQN-ILS) acceleration whose first step is relaxed
 * by refine/(refine+1); *_max: iteration caps.  Any relaxation converges to
 * the same fixed point.  coupling: a tl_coupling value (dn_tol, dn_theta and
 * dn_max apply to TL_COUPLE_DN and TL_COUPLE_CONSISTENT only); source: a tl_source value (face_quad
 * applies to TL_SOURCE_SURFACE only). */
typedef struct {
  double dt_coarse;
  int m_time;
  tl_precision precision;
  int face_quad;
  double newton_tol, cg_rtol, dn_tol, dn_theta;
  int newton_max, cg_max, dn_max;
  int coupling;
  int source;
} tl_options;

/* Energy ledger in J (FP64).  stored = sum over coarse nodes of the outside
 * lumped mass times H(T+) plus the same over fine nodes; absorbed = laser
 * energy taken in; bottom = heat that left through the bottom face; remap =
 * energy change caused by window moves; surface = heat that left through
 * the top surface.  Identity (to solver tolerance):
 * stored - stored0 = absorbed - bottom - surface + remap. */
typedef struct {
  double stored, stored0, absorbed, bottom, remap, surface;
} tl_ledger;

/* Counters and timings accumulated over the handle's life. */
typedef struct {
  int64_t macro_steps, micro_steps;
  int64_t newton_fine, newton_coarse;   /* Newton iterations                */
  int64_t cg_fine, cg_coarse;           /* CG iterations                    */
  int64_t line_search_halvings;
  int64_t dn_iters, window_moves;
  int64_t fine_solves, coarse_solves;
  double fine_dof_steps;    /* sum over micro steps of free fine nodes        */
  double step_ms;           /* wall time inside tl_step (host clock)         */
  double fine_op_bytes;     /* algorithmic bytes moved by fine CG operator
                               applies (read v,d,kappa + direction update,
                               write q): the roofline numerator              */
  int64_t fine_op_applies;
  int64_t fine_op_timed;    /* fine CG operator launches timed with events
                               (tl_set_profiling) and their summed duration */
  double fine_op_timed_ms;
  int fine_nodes[3];        /* fine grid nodes per axis                      */
  int coarse_nodes[3];
  int64_t newton_corr, cg_corr;   /* the part of newton_fine / cg_fine spent in
                                     the two-level correction (its fine solves,
                                     or its composite solves)                */
  double phase_ms[4];       /* GPU time of the macro steps' phases while
                               profiling is on (tl_set_profiling): window
                               update, coarse loads and predictor; micro
                               steps 1..m-1; two-level correction; ledger
                               and commit                                    */
} tl_stats;

typedef struct tl_sim tl_sim;

/* Bytes of device workspace tl_create needs for this mesh and options. */
size_t tl_workspace_bytes(const tl_mesh* mesh, const tl_options* opts);

/* Create a simulation (paper Section 2 problem + Algorithm 1 set-up).  All
 * structs and the track array are copied.  dev_workspace: device memory of at
 * least tl_workspace_bytes() bytes, 256-byte aligned, owned by the caller and
 * outliving the handle; the library never allocates device memory.
 * hip_stream: the hipStream_t to queue work on (NULL = default stream).  The
 * initial state is T_init everywhere with T_bottom on the bottom face; the
 * window is placed by the laser position at t_start + dt_coarse.  Errors:
 * TL_EINVAL for inconsistent geometry (window larger than the plate,
 * refine < 1, non-positive sizes), non-finite or non-physical parameters
 * (T_sol >= T_liq, T_lo >= T_hi, rho <= 0, ...), an empty scan path or
 * unsupported options; TL_ENOMEM if ws_bytes is too small. */
tl_status tl_create(const tl_mesh* mesh, const tl_material* material,
                    const tl_scan_path* scan, const tl_options* opts,
                    void* dev_workspace, size_t ws_bytes, void* hip_stream,
                    tl_sim** out);

/* Size of the static device workspace of tl_create_static: 32 MiB, enough
 * for the single-track problems of up to about 90k fine nodes in FP64. */
#define TL_STATIC_WORKSPACE_BYTES (32u * 1024u * 1024u)

/* tl_create for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same simulation, the same kernels and bitwise the same results, with the
 * workspace taken from a static device array of TL_STATIC_WORKSPACE_BYTES
 * that the library holds on every device it runs on until the process ends.
 * Calls no HIP allocator (device or pinned host memory); its host-side
 * tables are plain heap memory.  The array is the current device's;
 * hip_stream (NULL = default stream) must belong to that device (else
 * TL_EINVAL).  Only one handle per device may hold the array at a time: a
 * second tl_create_static on that device before tl_destroy of the first
 * returns TL_EBUSY and leaves the first untouched.  The array keeps the last
 * handle's contents; creation zero-fills it before use.  Problems whose
 * tl_workspace_bytes exceed TL_STATIC_WORKSPACE_BYTES return TL_ENOMEM (use
 * tl_create).  Other errors as for tl_create.  Work queued on the handle and
 * other work on the same array must not overlap: tl_destroy waits for the
 * handle's stream before it gives the array back. */
tl_status tl_create_static(const tl_mesh* mesh, const tl_material* material,
                           const tl_scan_path* scan, const tl_options* opts,
                           void* hip_stream, tl_sim** out);

/* Advance n_macro macro steps (Algorithm 1: window update, coarse predictor,
 * m-1 fine micro steps with time-blended Dirichlet data, two-level
 * correction).  On TL_ENOCONV the state is that of the last completed macro
 * step. */
tl_status tl_step(tl_sim* sim, int n_macro);

/* The two temperature fields of the method (paper Section 3): the global
 * field T+ on the coarse plate (level 0) and the local field T- on the fine
 * window (level 1), at the end of the last completed macro step.  Copies the
 * field to host_out (host memory owned by the caller), node (i,j,k) at
 * i + nx*(j + ny*k) with (nx,ny,nz) = dims_out.  With the Dirichlet-Neumann
 * or composite correction, the coarse nodes strictly inside the window hold
 * the injected fine values; with the alternate or consistent formulation
 * they hold the global problem's own values.  cap is the capacity of host_out in doubles
 * (TL_ENOMEM if too small, nothing copied); TL_EINVAL for a null handle or
 * buffer or a level other than 0 or 1.  fine_origin_out (may be NULL)
 * receives the fine-grid index of the window's first node on the plate-wide
 * fine lattice (refine * coarse cell origin). */
tl_status tl_get_temperature(tl_sim* sim, int level, double* host_out,
                             size_t cap, int dims_out[3],
                             int fine_origin_out[3]);

/* Energy balance of the thermal model (paper Section 2: enthalpy change =
 * absorbed laser heat - heat through the plate bottom - top-surface loss),
 * accumulated over the completed macro steps; see tl_ledger for the terms
 * and the identity they satisfy.  TL_EINVAL for null arguments. */
tl_status tl_get_ledger(tl_sim* sim, tl_ledger* out);

/* Counters and timings (tl_stats) over the handle's life.  TL_EINVAL for
 * null arguments. */
tl_status tl_get_stats(tl_sim* sim, tl_stats* out);

/* Simulation time of the committed state and the number of macro steps. */
tl_status tl_get_time(tl_sim* sim, double* t, int64_t* n_macro);

/* Checkpoint: serialise the committed state (coarse and fine temperatures,
 * window origin, step counter, ledger, stats) and the solver history later
 * steps depend on (two-level quasi-Newton secant pairs, CG budgets) into
 * host memory, so that a restored run continues exactly as the saved one;
 * *used receives the byte count (call with host = NULL to query; the count
 * changes as the history grows).  tl_load restores a buffer written by
 * tl_save for a handle created with the same mesh and options; a buffer of
 * another format or grid, a truncated one, or one whose window or solver
 * history does not fit the handle returns TL_EINVAL and leaves the handle
 * as it was. */
tl_status tl_save(tl_sim* sim, void* host, size_t cap, size_t* used);
tl_status tl_load(tl_sim* sim, const void* host, size_t n);

/* Time every sample_every-th launch of the fine CG operator kernel (the
 * fused direction update and matrix-free operator apply) with HIP events on
 * the handle's stream; the count and summed duration appear in tl_stats,
 * and so do the GPU times of each macro step's phases (phase_ms).  0
 * switches timing off (the default). */
tl_status tl_set_profiling(tl_sim* sim, int sample_every);

void tl_destroy(tl_sim* sim);

/* Message of the last failing call on this thread ("" if none). */
const char* tl_last_error(void);

/* ---- serving: continuous batching of many simulations ------------------- *
 * A server owns a caller-provided device pool.  Submitted requests wait in
 * arrival order; each tl_server_tick admits waiting requests while a slot is
 * free and the request's footprint (tl_workspace_bytes) fits the HBM budget
 * and the pool, then advances every active request by one macro step --
 * all their fine and coarse implicit steps as batched launches -- and
 * retires requests that reached their macro-step count, copying their
 * temperatures, ledger and counters to host memory and returning their
 * workspace to the pool.  A request's result does not depend on which other
 * requests share its ticks. */
typedef struct tl_server tl_server;

/* Host-clock record of one request (seconds since tl_server_create). */
typedef struct {
  double submit_s, admit_s, done_s;  /* -1 when not reached yet */
  int state;                         /* 0 queued, 1 active, 2 done, 3 failed */
  int pad;
  int64_t macro_steps;               /* macro steps run (done requests) */
} tl_request_info;

/* Device bytes the server keeps for its own tables (part of the pool). */
size_t tl_server_overhead_bytes(int max_slots);

/* dev_pool: caller-owned device memory of pool_bytes, 256-byte aligned,
 * outliving the server; hbm_budget caps the summed footprint of active
 * requests; max_slots caps their number (1..1024).  TL_ENOMEM if the pool
 * cannot hold the server's tables. */
tl_status tl_server_create(void* dev_pool, size_t pool_bytes,
                           size_t hbm_budget, int max_slots, void* hip_stream,
                           tl_server** out);

/* Queue a request of n_macro macro steps of the paper's Algorithm 1 (the
 * request ends at t_start + n_macro * dt_coarse); inputs are copied.  The
 * horizon is a step count rather than an end time so that the number of
 * macro steps, and with it the request's result, never depends on how an
 * end time rounds against dt_coarse.  TL_EINVAL as for tl_create or for
 * n_macro < 1; TL_EBUSY if the request alone exceeds the budget. */
tl_status tl_server_submit(tl_server* sv, const tl_mesh* mesh,
                           const tl_material* material,
                           const tl_scan_path* scan, const tl_options* opts,
                           int n_macro, uint64_t* id);

/* Admit, advance all active requests by one macro step, retire finished
 * ones.  Outputs (may be NULL): active and queued counts after the tick,
 * requests finished (done or failed) during it.  TL_EDEVICE on a HIP
 * error (the server is then unusable). */
tl_status tl_server_tick(tl_server* sv, int* n_active, int* n_queued,
                         int* n_finished);

/* Results of a finished request: temperature of `level` (as
 * tl_get_temperature; host_out may be NULL), counters, ledger, timing.
 * TL_EBUSY while queued or active; TL_ENOCONV with the message if it
 * failed (info is filled in every case). */
tl_status tl_server_result(tl_server* sv, uint64_t id, int level,
                           double* host_out, size_t cap, int dims_out[3],
                           tl_stats* st, tl_ledger* led,
                           tl_request_info* info);

/* Time every sample_every-th launch of the batched fine CG kernel with HIP
 * events attached to the dispatch (0: off); tl_server_get_profile returns
 * the number of timed launches that did work and their summed duration. */
tl_status tl_server_set_profiling(tl_server* sv, int sample_every);
tl_status tl_server_get_profile(tl_server* sv, int64_t* launches, double* ms);

/* Drop the host-side results of a finished request. */
tl_status tl_server_release(tl_server* sv, uint64_t id);

void tl_server_destroy(tl_server* sv);

#ifdef __cplusplus
}
#endif
#endif /* TL_H */
