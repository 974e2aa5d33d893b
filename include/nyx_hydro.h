/*
 * nyx_hydro.h -- C ABI of the MI355X (gfx950) comoving gas step.
 *
 * The library advances the gas state of Nyx (Almgren et al.) by one time step
 * on ghost-filled boxes: the unsplit PPM Godunov method with characteristic
 * tracing and full corner coupling, the iterative two-shock Riemann solver,
 * the conservative update with the expansion-factor and gravity sources, the
 * gravity corrector and the dual-energy sync (Sec. 3.2 Gas Dynamics, Sec. 3.6
 * Single-Level Integration Algorithm, Steps 2 and 6), and the hydro CFL time
 * step (Sec. 3.5).  Around the step it provides the level operations that
 * prepare its inputs and follow it: the ghost fill of an AMR level (Sec. 4.1,
 * with time interpolation for subcycling, Sec. 4.2), the two-level reflux and
 * average-down (Sec. 4.3) and the mesh side of the gravity input (Sec. 3.4).
 *
 * Conventions shared by every entry point
 *  - State U (Sec. 3.2): 6 components (rho, a rho U_x, a rho U_y, a rho U_z,
 *    a^2 rho E, a^2 rho e), FP64.  Gravity g: 3 components, FP64 in
 *    NYX_FP64 mode, FP32 in NYX_MIXED mode.
 *  - Box layout: n = (nx, ny, nz) valid cells (each even and >= 2; Sec. 4.1
 *    asks for an even number of cells per direction), ng >= 4 ghost cells on
 *    every side, component-major with x fastest:
 *      element (c, k, j, i) at off + c*comp_stride
 *                            + ((k+ng)*(ny+2ng) + (j+ng))*(nx+2ng) + (i+ng)
 *    for i in [-ng, nx+ng) and likewise j, k; comp_stride >= the padded cell
 *    count, which must stay below 2^29 (a box of up to about 800^3 cells;
 *    per-box offsets are 32-bit byte offsets).  dx is the comoving cell size,
 *    the same on every axis (Sec. 4.1).
 *  - Memory: every pointer marked (device) is device memory owned by the
 *    caller; the library never allocates or frees device memory.  Workspace
 *    sizes are queried first and passed in.  Host pointers are read during
 *    the call only.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls
 *    only enqueue work, except where an entry point says it synchronises
 *    (plan creation, autotuning, the Poisson solve's convergence checks).
 *    A plan and its workspace serve one stream at a time: calls on one plan
 *    that overlap on two streams race on its workspace.
 *  - Errors: argument errors return a negative nyx_status before anything is
 *    enqueued.  Conditions met on the device (non-finite values, rho <= 0,
 *    floors, rejected transverse corrections, learned-flux fallbacks) are only
 *    counted in an optional device nyx_stats block; values are never clamped
 *    silently.  No C++ exception crosses this interface.
 *  - The input state is U^n scaled with a_old, the output U^{n+1} scaled with
 *    a_new (Sec. 3.2); only valid cells of the output are written, so the
 *    caller refills its ghost cells before the next step.  Input and output
 *    must not overlap.
 */
#ifndef NYX_HYDRO_H
#define NYX_HYDRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NYX_OK = 0,
  NYX_E_NULL = -1,        /* a required pointer is NULL */
  NYX_E_SHAPE = -2,       /* box extents, ghost width or strides invalid */
  NYX_E_PARAM = -3,       /* dt, a, dx, cfl, gamma or an enum out of range */
  NYX_E_ALIAS = -4,       /* input and output state overlap */
  NYX_E_HIP = -5,         /* a HIP launch or runtime call failed */
  NYX_E_UNSUPPORTED = -6, /* combination not built into this library */
  NYX_E_WORKSPACE = -7,   /* workspace too small or misaligned */
  NYX_E_SCRATCH = -8      /* box too large for nyx_hydro_step_noalloc's scratch */
} nyx_status;

typedef enum { NYX_FP64 = 0, NYX_MIXED = 1 } nyx_precision;
/* Riemann solver of the faces (Sec. 3.2): the iterative two-shock solver;
 * the learned flux (this library's addition, with the two-shock solver as
 * fallback); or the simpler linearised approximate solver Sec. 3.2 compares
 * against: acoustic star state p* = (W_R p_L + W_L p_R + W_L W_R (u_L -
 * u_R))/(W_L + W_R), u* = (W_L u_L + W_R u_R + p_L - p_R)/(W_L + W_R) with
 * W_K = sqrt(gamma p_K rho_K), rho*_K = rho_K + (p* - p_K)/c_K^2, sampled
 * with the two-shock wave structure, no iteration. */
typedef enum {
  NYX_RIEMANN_TWOSHOCK = 0,
  NYX_RIEMANN_LEARNED = 1,
  NYX_RIEMANN_LINEARIZED = 2
} nyx_riemann;
/* Reconstruction of the time-centred edge states (Sec. 3.2): unsplit PPM, or
 * unsplit piecewise linear (limited centred slopes times the flattening
 * coefficient); both are traced with the reference state of Sec. 3.2. */
typedef enum { NYX_RECON_PPM = 0, NYX_RECON_PLM = 1 } nyx_recon;

typedef struct {
  double gamma;          /* gamma-law exponent, > 1 (Sec. 2.2: 5/3).  For any
                          * other value the a adot (2 - 3(gamma-1)) rho e term of
                          * both energy equations (Sec. 2.2) is applied, at a_old
                          * in the predictor and time-centred by the corrector */
  double eta_dual;       /* dual-energy threshold (Sec. 3.6 Step 6: 1e-4) */
  double small_dens;     /* density floor of primitives and edge states */
  double small_pres;     /* pressure floor of primitives, edge states, Riemann */
  double riemann_tol;    /* relative stopping tolerance of the two-shock iteration;
                          * the FP32-mixed form stores the star state in FP32 and
                          * stops once a Newton step is below
                          * max(sqrt(riemann_tol), 2^-12) of the pressure */
  double mlp_resid_tol;  /* learned flux: accepted two-shock residual (tau_r) */
  double cfl;            /* hydro CFL factor used for dt_next (Sec. 3.5) */
  int32_t riemann_maxiter;     /* 1..64 */
  int32_t precision;           /* nyx_precision */
  int32_t riemann;             /* nyx_riemann */
  int32_t learned_stages_mask; /* bit s set: stage s (0, 1, 2) uses the MLP */
  int32_t recon;               /* nyx_recon */
  int32_t grav_energy_form;    /* energy gravity term (Sec. 3.2): 1 = (aρU).g at
                                * cell centres; 2 = the update of a^2 rho E is
                                * the update of the kinetic energy the gravity
                                * momentum terms cause */
  const void* mlp_weights;     /* (device) packed learned-flux weights, or NULL */
  double mixed_riemann_stop;   /* FP32-mixed: relative Newton step below which the
                                * two-shock iteration stops; 0 selects the default
                                * max(sqrt(riemann_tol), 2^-12) (the star state is
                                * stored in FP32); riemann_tol gives the FP64 form's
                                * own rule */
} nyx_params;

typedef struct {
  int32_t n[3];          /* valid cells per axis */
  int32_t ng;            /* ghost cells per side, >= 4 */
  int64_t state_off;     /* element offset of (c=0, k=-ng, j=-ng, i=-ng) */
  int64_t grav_off;      /* same for the gravity buffer */
  int64_t comp_stride;   /* elements between state components */
  int64_t grav_stride;   /* elements between gravity components */
  double dx;             /* comoving cell size */
} nyx_box;

/* Device counters, accumulated with atomics; zero them before a step. */
typedef struct {
  unsigned long long nonfinite, neg_dens, neg_eint, floor_hits, trans_reverts,
      sync_E_from_e, riemann_iters, riemann_calls, mlp_used, mlp_fallback;
} nyx_stats;

/* Default parameters: gamma 5/3, eta 1e-4, floors 1e-20, tol 1e-14, 20
 * iterations, cfl 0.5, FP64, two-shock solver. */
void nyx_default_params(nyx_params* p);

/* Human-readable text of a status code (static storage). */
const char* nyx_status_string(int status);

/* Bytes of workspace nyx_hydro_step needs for this box and precision. */
int nyx_workspace_bytes(const nyx_params* p, const nyx_box* box, size_t* bytes);

/* Hydro CFL time step of one box (Sec. 3.5):
 *   dt = cfl * a * dx / max over valid cells and axes of (|U_d| + c),
 * with U_d = (a rho U_d)/(a rho) and c from the internal-energy slot.
 * state (device, FP64); dt_out (device, one double).  The maximum is exact,
 * so the result does not depend on the reduction order.  Uses `workspace`
 * (>= 16 bytes, device) for the running maximum. */
int nyx_estimate_dt(const nyx_params* p, const nyx_box* box, const double* state,
                    double a, double cfl, double* dt_out, void* workspace,
                    size_t ws_bytes, void* stream);

/* One gas step of one box (Sec. 3.6 Steps 2 and 6).
 * state_in, state_out (device, FP64, same layout, not overlapping); grav
 * (device, FP64 or FP32 per p->precision); dt > 0 and a_old, a_new > 0 are
 * host values.  dt_next (device, one double, or NULL): CFL time step of the
 * new state at a_new with p->cfl.  stats (device or NULL).  workspace
 * (device, 256-byte aligned) of at least nyx_workspace_bytes. */
int nyx_hydro_step(const nyx_params* p, const nyx_box* box, const double* state_in,
                   const void* grav, double dt, double a_old, double a_new,
                   double* state_out, double* dt_next, nyx_stats* stats,
                   void* workspace, size_t ws_bytes, void* stream);

/* The same step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no workspace argument.  The stage arrays live in a library-held device
 * array of nyx_noalloc_max_bytes() bytes (64 MiB), one per GPU, held until
 * the process ends; the call allocates nothing (no hipMalloc, no events).
 * A box whose nyx_workspace_bytes exceed it returns NYX_E_SCRATCH (FP64 up
 * to about 40^3 valid cells, FP32-mixed up to about 50^3).  Every call on a
 * GPU shares that GPU's array and leaves its contents there: calls that
 * overlap on one GPU (two streams, two threads) race on it; the counters and
 * the CFL maximum it holds are cleared by each call.  Other arguments,
 * results and errors are those of nyx_hydro_step, bit for bit. */
int nyx_hydro_step_noalloc(const nyx_params* p, const nyx_box* box, const double* state_in,
                           const void* grav, double dt, double a_old, double a_new,
                           double* state_out, double* dt_next, nyx_stats* stats,
                           void* stream);
/* Bytes of the scratch array of nyx_hydro_step_noalloc. */
int nyx_noalloc_max_bytes(size_t* bytes);

/* ---------------- batched boxes (one AMR level) ----------------
 * A plan describes a list of boxes living in shared state / gravity buffers
 * (each box at its own offsets).  The plan is host memory created once per
 * box layout; its device tables live in the caller's workspace.  Boxes are
 * advanced together: every stage runs as one launch over all boxes of a
 * group, groups being sized to fit the workspace.  dt is read per box from
 * device memory, so a captured HIP graph can be replayed step after step. */
typedef struct nyx_batch nyx_batch;

/* Minimum workspace (all boxes in groups of one) and the size that holds all
 * boxes in a single group. */
int nyx_batch_workspace_bytes(const nyx_params* p, int nbox, const nyx_box* boxes,
                              size_t* min_bytes, size_t* single_group_bytes);

/* Build a plan; uploads its tables into `workspace` on `stream` (the host
 * array is copied before return).  *out is freed with nyx_batch_destroy. */
int nyx_batch_create(const nyx_params* p, int nbox, const nyx_box* boxes,
                     void* workspace, size_t ws_bytes, void* stream, nyx_batch** out);
int nyx_batch_destroy(nyx_batch* plan);
int nyx_batch_num_groups(const nyx_batch* plan);

/* Per-box CFL time steps into dt (device, nbox doubles). */
int nyx_batch_estimate_dt(nyx_batch* plan, const double* state, double a, double cfl,
                          double* dt, void* stream);

/* Replace every entry of dt (device, nbox doubles) by their minimum: one level
 * time step for all boxes. */
int nyx_batch_min_dt(nyx_batch* plan, double* dt, void* stream);

/* One step of every box of the plan: the gas step of Sec. 3.6 (Step 2
 * predictor, Step 6 gravity corrector and dual-energy sync) applied to each
 * grid of a level, a level being a union of non-overlapping boxes with
 * ghost cells (Sec. 4.1), each advanced with its own time step (the hydro
 * CFL of Sec. 3.5 per box, or one level dt after nyx_batch_min_dt).
 * state_in, state_out (device, FP64) hold every box at its own offsets and
 * must not overlap; grav (device, FP64 or FP32 per precision); dt (device,
 * nbox doubles, read on the device, so a captured graph replays step after
 * step); dt_next (device, nbox doubles, or NULL) receives each box's CFL step
 * of the new state at a_new; stats (device or NULL) sums the counters of all
 * boxes.  Each box's result is bit for bit that of nyx_hydro_step on it,
 * whatever the grouping and launch orders.  Errors: NYX_E_NULL for a missing
 * plan or buffer, NYX_E_PARAM for a_old, a_new <= 0, NYX_E_ALIAS for
 * overlapping states; nothing is enqueued then. */
int nyx_hydro_step_batched(nyx_batch* plan, const double* state_in, const void* grav,
                           const double* dt, double a_old, double a_new,
                           double* state_out, double* dt_next, nyx_stats* stats,
                           void* stream);

/* ---------------- launch mode of a plan ----------------
 * NYX_LAUNCH_STAGED (the default): every stage of a group is its own launch
 * over all boxes of the group.  NYX_LAUNCH_PERSISTENT: the seven stages of a
 * group run as one launch of as many workgroups as the device keeps
 * resident at once; per stage, each workgroup first runs a static,
 * contiguous share of the work items (the blocks of the staged launch), then
 * takes the rest in chunks from atomic queues, one per XCD's range, which the
 * workgroups of that XCD drain first; a two-level grid barrier (per XCD, then
 * across XCDs) separates the stages.  Each item runs the staged kernel's code, so every box's result
 * is bit for bit that of the staged launches.  The barrier gives up after 5 s
 * of wall clock if some workgroup never became resident (another kernel
 * holding the device); the launch then ends early, and
 * nyx_batch_persistent_aborted reports it.  Available for plain steps in
 * both precisions and for the learned flux on all three stages; a plan that
 * harvests training records runs staged.  Stage timing (nyx_profile_*) sees
 * only the staged and fused launches.
 * NYX_LAUNCH_FUSED: staged launches, except for two fusions.  The last two
 * stages (the final Riemann solves of Sec. 3.2 and the conservative update
 * with the gravity corrector and the dual-energy sync of Sec. 3.6, Steps 2
 * and 6) run as one launch: a workgroup takes a tile of cell columns of a box
 * and marches up the box in z, solving each final face once (plus the faces
 * past the tile's last column and row) and updating every cell as soon as
 * its six faces are known, so the final face states never reach HBM.  And
 * the tracing and the first Riemann solves of x run as one launch: each lane
 * traces one cell and solves the x-face below it with the edge state its
 * neighbouring lane just traced (y and z keep their staged launches).  Bit
 * for bit the result of the staged launches.  A plan that uses the learned
 * flux on the final stage, harvests training records or feeds flux
 * registers runs the last two stages staged, and one with the learned flux
 * on the first solves runs those staged; nyx_profile_* reports each fused
 * launch as its first stage (the x front with the y, z tracing as stage 3)
 * and a shorter or zero-length second stage. */
enum { NYX_LAUNCH_STAGED = 0, NYX_LAUNCH_PERSISTENT = 1, NYX_LAUNCH_FUSED = 2 };
/* NYX_E_UNSUPPORTED when the persistent mode is not available for the
 * plan's parameters. */
int nyx_batch_set_launch_mode(nyx_batch* plan, int mode);
int nyx_batch_get_launch_mode(const nyx_batch* plan, int* mode);
/* *aborted = 1 if the last persistent launch of the plan gave up at a grid
 * barrier (synchronises `stream`). */
int nyx_batch_persistent_aborted(nyx_batch* plan, int* aborted, void* stream);
/* Times `reps` whole steps (after one untimed) in each available mode with
 * the plan's current launch orders and keeps the fastest; ms_out[3] (host,
 * or NULL) receives the best step time of each mode (-1: not available);
 * *mode_out (or NULL) the mode kept.  Synchronises `stream`. */
int nyx_batch_autotune_mode(nyx_batch* plan, const double* state_in, const void* grav,
                            const double* dt, double a_old, double a_new, double* state_out,
                            int reps, float* ms_out, int* mode_out, void* stream);

/* ---------------- launch-order autotuning of a plan ----------------
 * Each of the NYX_NSTAGES stage kernels of a plan's step walks its cells in
 * one of NYX_TUNE_CANDIDATES launch orders (fields of a tuning entry):
 *   NYX_TUNE_CELL_MAJOR  kernels with one launch row per direction walk the
 *                        directions of one range of cells back to back (the
 *                        stage arrays the directions share are then reread
 *                        through one L2) instead of one direction after the
 *                        other;
 *   NYX_TUNE_HW_ORDER    the hardware's workgroup order instead of numbering
 *                        the workgroups so that each XCD walks one contiguous
 *                        range of the grid;
 *   bits NYX_TUNE_SLAB_SHIFT.. (0-3): cell order within a box, 0 plane by
 *                        plane; s > 0 tiles of 2^(s+2) rows, each walked
 *                        plane by plane along z (z-pencils of row tiles), so
 *                        that a cell's z-neighbours are read soon after it.
 * The order changes no result bit (every cell and face computes the same
 * expressions).  A new plan uses entry 0 for every stage.
 *
 * nyx_batch_autotune runs reps + 1 steps per candidate with the arguments of
 * nyx_hydro_step_batched (no counters; state_out and dt_next, when not NULL,
 * receive the step's results; pass dt_next when the tuned steps will produce
 * it, since the fused CFL maximum is part of the update stage's time), times
 * every stage from HIP events around its launches,
 * keeps the fastest candidate per stage in the plan and returns it in
 * tune_out[NYX_NSTAGES] (host, or NULL); ms_out (host, NYX_NSTAGES x
 * NYX_TUNE_CANDIDATES floats, or NULL) receives each stage's fastest
 * repetition per candidate, in milliseconds.  It synchronises the stream and must not be called
 * while the stream is being captured.  nyx_batch_set_tuning /
 * nyx_batch_get_tuning store and read a plan's entries (host arrays of
 * NYX_NSTAGES ints in 0..NYX_TUNE_CANDIDATES-1), e.g. from a cache of earlier
 * tuning runs. */
#define NYX_TUNE_CELL_MAJOR 1
#define NYX_TUNE_HW_ORDER 2
#define NYX_TUNE_SLAB_SHIFT 2
#define NYX_TUNE_CANDIDATES 16
int nyx_batch_autotune(nyx_batch* plan, const double* state_in, const void* grav,
                       const double* dt, double a_old, double a_new, double* state_out,
                       double* dt_next, int reps, float* ms_out, int* tune_out, void* stream);
int nyx_batch_set_tuning(nyx_batch* plan, const int* tune);
int nyx_batch_get_tuning(const nyx_batch* plan, int* tune);

/* ---------------- ghost fills (outside the step) ---------------- */
/* Periodic ghost cells of one box from its own valid cells (the box is its
 * own periodic domain).  state (device), ncomp components at box->state_off
 * with box->comp_stride. */
int nyx_fill_ghosts_periodic(const nyx_box* box, double* state, int ncomp, void* stream);

/* Ghost fill of every box of a plan (6 state components):
 *   mode 0: each box is its own periodic domain;
 *   mode 1: the boxes tile a periodic domain as a gx*gy*gz grid of equal
 *           boxes, box b = (bz*gy + by)*gx + bx, and ghosts are copied from
 *           the neighbouring boxes' valid cells (the same-level ghost fill of
 *           Sec. 4.1 for one uniform level). */
int nyx_batch_fill_ghosts(nyx_batch* plan, int mode, int gx, int gy, int gz, double* state,
                          void* stream);

/* Where later steps of a plan take the input state's ghost cells (Sec. 4.1:
 * a level's ghost cells hold copies of the cells they stand for):
 *   mode -1: from the input's own ghost cells (the default; the caller fills
 *            them, e.g. with nyx_batch_fill_ghosts);
 *   mode 0:  from each box's own valid cells, the box being its own periodic
 *            domain;
 *   mode 1:  from the neighbouring boxes' valid cells, the boxes tiling a
 *            periodic domain as a gx*gy*gz grid as in nyx_batch_fill_ghosts
 *            mode 1 (grid checked here: NYX_E_SHAPE).
 * Modes 0 and 1 give the step the same result as filling the input's ghosts
 * with nyx_batch_fill_ghosts in that mode first, bit for bit, without reading
 * or writing the input's ghost cells; the output's ghost cells are then left
 * as they were.  Only the primitive stage reads ghost cells of the state.
 * Other modes: NYX_E_PARAM. */
int nyx_batch_set_ghost_source(nyx_batch* plan, int mode, int gx, int gy, int gz);

/* ---------------- ghost fill of an AMR level (Sec. 4.1) ----------------
 * A level is nbox boxes of one cell size in a periodic domain of dom[3]
 * cells (host, 3 ints, each even and at least the ghost width).  lo (host,
 * 3*nbox ints) gives the global index of each box's valid cell (0,0,0); the
 * boxes' valid regions must not overlap, and all boxes share one ghost
 * width.  Every ghost cell of every box is filled:
 *   - from the valid cell of the level that covers it (periodic images
 *     included), copied bit for bit;
 *   - otherwise from the level below (refinement ratio 2, domain dom/2;
 *     cboxes/clo, ncoarse >= 1, its own ghost cells already filled) by the
 *     limited linear profile of the coarse cell X = floor(x/2) at the fine
 *     cell centre: per direction the MC-limited centred difference of X and
 *     its two neighbours, all three slopes scaled by the largest factor in
 *     [0, 1] that keeps the eight children of X within the minimum and
 *     maximum over X and its six face neighbours, and the child value
 *     U(X) + sum_d (-/+ s_d / 4).  The children average to U(X) (the
 *     interpolation conserves), and create no new extrema.
 * A ghost cell covered by neither level (improper nesting, or ncoarse = 0)
 * is a NYX_E_SHAPE error of the plan.  The host plans once per box layout
 * (nyx_fill_plan_bytes, nyx_fill_plan_create: the plan's tables live in the
 * caller's device workspace, 256-byte aligned; create synchronises the
 * stream); nyx_fill_level then enqueues the fill of ncomp components of
 * the FP64 state (device; each box at its state_off with its comp_stride)
 * from coarse_state (device, or NULL without a coarse level; it must not
 * overlap the fine state). */
typedef struct nyx_fill_plan nyx_fill_plan;
int nyx_fill_plan_bytes(int nbox, const nyx_box* boxes, const int32_t* lo, const int32_t* dom,
                        int ncoarse, const nyx_box* cboxes, const int32_t* clo, size_t* bytes);
int nyx_fill_plan_create(int nbox, const nyx_box* boxes, const int32_t* lo, const int32_t* dom,
                         int ncoarse, const nyx_box* cboxes, const int32_t* clo, void* workspace,
                         size_t ws_bytes, void* stream, nyx_fill_plan** plan);
int nyx_fill_plan_counts(const nyx_fill_plan* plan, long long* copied, long long* interpolated);
int nyx_fill_level(nyx_fill_plan* plan, double* state, const double* coarse_state, int ncomp,
                   void* stream);
/* The same fill at an intermediate time of a subcycled fine level (Sec.
 * 4.2): every coarse value the interpolation reads is
 * coarse_state + theta (coarse_state_new - coarse_state), with theta in
 * [0, 1] the fine time's fraction of the coarse step (else NYX_E_PARAM);
 * coarse_state_new (device, the coarse level at the end of its step, same
 * layout, ghosts filled) may be NULL, which is nyx_fill_level. */
int nyx_fill_level_time(nyx_fill_plan* plan, double* state, const double* coarse_state,
                        const double* coarse_state_new, double theta, int ncomp, void* stream);
int nyx_fill_plan_destroy(nyx_fill_plan* plan);

/* ---------------- two-level synchronisation (Sec. 4.3) ----------------
 * After a coarse level has taken a step and the fine level above it
 * (refinement ratio 2) its substeps, the multilevel algorithm (Sec. 4.3,
 * Steps 2 and 8) refluxes the coarse cells next to the fine level, so that
 * the composite solution conserves what the fine fluxes moved, and then
 * averages the fine solution down onto the coarse cells it covers.
 *
 * Geometry: the fine level is nfine boxes (lo: global index of valid cell
 * (0,0,0), 3 ints per box; lo and n even) in a periodic domain of dom
 * cells (even); the coarse level is ncoarse boxes in the domain dom / 2.
 * Boxes lie inside their domain and do not overlap within a level.  A coarse
 * cell is covered when its eight children lie in a fine box.  Every
 * uncovered face neighbour of a covered cell must lie in a coarse box
 * (proper nesting), else NYX_E_SHAPE.
 *
 * Flux register: one slot per interface face (a coarse face with exactly
 * one covered side, periodic images included), 6 FP64 components stored
 * component-major: reg[c * faces + slot] (device, caller-zeroed before the
 * coarse step).  nyx_batch_set_flux_register attaches it to a batch plan
 * whose boxes are the sync plan's coarse boxes (level 0) or fine boxes
 * (level 1), in the same order and shapes; every later
 * nyx_hydro_step_batched of that plan then adds, per interface face, its
 * final comoving flux F (Sec. 3.2 flux vector) times -dt (level 0: the
 * face's flux in the box of the uncovered cell) or times dt / 4 summed over
 * the four fine faces (level 1), so that after one coarse step and the fine
 * substeps reg = sum_s dt_s <F_fine> - dt_c F_coarse.  reg = NULL detaches
 * it.  nyx_batch_autotune does not feed the register.
 *
 * nyx_reflux adds to each uncovered coarse cell next to the fine level the
 * sum over its interface faces (in the order x-, x+, y-, y+, z-, z+) of
 * +reg (the cell's low face) or -reg (its high face), divided by the coarse
 * box's dx, for the first ncomp components.  nyx_average_down sets each
 * covered coarse cell to the mean of its eight children (ncomp components;
 * fine and coarse states must not overlap).  Plans, like fill plans, keep
 * their tables in the caller's device workspace (256-byte aligned;
 * nyx_sync_plan_create synchronises the stream); a batch plan that feeds a
 * register reads the sync plan's tables, so both must outlive that use. */
typedef struct nyx_sync_plan nyx_sync_plan;
int nyx_sync_plan_bytes(int nfine, const nyx_box* fboxes, const int32_t* flo, const int32_t* dom,
                        int ncoarse, const nyx_box* cboxes, const int32_t* clo, size_t* bytes);
int nyx_sync_plan_create(int nfine, const nyx_box* fboxes, const int32_t* flo, const int32_t* dom,
                         int ncoarse, const nyx_box* cboxes, const int32_t* clo, void* workspace,
                         size_t ws_bytes, void* stream, nyx_sync_plan** plan);
int nyx_sync_plan_counts(const nyx_sync_plan* plan, long long* faces, long long* reflux_cells,
                         long long* covered_cells);
int nyx_sync_plan_destroy(nyx_sync_plan* plan);
int nyx_batch_set_flux_register(nyx_batch* plan, const nyx_sync_plan* sync, int level,
                                double* reg);
int nyx_reflux(nyx_sync_plan* plan, double* coarse_state, const double* reg, int ncomp,
               void* stream);
int nyx_average_down(nyx_sync_plan* plan, double* coarse_state, const double* fine_state,
                     int ncomp, void* stream);

/* ---------------- gravity input of the step (Sec. 2.4, Sec. 3.4) ----------------
 * The mesh side of self-gravity on a periodic domain of dom[3] cells (each
 * even, at most 2^16, product below 2^31) of size dx.  Mesh fields (rho,
 * phi) are FP64 device arrays of the domain, x fastest, no ghost cells;
 * cell (i, j, k) is centred at ((i + 1/2) dx, ...).
 *
 * nyx_cic_deposit adds the cloud-in-cell comoving density of np particles
 * to rho: a particle's mass is spread uniformly over a cube of side dx
 * centred at it, each cell receives the mass times the volume of its
 * intersection with the cube, divided by dx^6 (dx^3 for the fraction, dx^3
 * for a density).  pos: device, three arrays of np positions (x, then y,
 * then z; taken periodically; a particle with a non-finite coordinate, or
 * one beyond 1e15 cells, is skipped); mass: device, np values.
 * The additions use FP64 atomics: the result is exact up to their order.
 *
 * nyx_poisson_solve solves lap7(phi) = coef (rho_t - mean(rho_t)), lap7 the
 * 7-point Laplacian, rho_t = rho plus, when state is not NULL, the gas
 * density (component 0) of the state of box `box` (host; a box of dom
 * cells: the whole domain as one padded box).  coef is 4 pi G / a
 * (Sec. 2.4).  Geometric multigrid: V-cycles with two red-black
 * Gauss-Seidel sweeps before and after the coarse correction, averaging
 * restriction of the residual, trilinear cell-centred prolongation, levels
 * halved while every extent is a multiple of 4, 32 sweeps on the coarsest.
 * phi (device) is the initial guess on entry (the previous solution serves,
 * Sec. 3.4) and the zero-mean solution on return.  The cycles stop once
 * max|rhs - lap7 phi| <= tol max|rhs| (the paper's typical tol is 1e-12;
 * FP64 rounding of the residual limits what large meshes can reach) or
 * after max_vcycles.  With tol > 0 or rel_resid given, the call
 * synchronises the stream once per V-cycle; with tol = 0 and rel_resid NULL
 * it runs exactly max_vcycles cycles and only enqueues kernels.  vcycles
 * and rel_resid (host, or NULL) receive the cycles run and the final
 * relative residual.  workspace: device, nyx_poisson_workspace_bytes
 * bytes, 256-byte aligned.  Every reduction has a fixed order: the same
 * inputs give the same bits.
 *
 * nyx_gravity_from_phi writes g = -(phi(c + e_d) - phi(c - e_d)) / (2 dx)
 * into every padded cell of box `box` (host; dom cells; ghosts are the
 * periodic images) of grav (device), at box->grav_off with box->grav_stride,
 * in FP64 (precision NYX_FP64) or FP32 (NYX_MIXED): the gravity input of a
 * step of that box. */
int nyx_cic_deposit(const double* pos, const double* mass, long long np, const int32_t* dom,
                    double dx, double* rho, void* stream);
int nyx_poisson_workspace_bytes(const int32_t* dom, size_t* bytes);
int nyx_poisson_solve(const int32_t* dom, double dx, double coef, const double* rho,
                      const double* state, const nyx_box* box, double* phi, double tol,
                      int max_vcycles, void* workspace, size_t ws_bytes, void* stream,
                      int* vcycles, double* rel_resid);
int nyx_gravity_from_phi(const int32_t* dom, double dx, const double* phi, const nyx_box* box,
                         void* grav, int precision, void* stream);

/* ---------------- learned Riemann flux ----------------
 * A small network 10 -> 64 -> 64 -> 64 -> 5 (ReLU) stands in for the
 * iteration of the two-shock Riemann solver (Sec. 3.2 names the solver; the
 * network is this library's addition).  Its inputs are the left and right
 * face states (rho, u_n, u_t1, u_t2, p) normalised by the mean density, mean
 * sound speed and mean normal velocity of the face; its first output is
 * ln(p* / (rbar cbar^2)), the others are the normalised star velocity, star
 * densities and Godunov density.  In a step with p->riemann ==
 * NYX_RIEMANN_LEARNED (FP32-mixed precision only) the stages selected by
 * p->learned_stages_mask evaluate the network with BF16 MFMA and FP32
 * accumulation, correct its pressure by one FP64 Newton step of the
 * two-shock relations and accept the face when the two-shock velocity
 * residual divided by cbar is below p->mlp_resid_tol and the star state is
 * positive and finite; every other face is solved by the plain iteration.
 * Counters mlp_used / mlp_fallback record the split.
 *
 * Training records (float, 15 per face): left state, right state, p*, u*,
 * rho*_L, rho*_R, Godunov density, as the plain solver computed them. */
#define NYX_MLP_NPARAM 9349
#define NYX_MLP_PACKED_BYTES 23552

/* Harvest records of the final-stage faces of subsequent batched steps: a
 * face is kept when a hash of (seed, box, face) falls below keep_fraction;
 * records (device, capacity x 15 floats) are appended at *count (device,
 * caller-zeroed); faces beyond the capacity are counted but not written.
 * records == NULL disables harvesting. */
int nyx_batch_set_harvest(nyx_batch* plan, float* records, unsigned long long* count,
                          long long capacity, double keep_fraction, unsigned long long seed);

/* FP32 master parameters (device, NYX_MLP_NPARAM floats, layout W1[64][10],
 * b1, W2[64][64], b2, W3[64][64], b3, W4[5][64], b4): Glorot-uniform
 * weights from a counter-based generator of `seed`, zero biases. */
int nyx_mlp_init(float* params, unsigned long long seed, void* stream);

/* Mean-squared loss over the normalised targets and its gradient for n
 * records, both ADDED to loss (device, 1 float) and grad (device,
 * NYX_MLP_NPARAM floats), each scaled by inv_batch (1 / samples in the whole
 * batch, so several calls can form one batch).  FP32 arithmetic. */
int nyx_mlp_loss_grad(const float* params, const float* records, long long n, double gamma,
                      double inv_batch, float* grad, float* loss, void* stream);

/* One Adam update (step t >= 1) of params with moments m, v (device). */
int nyx_mlp_adam(float* params, float* m, float* v, const float* grad, int t, double lr,
                 double beta1, double beta2, double eps, void* stream);

/* Convert FP32 parameters into the packed BF16 inference weights (device,
 * NYX_MLP_PACKED_BYTES, 16-byte aligned) read by learned steps. */
int nyx_mlp_pack(const float* params, void* packed, void* stream);

/* Network outputs (device, n x 5 floats) for n records with the inference
 * path (BF16 MFMA). */
int nyx_mlp_predict(const void* packed, const float* records, long long n, double gamma,
                    float* out, void* stream);

/* ---------------- stage timing (profiling aid, off by default) ----------------
 * When enabled, every step records HIP events around each of its
 * NYX_NSTAGES stage launches on the step's own stream, in this order:
 * primitives, flattening, PPM + tracing, stage-0 Riemann, stage-1 transverse
 * Riemann, stage-2 final Riemann, update.  nyx_profile_read waits for the
 * recorded events and returns the milliseconds accumulated per stage (ms[7])
 * and the number of timed stage sequences since the last reset.  Do not enable
 * it while a stream is being captured into a HIP graph. */
#define NYX_NSTAGES 7
int nyx_profile_enable(int on);
int nyx_profile_read(double* ms, long long* sequences, int reset);

#ifdef __cplusplus
}
#endif
#endif
