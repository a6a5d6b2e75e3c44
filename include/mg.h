/*
 * mg.h -- C ABI of the MI355X complex additive multilevel Helmholtz library.
 *
 * The library solves the channel Helmholtz equation of the paper's Section 2,
 *     -Lap u - phi u = chi   on (0,1)^d, d in {2,3}, zero Dirichlet boundary,
 * discretised with d-linear finite elements on the regular levels of a
 * 3-partitioned spacetree (Sections 3 and 4), with the complex grid rotation
 * h -> h exp(i theta) (CSG) and complex phi (CSL shift) of Section 2.  One
 * cycle is the single-sweep pipelined additive FAS of Section 5 (Algorithms
 * tdAdd and tdBPX, with the hierarchical-basis mask of eq. hb-omega): damped
 * Jacobi on every level, factor-3 d-linear prolongation P, R = P^T, and
 * injection I.
 *
 * Conventions for every entry point
 *   - Vectors are caller-owned DEVICE buffers of complex128 (mg_c128, the
 *     layout of torch.complex128), contiguous C order of shape (n,)*d with
 *     n = 3^level_max + 1 and x fastest; boundary vertices are included.
 *     Input boundary entries are ignored; output boundary entries are zero.
 *     Buffers are borrowed for the duration of the call and never retained.
 *   - All device work is enqueued on the stream given to mg_setup.  Calls
 *     that return host scalars synchronise that stream.
 *   - int-returning calls return MG_OK or a negative MG_E* code;
 *     mg_last_error() returns a thread-local message for the last failure.
 *   - A context is used by one host thread at a time.
 */
#ifndef MG_H
#define MG_H

#ifdef __cplusplus
extern "C" {
#endif

#define MG_OK          0
#define MG_EINVAL     (-1)   /* bad argument or size                         */
#define MG_ENOMEM     (-2)   /* device allocation failed                     */
#define MG_EDEVICE    (-3)   /* a HIP runtime call or kernel launch failed   */
#define MG_ENOTCONV   (-4)   /* maxit reached; outputs hold the last iterate */
#define MG_EDIVERGED  (-5)   /* non-finite residual or ||r|| > 1e8 ||r0||    */

typedef struct { double re, im; } mg_c128;
typedef struct mg_ctx mg_ctx;   /* opaque; owns all level buffers */

/* Solver variants (Section 5.2): plain additive MG, hierarchical basis
 * (c-point omega masked, eq. hb-omega), BPX (Algorithm tdBPX). */
enum { MG_ADD = 0, MG_HB = 1, MG_BPX = 2 };

/* Relaxation schemes omega_l (table of Section 5.1), succ = l_max - l:
 * CONST omega; JACOBI omega on l_max only; LGRID omega where succ <= omega_L;
 * EXP omega^(succ+1); TRANSITION omega^((1-1/n)(succ+1)), n = cycle counter.
 * TWO_PHASE: the two-phase relaxation of Section 7.4 (used there with plain
 * Jacobi, level_min = level_max): omega on odd cycles n and -conj(omega) on
 * even ones, on every level.  The zero-start cycle of the Krylov driver uses
 * n = 1 for every scheme. */
enum { MG_OMEGA_CONST = 0, MG_OMEGA_JACOBI = 1, MG_OMEGA_LGRID = 2,
       MG_OMEGA_EXP = 3, MG_OMEGA_TRANSITION = 4, MG_OMEGA_TWO_PHASE = 5 };

/* Arithmetic of the cycle: complex128 throughout, or complex64 level
 * corrections inside an FP64 residual-refinement loop (mg_solve only; the
 * operator application mg_apply is always FP64). */
enum { MG_FP64 = 0, MG_FP32_REFINE = 1 };

/* Solve drivers: repeated cycles, or BiCGStab preconditioned by one cycle
 * from a zero start. */
enum { MG_STATIONARY = 0, MG_BICGSTAB = 1 };

/* How the coarse FAS right-hand side b_(l-1) is formed.
 * FAS:      b_(l-1) = R (b_l - H_l uhat_l), uhat = u - P u_(l-1)  (eq. HTMG);
 * GALERKIN: b_(l-1) = R r_l + H_(l-1) u_(l-1) (the paper's Lemma 2), valid
 *           when R H_l P = H_(l-1): constant phi and uniform rotation.  The
 *           coarse b slot then holds R r_l and the coarse residual is read
 *           from it directly, so the coarse iterates u_l (l < level_max) are
 *           read by no step and are not formed;
 * AUTO:     GALERKIN for constant phi, FAS otherwise. */
enum { MG_RESTRICT_AUTO = 0, MG_RESTRICT_FAS = 1, MG_RESTRICT_GALERKIN = 2 };

/* Finest-level sweep implementation: AUTO picks FUSED when supported (constant
 * phi, GALERKIN form), GENERIC runs the level operations as separate passes. */
enum { MG_SWEEP_AUTO = 0, MG_SWEEP_GENERIC = 1, MG_SWEEP_FUSED = 2 };

/* Level fields for mg_get_level. */
enum { MG_FIELD_U = 0, MG_FIELD_B = 1, MG_FIELD_SC = 2, MG_FIELD_SF = 3, MG_FIELD_SI = 4 };

typedef struct {
  int dim;                   /* 2 or 3                                             */
  int level_min, level_max;  /* 1 <= level_min <= level_max; 3^level cells/axis    */
  double theta;              /* CSG rotation: cell side h -> h exp(i theta)        */
  mg_c128 phi;               /* constant phi of  -Lap u - phi u = chi              */
  const mg_c128* phi_field;  /* optional DEVICE nodal phi on the finest level      */
                             /* (NULL: constant).  Read during mg_setup only;      */
                             /* coarse levels sample it at their vertices.         */
  int variant;               /* MG_ADD | MG_HB | MG_BPX                            */
  int omega_scheme;          /* MG_OMEGA_*                                         */
  mg_c128 omega;             /* omega_S                                            */
  int omega_L;               /* grid bound of MG_OMEGA_LGRID                       */
  int precision;             /* MG_FP64 | MG_FP32_REFINE                           */
  int conjugate;             /* 1: operator is H^H = conj(H) (adjoint solves)      */
  int restrict_form;         /* MG_RESTRICT_*                                      */
  int sweep;                 /* MG_SWEEP_*                                         */
  double inner_rtol;         /* MG_FP32_REFINE: relative residual each complex64   */
                             /* inner solve aims for (0: 0.3); an outer step       */
                             /* then reduces the FP64 residual by about this much  */
  /* Absorbing layer (Section 7.4): on every level, a cell whose centre lies   */
  /* closer than layer_width to one of the faces in layer_faces is rotated by  */
  /* layer_theta instead of theta (stiffness eta_c^(d-2), mass eta_c^d of that */
  /* cell; diagonal accumulated cell by cell).  Faces: bit 2a is x_a = 0, bit  */
  /* 2a+1 is x_a = 1, with x_0 = x the fastest-varying coordinate.  A layer    */
  /* (layer_width > 0) takes the nodal-coefficient path (FAS form, no fused    */
  /* sweep); it is not available with batches, nested solves or gradients.    */
  double layer_theta;
  double layer_width;        /* 0: no layer                                        */
  int layer_faces;
} mg_params;

/* Fills *p with: dim 3, levels 1..3, theta 0, phi 0, constant, BPX, CONST,
 * omega 0.6, omega_L 1, FP64, no conjugation, AUTO forms. */
void mg_params_default(mg_params* p);

/* Builds a context: allocates every level's fields (u, b, sc, sf, si; the
 * finest level keeps the folded iterate u + sc in two ping-pong buffers),
 * derives per-level operator data (Section 4: rediscretisation on each level;
 * for a phi field, nodal phi by injection, cell averages and the accumulated
 * diagonal), zeroes the state.  hip_stream: a hipStream_t or NULL (default
 * stream).  Returns MG_EINVAL for bad params, MG_ENOMEM/MG_EDEVICE on device
 * failures; *out is NULL on failure. */
int mg_setup(const mg_params* p, void* hip_stream, mg_ctx** out);

/* Frees everything the context owns.  NULL is accepted. */
void mg_destroy(mg_ctx* ctx);

/* Thread-local text of the last error ("" if none). */
const char* mg_last_error(void);

/* Number of vertices per axis on `level` (3^level + 1), or MG_EINVAL. */
int mg_level_size(const mg_ctx* ctx, int level);

/* y = H_(level_max) x on interior vertices, y = 0 on the boundary (Section 4 /
 * Appendix B: element-wise matrix-free operator, FP64). x and y must not
 * alias. */
int mg_apply(mg_ctx* ctx, const mg_c128* x, mg_c128* y);

/* Lumped discrete load: b = eta_L^d chi at interior vertices, 0 on the
 * boundary, eta_L = 3^-L exp(i theta) (the weight of the discretised
 * right-hand side, Section 4).  With an absorbing layer the weight of a vertex
 * is the mean of eta_c^d over its 2^d cells.  chi and b may alias. */
int mg_rhs_from_nodal(mg_ctx* ctx, const mg_c128* chi, mg_c128* b);

/* Sets the finest right-hand side and resets the pipeline helpers
 * (sc = sf = si = 0, the start of the single-sweep iteration of Section 5.1)
 * and the cycle counter of the iteration-dependent relaxation schemes; a
 * pending update is discarded (call mg_flush first to keep it).  b: device,
 * finest size; boundary entries ignored. */
int mg_set_rhs(mg_ctx* ctx, const mg_c128* b);

/* Sets the finest iterate, injects it into every coarser level (the FAS
 * constraint u_(l-1) = I u_l of Section 4) and resets the helpers and the
 * cycle counter. */
int mg_set_solution(mg_ctx* ctx, const mg_c128* u);

/* Runs ncycles pipelined cycles (one traversal each).  Cycle k reports the
 * residual of the iterate it started from (the half-iteration shift of
 * Section 5): res_h[k] = |b - H u|_h, |x|_h^2 = sum |h|^d |x_i|^2 over interior
 * vertices (Section 7), res_max[k] the max norm.  res_h / res_max may be
 * NULL; when given they are host arrays of ncycles doubles and the call
 * synchronises. */
int mg_cycle(mg_ctx* ctx, int ncycles, double* res_h, double* res_max);

/* Applies the pending update (the descent of Algorithms tdAdd / tdBPX alone,
 * which completes the half-shifted iteration of Section 5.1), clears the
 * helpers and, if u_out != NULL, copies the finest iterate into it (device,
 * finest size).  The cycle counter is kept: the transition and two-phase
 * schemes continue with the next cycle number after a flush. */
int mg_flush(mg_ctx* ctx, mg_c128* u_out);

/* Copies one level field into a device buffer of (3^level+1)^d complex128.
 * Finest level: MG_FIELD_U returns the folded iterate u + sc (the finest
 * smoothing update is applied eagerly, only the coarse correction is
 * pending); MG_FIELD_SC/SF/SI return zeros.  Coarse levels with the GALERKIN
 * form: MG_FIELD_B returns the restricted residual R r_(l+1) (= b_l - H_l u_l)
 * and MG_FIELD_U returns zeros (the coarse iterates are not formed). */
int mg_get_level(mg_ctx* ctx, int level, int field, mg_c128* out);

/* z = B v: one additive cycle from a zero start with right-hand side v
 * (restriction chain, damped Jacobi scaling per level, prolongation chain of
 * the variant's corrections; no operator application survives u = 0). */
int mg_precondition(mg_ctx* ctx, const mg_c128* v, mg_c128* z);

/* z = B v and y = H z in one call: the step of the Krylov driver.  In 3D with
 * constant phi the finest level of B and the operator run as one pass over
 * the finest grid (read v, write z and y).  v, z, y: device buffers of the
 * finest size, not aliased; boundary entries of v are ignored, z and y get
 * zero boundaries.  Complex128 contexts only (MG_EINVAL otherwise). */
int mg_precondition_apply(mg_ctx* ctx, const mg_c128* v, mg_c128* z, mg_c128* y);

/* Solves H u = b to relative residual rtol (|b - H u| / |b|, Euclidean over
 * interior vertices).  u holds the initial guess on entry and the result on
 * exit; b, u: device, finest size.  driver:
 *   MG_STATIONARY  the paper's iteration (Section 5.1): pipelined cycles until
 *                  the residual a cycle reports (that of the iterate before
 *                  it) meets rtol, then a flush; *iters_out = cycles run, u =
 *                  the iterate after them.  MG_ENOTCONV also when the returned
 *                  iterate itself misses rtol;
 *   MG_BICGSTAB    BiCGStab preconditioned by one cycle from a zero start (the
 *                  cycle used as a preconditioner, Sections 2 and 4; the Krylov
 *                  method is an addition to the paper).
 * With MG_FP32_REFINE the inner corrections run in complex64 inside an FP64
 * residual-refinement loop.  iters_out / relres_out may be NULL; *relres_out
 * is the returned iterate's relative residual.  Returns MG_ENOTCONV or
 * MG_EDIVERGED (non-finite residual or one above 1e8 times the first; u
 * valid) when the target is missed.  Resets the cycle state. */
int mg_solve(mg_ctx* ctx, const mg_c128* b, mg_c128* u, double rtol, int maxit,
             int driver, int* iters_out, double* relres_out);

/* res_h = |b - H u|_h (FP64). */
int mg_residual_norm(mg_ctx* ctx, const mg_c128* u, const mg_c128* b, double* res_h);

/* For callers that cannot allocate device memory in the call (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same norms as mg_residual_norm, res_h = |b - H u|_h and res_max = max |r_j|
 * over interior vertices (FP64; either output may be NULL, not both), without
 * any allocation.  The residual is not stored; the per-block partials and
 * the two results live in a fixed library array of 2 * 1024 + 2 doubles per
 * device (resolved at mg_setup, held until the process ends), so every level
 * with at most 1024 * 64 vertices per axis is accepted (MG_EINVAL beyond).
 * All calls on one device share that array: calls that overlap on a device
 * (other host threads or streams) race.  Synchronises the context stream. */
int mg_residual_norm_noalloc(mg_ctx* ctx, const mg_c128* u, const mg_c128* b, double* res_h,
                             double* res_max);

/* uf = P uc: d-linear prolongation (factor 3) from level - 1 to level, the
 * paper's P of Section 4.  uc: device buffer of (3^(level-1)+1)^dim entries,
 * uf: (3^level+1)^dim entries (C order, x fastest), not aliased; uf is zero
 * on the boundary.  2 <= level <= level_max (MG_EINVAL otherwise).  Enqueued
 * on the context stream. */
int mg_prolong(mg_ctx* ctx, int level, const mg_c128* uc, mg_c128* uf);

/* Nested (FMG-like) solve, the regular-grid form of the paper's remark on
 * FMG-like cycles (Section 5): coarse solution approximations serve as
 * initial guesses on finer grids.  chi: the nodal load on the finest grid
 * (device, (3^level_max+1)^dim entries; b = eta_L^dim chi at interior
 * vertices, as mg_rhs_from_nodal).  For l = level_start .. level_max - 1 the
 * load is sampled at the vertices of level l, H_l u_l = b_l is solved to
 * relative residual coarse_rtol (driver, maxit as mg_solve; MG_ENOTCONV on a
 * coarse level is accepted) starting from P u_(l-1) (zero on level_start),
 * each on a context with the parameters of ctx and level_max = l.
 * Then u = P u_(level_max - 1) is the initial guess of mg_solve on ctx with
 * rtol (u's entry value is ignored; level_start == level_max starts from
 * zero).  iters_out / relres_out: those of the finest solve (may be NULL).
 * Constant phi only (MG_EINVAL otherwise).  chi and u must not alias.  The
 * coarser levels' contexts and buffers are made on the first call and kept
 * with ctx (mg_destroy frees them).  Synchronises. */
int mg_solve_nested(mg_ctx* ctx, const mg_c128* chi, mg_c128* u, int level_start, double coarse_rtol,
                    double rtol, int maxit, int driver, int* iters_out, double* relres_out);

/* Gradient of J = sum_S |u|^2 with respect to a nodal potential V entering
 * phi = phi0 - V (cell-averaged mass weight):
 *   dJdV_j = -2 Re sum_{cells c containing j} 2^-d eta^d lam_c^H M u_c,
 * u the forward solution, lam = H^-H (1_S u) the adjoint solution (both
 * device complex128, zero boundary), dJdV a device array of n^d doubles
 * (every vertex, boundary included). */
int mg_grad_potential(mg_ctx* ctx, const mg_c128* u, const mg_c128* lam, double* dJdV);

/* Tile variants of the fused finest-level sweep (block shape and z extent).
 * mg_tiles reports the current tile and the number of variants; mg_set_tile
 * selects one (MG_EINVAL when out of range or when the context has no fused
 * sweep). */
int mg_tiles(const mg_ctx* ctx, int* current, int* count);
int mg_set_tile(mg_ctx* ctx, int tile);

/* Autotuner of the fused sweep: launches every tile variant `reps` times on the
 * context's current data, writing into scratch buffers (the cycle state is not
 * modified), times each launch (with its seam pass) with HIP events after
 * filling two finest-size scratch arrays, so that the caches hold other data
 * as they do inside a cycle, and selects the fastest.
 * best_tile / best_us (average microseconds per launch) may be NULL;
 * times_us, when not NULL, receives one average per variant (mg_tiles count).
 * Synchronises. */
int mg_autotune(mg_ctx* ctx, int reps, int* best_tile, double* best_us, double* times_us);

/* Measurement hook for the finest-level sweep (the kernel that moves most of
 * a cycle's bytes).  enable != 0: every following finest sweep launched by
 * mg_cycle is timed by a HIP event pair on the context stream -- for the
 * fused sweep the pair goes with the launch (hipExtLaunchKernel) and takes the
 * kernel's own start and end; the unfused sweep's kernels are bracketed by
 * two recorded events.  enable == 0 stops recording.  Enabling clears earlier
 * records. */
int mg_time_sweeps(mg_ctx* ctx, int enable);

/* Synchronises and returns the summed event time (milliseconds) and the number
 * of finest sweeps recorded since mg_time_sweeps(ctx, 1). */
int mg_sweep_time(mg_ctx* ctx, double* total_ms, int* count);

/* ---------------------------------------------------------------------------
 * Batched cycles (many independent problems; one persistent launch per cycle
 * for the problems below 2^22 finest vertices).
 *
 * The multilevel cycle of the method (Section 5, the pipelined additive
 * schemes tdAdd and tdBPX) applied to a set of independent problems --
 * several right-hand sides, wavenumbers, dimensions and depths -- at once.
 * Each problem lives in its own context (created by mg_batch_setup, reachable
 * through mg_batch_problem for mg_set_rhs / mg_set_solution / mg_get_level /
 * mg_flush); a batched cycle advances every problem by exactly one pipelined
 * cycle and leaves each context in the state mg_cycle(ctx, 1, ...) would, with
 * the fused sweep in the batch's tiling.  Requirements per problem: constant
 * phi, level_max > level_min, level_max <= 7, an iteration-independent omega
 * scheme (not MG_OMEGA_TRANSITION or MG_OMEGA_TWO_PHASE); all problems share
 * one precision.
 * Problems below 2^22 finest vertices are advanced concurrently in one
 * persistent launch per cycle, which overlaps their coarse levels with the
 * finest sweeps of others; a problem of 2^22 finest vertices or more fills the
 * device by itself and runs mg_cycle's own launches (its fused tile chosen by
 * its own autotuner, 3D default: 4 coarse rows, 28 planes, y-band order). */
typedef struct mg_batch mg_batch;

/* Creates `count` contexts from params[0..count-1] (sweep forced to FUSED) on
 * hip_stream (NULL = default stream).  *out = NULL on failure. */
int mg_batch_setup(const mg_params* params, int count, void* hip_stream, mg_batch** out);
void mg_batch_destroy(mg_batch* batch);

/* The context of problem i (owned by the batch; do not mg_destroy it).  Its
 * fused tile (mg_tiles) is kept equal to the batch's tiling of that problem
 * (for a large problem: the tile it runs with), so mg_cycle on it reproduces
 * a batched cycle exactly. */
int mg_batch_problem(mg_batch* batch, int i, mg_ctx** ctx);

/* ncycles batched cycles.  res_h, when not NULL, receives ncycles * count
 * doubles: res_h[k * count + i] = |r|_h of problem i before its finest update
 * in cycle k (as mg_cycle's res_h).  Synchronises.  MG_EDEVICE if an internal
 * dependency wait exceeded its bound (the launch still completes; the state
 * is then undefined). */
int mg_batch_cycle(mg_batch* batch, int ncycles, double* res_h);

/* Autotunes the fused tile of each problem of 2^22 finest vertices or more
 * (mg_autotune, state untouched), then times every batch configuration (fused
 * z extent per dimension, queue order) with `reps` batched cycles each and
 * keeps the fastest.  The cycles run on
 * the contexts' current data and advance them: reset the state afterwards.
 * config / us_per_cycle may be NULL; times_us, when not NULL, receives the
 * average microseconds per batched cycle of each of the mg_batch_configs()
 * configurations. */
int mg_batch_autotune(mg_batch* batch, int reps, int* config, double* us_per_cycle, double* times_us);

/* Number of batch configurations the autotuner tries. */
int mg_batch_configs(void);

/* Selects batch configuration `config` (0 <= config < mg_batch_configs()),
 * as the autotuner would: the 3D and 2D sweep tiles and the queue order of
 * the cycle, and the tiles of the batched preconditioner.  The problems'
 * state is kept.  MG_EINVAL out of range. */
int mg_batch_set_config(mg_batch* batch, int config);

/* Bound of every dependency wait inside the batched kernel, in polls (default
 * 2^20, about a second; 0 <= polls <= 2^26, MG_EINVAL otherwise).  A wait
 * that reaches it gives up: the item is skipped, the launch still drains, and
 * the mg_batch_cycle call returns MG_EDEVICE with the state undefined.  For
 * tests of that error path (a bound of 0 makes every wait that finds its
 * dependency unfinished give up at once). */
int mg_batch_set_spin_limit(mg_batch* batch, long long polls);

/* Scheduler trace.  mg_batch_trace(b, 1) makes every following batched cycle
 * record, per work item, the device wall clock (100 MHz) when its workgroup
 * starts waiting for the item's dependencies, when they are met and when the
 * item is published, and the XCD and workgroup that ran it.
 * mg_batch_get_trace copies the last cycle's record: 8 values per item in
 * queue order -- problem, phase, tile, kind (0 descent, 1/2 finest sweep 3D/2D,
 * 3 Galerkin backtracking, 4 coarsest update, 5 norm, 6 seam rows of the 3D
 * sweep's restriction), wait start, ready,
 * done, XCD << 16 | workgroup -- for min(cap, count) items; *count receives
 * the number of items.  Synchronises. */
int mg_batch_trace(mg_batch* batch, int enable);
int mg_batch_get_trace(mg_batch* batch, long long* out, int cap, int* count);

/* z_i = B_i v_i and y_i = H_i z_i for every problem of the batch, the
 * problems with fewer than 2^22 finest vertices in one persistent launch and
 * each larger one with its own launches (mg_precondition_apply's; such a level
 * fills the device by itself), B_i the problem's additive cycle from a zero start (the
 * preconditioner of the Krylov driver: restrictions down to level_min, then
 * omega_l D_l^-1 on every level with the variant's level operator and P going
 * up; Section 5's cycle applied to u = 0).  vs, zs, ys: arrays of count
 * device pointers to complex128 vectors of each problem's finest size (v
 * boundary entries ignored; z, y zero on the boundary; none may alias).
 * Complex64 batches compute in complex64 and convert.  Synchronises. */
int mg_batch_precondition_apply(mg_batch* batch, const mg_c128* const* vs, mg_c128* const* zs,
                                mg_c128* const* ys);

/* Solves H_i u_i = b_i for every problem of the batch (bs[i], us[i]: device
 * complex128 vectors of each problem's finest size; us[i] holds the initial
 * guess and receives the solution) to |b - H u| <= rtol |b| per problem.
 * MG_BICGSTAB: BiCGStab for all problems in lockstep, each iteration's two
 * preconditioner applications with the operator and the dot products as in
 * mg_batch_precondition_apply (one persistent launch for the problems below
 * 2^22 finest vertices, own launches for the larger ones) and every vector update
 * of all problems in one launch, inside FP64 residual refinement: r = b - H u
 * and |r| in FP64, the batched solve of H e = r / |r| in the batch's
 * precision (complex64 to each problem's inner_rtol, 0.3 if 0; an FP64
 * batch to rtol directly), u += |r| e in FP64.  maxit bounds each problem's
 * inner iterations.  MG_STATIONARY solves problem by problem with mg_solve.
 * iters / relres: arrays of count entries or NULL (inner iterations; the
 * final FP64 relative residual).  Returns MG_OK, MG_ENOTCONV or MG_EDIVERGED
 * (the worst over the problems; outputs valid).  Synchronises. */
int mg_batch_solve(mg_batch* batch, const mg_c128* const* bs, mg_c128* const* us, double rtol,
                   int maxit, int driver, int* iters, double* relres);

/* ---------------------------------------------------------------------------
 * Same-grid multichannel form (Section 7.5): nchan channels -- independent
 * problems  -Lap u_c - phi_c u_c = chi_c  that share the grid, the rotation,
 * the variant and the relaxation -- fused into one problem on one grid.  Every
 * vector is array-of-structures: nchan complex128 values per vertex, channel
 * c of vertex i (C order, x fastest, boundary included) at i * nchan + c.  One
 * cycle advances every channel by the pipelined additive cycle (Galerkin form
 * of the coarse right-hand side, Lemma 2); index, stencil and transfer work is
 * shared by the channels of a vertex.
 */
typedef struct mg_mc mg_mc;

/* p: dim, levels (level_min < level_max), theta, variant, omega scheme and
 * omega, conjugate; p->phi is ignored, phi_field must be NULL, no absorbing
 * layer, FP64.  nchan in {1, 2, 4, 8, 16}; phis: host array of the nchan
 * constant phi_c.  Allocates 16 nchan bytes per vertex per field.  MG_EINVAL
 * for anything else. */
int mg_mc_setup(const mg_params* p, int nchan, const mg_c128* phis, void* hip_stream, mg_mc** out);
void mg_mc_destroy(mg_mc* ctx);
/* y_c = H_c x_c for every channel (interior; y = 0 on the boundary). */
int mg_mc_apply(mg_mc* ctx, const mg_c128* x, mg_c128* y);
/* Finest right-hand sides of all channels; helpers and cycle counter reset. */
int mg_mc_set_rhs(mg_mc* ctx, const mg_c128* b);
/* Finest iterates of all channels; helpers and cycle counter reset. */
int mg_mc_set_solution(mg_mc* ctx, const mg_c128* u);
/* ncycles cycles; res_h (host, ncycles * nchan, or NULL) receives
 * |b_c - H_c u_c|_h of the iterate each cycle started from, cycle-major. */
int mg_mc_cycle(mg_mc* ctx, int ncycles, double* res_h);
/* Applies the pending update and copies every channel's finest iterate to u
 * (device, AoS; may be NULL). */
int mg_mc_flush(mg_mc* ctx, mg_c128* u);

/* ---------------------------------------------------------------------------
 * Feature-based dynamic adaptivity (Section 5.3) with hanging vertices
 * (Section 4), on a dense envelope of levels level_min..level_max: every level
 * is held as its full regular grid (3^l + 1 vertices per axis, C order, x
 * fastest), with one byte per cell ("refined into the 3^d cells of level
 * l+1", levels below level_max) and one class byte per vertex.  A cell is
 * present on level_min, and below it where its parent cell is refined.
 *
 * Vertex classes: MG_AMR_ABSENT (no adjacent cell present), PERSISTENT
 * (interior, all 2^d adjacent cells present: an unknown of the level),
 * HANGING (interior, some adjacent cells present: its value comes from the
 * coarser level through P), BOUNDARY (on the domain boundary, present).
 * Marks: MG_AMR_KEEP, REFINE (refine the vertex's 2^d cells), ERASE (return
 * them to leaves).  The device arrays are owned by the object; all calls run
 * on its stream; calls with host outputs synchronise it.
 */
typedef struct mg_amr mg_amr;
enum { MG_AMR_ABSENT = 0, MG_AMR_PERSISTENT = 1, MG_AMR_HANGING = 2, MG_AMR_BOUNDARY = 3 };
enum { MG_AMR_KEEP = 0, MG_AMR_REFINE = 1, MG_AMR_ERASE = 2 };

/* dim 2 or 3, 1 <= level_min <= level_keep <= level_max (3D: <= 6, 2D: <= 9).
 * level_keep is the coarsest admissible mesh (h_max = 3^-level_keep): cells of
 * coarser levels stay refined; level_max the finest (h_min).  Starts as the
 * regular grid of level_keep.  Allocates 3 bytes per vertex and 1 per cell of
 * every level.  MG_EINVAL / MG_ENOMEM / MG_EDEVICE; *out NULL on failure. */
int mg_amr_setup(int dim, int level_min, int level_keep, int level_max, void* hip_stream, mg_amr** out);
void mg_amr_destroy(mg_amr* amr);

/* Marks one level (Section 5.3).  u: DEVICE level field (complex128, n^d);
 * r: DEVICE residual of the level or NULL (no veto); diag: the level's
 * constant diagonal, or diag_field: DEVICE per-vertex diagonal (n^d; varying
 * phi or a layer), which replaces diag when not NULL.  Candidates are the
 * persistent vertices; their
 * criterion s = max over axes a of |u(j+e_a) - 2u(j) + u(j-e_a)| is binned
 * into nbins (1..64; the paper: 20) equal subranges of [min s, max s]; the k
 * top bins whose count is closest to refine_pct % of the candidates are
 * marked REFINE (none on level_max), the e bottom bins closest to erase_pct %
 * (e <= nbins - k) ERASE (none below level_keep); ties take fewer bins.  A
 * vertex with |r|^2 > veto^2 |diag|^2 (the paper: veto 1e-2; |diag_i| with a
 * diagonal field) keeps.  The
 * marks are kept for mg_amr_adapt (and readable with mg_amr_get).
 * counts (HOST, nbins + 5, or NULL): the bin counts, k, e, candidates, REFINE
 * marks, ERASE marks; s_range (HOST, 2, or NULL): min s, max s. */
int mg_amr_mark(mg_amr* amr, int level, const mg_c128* u, const mg_c128* r, mg_c128 diag,
                const mg_c128* diag_field, int nbins, int refine_pct, int erase_pct, double veto,
                long long* counts, double* s_range);

/* One adaptation step from the marks of the levels marked since the last
 * step: refined-cell flags from level_max - 1 up to level_min (REFINE refines
 * the vertex's cells; ERASE returns a cell to a leaf unless a REFINE mark also
 * touches it or one of its children is refined after the step), then the
 * vertex classes of every level (the previous ones are kept for
 * mg_amr_interpolate).  class_counts (HOST, 4 per level from level_min, or
 * NULL): absent, persistent, hanging, boundary vertices. */
int mg_amr_adapt(mg_amr* amr, long long* class_counts);

/* Values of level `level` (level_min < level <= level_max) after a step
 * (Sections 4 and 5.3): vertices now hanging, and vertices now persistent that
 * were not, take (P u_coarse); vertices that became absent or boundary are set
 * to 0; every other vertex keeps its value (a caller that starts a level from
 * zeros keeps zeros on its absent and boundary vertices).  u_coarse: DEVICE
 * level - 1 field; u: DEVICE, in/out. */
int mg_amr_interpolate(mg_amr* amr, int level, const mg_c128* u_coarse, mg_c128* u);

/* Copies state to DEVICE memory: what 0 = vertex classes, 1 = classes before
 * the last step (n^d bytes each), 2 = refined-cell flags ((n-1)^d bytes, not
 * on level_max), 3 = the level's last marks at its candidates, MG_AMR_KEEP
 * elsewhere (n^d bytes). */
int mg_amr_get(mg_amr* amr, int level, int what, unsigned char* out);

/* Replaces the refined-cell flags of one level (level_min <= level <
 * level_max) from DEVICE bytes and recomputes every level's classes (previous
 * classes = new ones).  A refined cell whose parent is not refined is the
 * caller's error and is not checked. */
int mg_amr_set_cells(mg_amr* amr, int level, const unsigned char* cells);

#ifdef __cplusplus
}
#endif
#endif /* MG_H */
