/*
 * fe_abi.h - C ABI of the MI355X (gfx950) finite-element library for the
 * exact-gradient step of minimum-compliance topology optimisation
 * (Zhang et al., "Speeding up Computational Morphogenesis with Online Neural
 * Synthetic Gradients": problem (4), gradient (5), Sec. III-D).
 *
 * The step: given a physical density rho = P z on a structured nx*ny*nz
 * grid of cubic 8-node bricks, solve K(rho) u = f (linear elasticity, SIMP
 * modulus E(rho) = Emin + rho^p (E0 - Emin)), then return the compliance
 * f^T u, its gradient dc/drho (Eq. 5), the filter P and its transpose (the
 * volume gradient P^T v of Sec. III-D) and the optimality-criteria update.
 *
 * Layouts (all "canonical"):
 *   element e = i + nx*(j + ny*k),  node n = i + (nx+1)*(j + (ny+1)*k),
 *   dof 3*n + c with c = x, y, z.
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller, in
 * float64, unless stated otherwise.  Every device array the library works on
 * (vectors, moduli, multigrid levels, reduction partials, scalars) lives in
 * the caller's workspace; the library makes no device-array allocation.
 * What it does create, per handle, outside the workspace:
 *   - fe_setup: the host handle (operator new), two small pinned host
 *     buffers (hipHostMalloc: the CG state mirror and four scalars), one
 *     event (hipEventCreateWithFlags) and one non-blocking capture stream
 *     (hipStreamCreateWithFlags); fe_setup also synchronises the stream
 *     once (its host-to-device copies read host stack arrays);
 *   - the first solve of each vector type (and the first after a change of
 *     multigrid parameters, precision path or profiling): one captured and
 *     instantiated HIP graph of a chunk of CG iterations (hipGraphInstantiate
 *     allocates the graph's own runtime memory); oc_update on the same
 *     arrays a second time: one captured graph of the update;
 *   - fe_batch_create: the host batch object, one event, a pinned array of
 *     the slots' CG states and one handle per slot, each created as by
 *     fe_setup (pinned buffers, event, capture stream), and the batch's own
 *     captured graph on its first round;
 *   - with profiling on: event pairs (hipEventCreate), reused;
 *   - the synthetic-gradient model (fe_onsg_create): a rocBLAS handle.
 * fe_destroy / fe_batch_destroy / fe_onsg_destroy release all of it.
 * Blocking calls: fe_setup, fe_solve, fe_set_load, fe_kernel_stats (when
 * events are pending), fe_batch_setup_slot and fe_batch_round_end wait for
 * the handle's stream; everything else is asynchronous.
 *
 * Streams: every call is ordered on the stream given to fe_setup.  Calls that
 * return host scalars (fe_solve) synchronise that stream before returning;
 * the others are asynchronous and may write device scalars.  One handle must
 * not be used from two host threads at once.
 *
 * Errors: nothing throws across the ABI.  Every entry point returns an
 * fe_status; on failure fe_last_error() gives a message (thread-local).
 */
#ifndef FE_ABI_H
#define FE_ABI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifndef FE_API
#define FE_API __attribute__((visibility("default")))
#endif

typedef enum {
  FE_OK = 0,
  FE_EINVAL = -1,      /* bad argument: dims < 1, 3 (nx+1)(ny+1)(nz+1) >= 2^31 (dof indices
                          are 31-bit), nu not in (-1, 0.5), Emin not in (0, E0), penal < 1,
                          filter_r not in (0, 8], NULL required pointer, ... */
  FE_ENOMEM = -2,      /* workspace smaller than fe_workspace_size(cfg) */
  FE_EDEVICE = -3,     /* a HIP runtime call failed */
  FE_ENOTCONV = -4,    /* iteration limit reached; u holds the last iterate */
  FE_EBREAKDOWN = -5   /* p^T K p <= 0 or a non-finite value inside CG */
} fe_status;

enum { FE_PREC_FP64 = 0,     /* vectors, K*u and dots in float64 */
       FE_PREC_FP32_IR = 1,  /* float32 CG inside float64 iterative refinement */
       FE_PREC_BF16_IR = 2,  /* as FP32_IR with the element contraction Ke*u_e of
                                the finest-grid K*u on bf16 matrix cores (rigid
                                motion of each brick removed before rounding),
                                float32 accumulation */
       FE_PREC_BF16X3_IR = 3 /* as BF16_IR with Ke and u_e each split into a
                                hi + lo pair of bf16 numbers (three products) */ };

enum { FE_PRECOND_JACOBI = 0, FE_PRECOND_GMG = 1 };

typedef struct fe_config {
  int32_t nx, ny, nz;   /* elements per axis, each >= 1 */
  double h;             /* element edge length (> 0) */
  double E0, Emin;      /* SIMP moduli, 0 < Emin < E0 */
  double nu;            /* Poisson ratio, -1 < nu < 0.5 */
  double penal;         /* SIMP exponent p >= 1 */
  double filter_r;      /* density-filter radius in element units, 0 < filter_r <= 8 */
  int32_t precision;    /* FE_PREC_* */
  int32_t precond;      /* FE_PRECOND_* */
  int32_t mg_levels;    /* levels of the geometric multigrid, 2..6 when precond = GMG;
                           level l + 1 has ceil(n / 2) elements of twice the edge per
                           axis of level l (any dimensions: an odd axis ends in a
                           coarse element overhanging the mesh, its missing children
                           counted as void) */
  int32_t reserved;     /* must be 0 */
} fe_config;

typedef struct fe_solve_info {
  int32_t iters;        /* total inner CG iterations */
  int32_t outer_iters;  /* float64 refinement steps (0 for FE_PREC_FP64) */
  double rel_res;       /* ||f - K u||_2 / ||f||_2 over the free dofs, in float64 */
  double compliance;    /* f^T u (Eq. 4 objective) */
} fe_solve_info;

typedef struct fe_problem fe_problem;

/* Bytes of device workspace fe_setup needs for cfg (pure host arithmetic;
 * 0 when cfg is invalid). */
FE_API size_t fe_workspace_size(const fe_config* cfg);

/* Build a problem in the caller's workspace.
 *   fixed : device uint8[ndof], 1 = dof held at zero; NULL = clamp every dof
 *           of the face x = 0 (the cantilever support of Sec. IV).
 *   f     : device float64[ndof] load vector (copied; entries on fixed dofs
 *           are ignored).
 *   ws    : device memory of ws_bytes >= fe_workspace_size(cfg), 256-byte
 *           aligned, untouched by the caller until fe_destroy.
 *   stream: hipStream_t to order all work on (NULL = default stream).
 * Precomputes Ke by 2x2x2 Gauss quadrature, the filter row sums and the
 * multigrid geometry. */
FE_API fe_status fe_setup(const fe_config* cfg, const uint8_t* fixed, const double* f,
                   void* ws, size_t ws_bytes, void* stream, fe_problem** out);

/* y = K(rho) u restricted to the free dofs (fixed rows and columns removed,
 * y = 0 on fixed dofs).  variant: 0 = float64, 1 = float32 vector,
 * 2 = bf16 matrix cores (float32 accumulation), 3 = float64 dense-Ke
 * reference kernel, 4 = split-bf16 matrix cores; variants 1, 2 and 4 need a
 * problem set up with a reduced precision and convert u and y at the
 * boundary.  rho: float64[nelem]. */
FE_API fe_status fe_apply_K(fe_problem* p, const double* rho, const double* u, double* y,
                     int32_t variant);

/* Solve K(rho) u = f for the free dofs (Sec. III-D; CG preconditioned by
 * Jacobi or geometric multigrid, Sec. III-D "PCG and multi-grid methods").
 *   rho : float64[nelem], physical (filtered) density in [0, 1].
 *   u   : float64[ndof]; in: initial guess, out: solution (0 on fixed dofs).
 *   rtol: stop when ||f - K u||_2 <= rtol ||f||_2 (float64 residual).
 *   max_iters: cap on inner CG iterations over the whole solve.
 *   info: host pointer, may be NULL.
 * Synchronises the stream.  FE_ENOTCONV / FE_EBREAKDOWN leave the last
 * iterate in u and fill info. */
FE_API fe_status fe_solve(fe_problem* p, const double* rho, double* u, double rtol,
                   int32_t max_iters, fe_solve_info* info);

/* The same solve without blocking, for callers that keep several problems in
 * flight on different streams (continuous batching):
 *   fe_solve_begin enqueues the start of the solve and returns;
 *   fe_solve_step advances it by at most one stage if the previous stage
 *     has completed on the device (never waits), *done = 1 once finished;
 *   fe_solve_end returns the status and info of a finished solve.
 * The arithmetic is exactly that of fe_solve (which is begin, step until
 * done, end), so a design's result does not depend on what else runs.
 * u and rho must stay valid until the solve is finished; one solve per
 * problem at a time (FE_EINVAL otherwise). */
FE_API fe_status fe_solve_begin(fe_problem* p, const double* rho, double* u, double rtol,
                                int32_t max_iters);
FE_API fe_status fe_solve_step(fe_problem* p, int32_t* done);
FE_API fe_status fe_solve_end(fe_problem* p, fe_solve_info* info);

/* Gradient of the compliance with respect to the physical density (Eq. 5):
 *   dc[e] = -penal rho_e^(penal-1) (E0 - Emin) u_e^T Ke u_e.
 * compliance: device float64 scalar receiving f^T u, may be NULL.
 * Asynchronous. */
FE_API fe_status fe_sensitivity(fe_problem* p, const double* rho, const double* u,
                         double* dc, double* compliance);

/* The state-equation term of the adjoint gradient (Sec. III-A, Eq. 3) for
 * r(rho, u) = K(rho) u - f:
 *   g[e] = -lam^T dr/drho_e = -penal rho_e^(penal-1) (E0 - Emin) lam_e^T Ke u_e,
 * where u solves K u = f and lam solves K lam = dJ/du (K is symmetric: a
 * second fe_solve after fe_set_load(p, dJ/du) gives lam).  The gradient of
 * an objective J(rho, u) is its explicit dJ/drho (the caller's) plus g; for
 * the compliance lam = u and g is fe_sensitivity's dc.  rho: float64[nelem],
 * u and lam: float64[ndof], g: float64[nelem]; device arrays owned by the
 * caller.  Asynchronous. */
FE_API fe_status fe_sensitivity_adjoint(fe_problem* p, const double* rho, const double* u, const double* lam,
                                 double* g);

/* Replaces the problem's load by f (float64[ndof], device, caller-owned;
 * entries at fixed dofs are ignored), e.g. by dJ/du for the adjoint solve of
 * Eq. (3); the supports are unchanged.  Blocks until the new load's norm is
 * known on the host.  FE_EINVAL while a solve is in progress or on a batch
 * slot (fe_batch_setup_slot sets those). */
FE_API fe_status fe_set_load(fe_problem* p, const double* f);

/* Density filter of problem (4): out = P in (transpose = 0) or
 * out = P^T in (transpose = 1), with P_ij = w_ij / sum_j w_ij and
 * w_ij = max(0, r - |c_i - c_j|) over element centroids in element units.
 * in and out are float64[nelem] and must not alias.  Asynchronous. */
FE_API fe_status fe_filter(fe_problem* p, const double* in, double* out, int32_t transpose);

/* Optimality-criteria update of the design (Sec. III-D):
 *   x_new = clamp(x * sqrt(max(0, -dcx) / (lambda * dv)),
 *                 max(0, x - move), min(1, x + move)),
 * lambda chosen so that sum(dv * x_new) = volfrac * nelem, to a relative
 * bracket of 1e-12 on lambda.  dv = P^T v with unit element volumes.
 * change: device float64 scalar receiving max |x_new - x|, may be NULL.
 * x and x_new may alias.  Asynchronous. */
FE_API fe_status oc_update(fe_problem* p, const double* x, const double* dcx, const double* dv,
                    double volfrac, double move, double* x_new, double* change);

/* oc_update without a problem handle and without any allocation, for
 * callers that cannot allocate device or host memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and launch sequence as oc_update (so the same x_new and change
 * bit for bit), launched directly on `stream` (hipStream_t, NULL = default
 * stream) with their partial sums and search state in a static device array
 * of the library (65,536 float64 partial sums and a 48-byte search state,
 * 512 KiB + 48 B, held by each GPU the library runs on until the process
 * ends; the amount does not grow
 * with nelem: the update's partials are bounded by its launch grid).  The
 * first call on a device looks up that device's copy (hipGetSymbolAddress,
 * with the device current); no call calls hipMalloc, hipFree or any other
 * allocating routine, and none synchronises.
 *   nelem: elements, 1 <= nelem <= FE_NOALLOC_MAX_ELEMS = 2^31 - 1 (else
 *          FE_EINVAL; the scratch is the same for every nelem up to it);
 *   x, dcx, dv, x_new, change: device float64 arrays of nelem entries
 *   (change: one scalar, may be NULL), as for oc_update; x and x_new may
 *   alias.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (each call writes every entry before reading it, so nothing needs
 * clearing): calls that may overlap on one GPU (different streams, threads)
 * race and must be ordered by the caller.  Asynchronous; errors of the launch
 * are returned as FE_EDEVICE. */
#define FE_NOALLOC_MAX_ELEMS 2147483647LL
FE_API fe_status oc_update_noalloc(int64_t nelem, const double* x, const double* dcx, const double* dv,
                                   double volfrac, double move, double* x_new, double* change, void* stream);

/* Coarse-grained design variables of the two-scale scheme (Sec. III-C and
 * III-E, the coarse-graining step of Alg. 1): zc[ec] is the mean of z over
 * the nb x nb x nb block of fine elements of coarse element ec.  z is
 * float64[nelem] in the fine element order; zc is float64[nelem / nb^3] in
 * the element order of the (nx/nb) x (ny/nb) x (nz/nb) coarse grid, coarse
 * element (I, J, K) holding fine elements i = nb I .. nb I + nb - 1 (and the
 * same in y, z).  Both are device arrays owned by the caller and must not
 * alias.  FE_EINVAL unless 1 <= nb and nb divides nx, ny and nz.  The coarse
 * problem of the scheme is an fe_problem of that grid with element edge nb h
 * and filter radius filter_r / nb (the same physical radius).
 * Asynchronous. */
FE_API fe_status fe_block_mean(fe_problem* p, const double* z, int32_t nb, double* zc);

/* Initial guess of the next solve of an optimisation loop.  The loop of
 * Algorithm 1 (Sec. III-D's problem solved once per design update) solves a
 * sequence of nearby systems; starting each from the linear extrapolation of
 * the last two solutions instead of the last one alone saves iterations
 * (the 224 x 112 x 56 cantilever loop: 73.8 -> 67.5 CG iterations per solve
 * to the same tolerance).  Per dof: u <- u + theta (u - u_hist), then
 * u_hist <- the old u.  u: the last solution (float64[ndof], device, in the
 * layout of fe_solve); u_hist: the caller's history array of the same size
 * (the solution before it; theta = 0 only records u there).  Fixed dofs stay
 * zero.  FE_EINVAL for NULL or aliasing arrays or theta outside [0, 4].
 * Asynchronous, on the handle's stream. */
FE_API fe_status fe_extrapolate(fe_problem* p, double* u, double* u_hist, double theta);

/* Multigrid parameters (used when precond = FE_PRECOND_GMG): nu damped
 * Jacobi sweeps (damping omega) before and after each coarse correction
 * (1..8), and the degree (1..10000) of the Jacobi-preconditioned Chebyshev
 * iteration that solves the coarsest level, on the interval
 * [lambda_max / coarse_ratio, lambda_max] (2 <= coarse_ratio <= 1e12) with
 * lambda_max = largest eigenvalue of diag(Ke)^-1 Ke (5.32 for nu = 0.3),
 * which bounds that of D^-1 K for any density field.  Defaults: nu = 1,
 * omega = 0.35, and for the coarsest grid's longest dimension n the degree
 * 2 clamp(round(12 n / 28), 4, 24) and coarse_ratio
 * max(50, 5000 min(1, (n / 56)^2)) (48 and 5000 at n = 56, the 224 x 112 x 56
 * grid with 3 levels).  The V-cycle is linear and
 * symmetric, and positive definite while omega * lambda_max < 2 (checked:
 * FE_EINVAL otherwise; the Chebyshev residual polynomial stays in (0, 1)
 * below the interval for any ratio), so plain CG applies. */
FE_API fe_status fe_set_mg_params(fe_problem* p, int32_t nu, int32_t coarse_sweeps, double omega,
                           double coarse_ratio);

/* Smoothing of the levels between the finest and the coarsest.  With
 * cheb_from_level = k (1 <= k <= levels - 2), levels k .. levels - 2 are
 * smoothed by `degree` steps of Jacobi-preconditioned Chebyshev iteration on
 * [lambda_max / ratio, 1.02 lambda_max] (lambda_max as in fe_set_mg_params)
 * instead of damped Jacobi sweeps: from zero before the coarse correction
 * (the restricted residual is the iteration's own), and on the residual
 * r - K z after it (the same polynomial in D^-1 K times D^-1, so the cycle
 * stays symmetric; the Chebyshev residual polynomial stays below 1 in
 * magnitude on the whole spectrum, so the smoother converges for any
 * ratio).  The steps run in the launches the coarsest-level solve uses
 * (fe_set_coarse_fusion).  cheb_from_level = 0: damped Jacobi on every
 * level (degree and ratio ignored).  Default: level 2 on, degree 6, ratio
 * 100, for hierarchies of four or more levels whose coarsest grid has 24 or
 * more elements along its longest axis; off otherwise.  FE_EINVAL
 * for other values and on batch slots.  fe_get_mg_smoother returns the
 * setting in effect (0: off); its output pointers are host memory and may
 * be NULL. */
FE_API fe_status fe_set_mg_smoother(fe_problem* p, int32_t cheb_from_level, int32_t degree, double ratio);
FE_API fe_status fe_get_mg_smoother(const fe_problem* p, int32_t* cheb_from_level, int32_t* degree,
                             double* ratio);

/* Levels first_level .. nlev-1 of the multigrid preconditioner of
 * FE_PREC_FP64 solves run in float32 on their float32 moduli and inverse
 * diagonals.  first_level = 0 (default): the whole V-cycle, the finest
 * level's smoothing included, reads a float32 copy of the residual that the
 * CG update writes, and the CG direction kernel reads its float32 result
 * directly; first_level >= 1:
 * the restriction into first_level sums in float64 and rounds once, the
 * prolongation out of it widens the correction; first_level = nlev keeps the
 * preconditioner in float64.  The CG itself (the operator K p, its vectors,
 * reductions and the returned residual) stays float64 either way, and the
 * preconditioner remains a fixed linear map up to float32 rounding.  No
 * effect on float32 inner solves.  FE_EINVAL unless 0 <= first_level <=
 * nlev. */
FE_API fe_status fe_set_float32_levels(fe_problem* p, int32_t first_level);

/* The multigrid parameters in effect (the defaults above or the last
 * fe_set_mg_params); each output pointer is host memory and may be NULL. */
FE_API fe_status fe_get_mg_params(const fe_problem* p, int32_t* nu, int32_t* coarse_sweeps, double* omega,
                           double* coarse_ratio);

/* Launches of the Chebyshev steps (the coarsest-level solve and the
 * Chebyshev smoothing of middle levels; on small grids they are bound by
 * launch and memory latency, not by arithmetic):
 *   5: three steps in one launch on 3D tiles with a three-node halo, of
 *     2 x 2 x 4, 2 x 4 x 4 or 4 x 4 x 4 nodes (the smallest whose launch has
 *     at most one workgroup per compute unit; float32 levels, float64 ones
 *     take form 3), the remainder in pairs (a single step for an odd
 *     remainder);
 *   3, 4: pairs of steps in one launch on 3D tiles (a workgroup owns 4 x 4 x 4
 *     nodes (3) or 4 x 4 x 8 (4; float32 levels only, float64 levels take
 *     4 x 4 x 4), works on all their levels at once and recomputes the
 *     two-node halo its second step needs);
 *   2: pairs of steps in one launch on z-marching tiles (each workgroup
 *     recomputing the ring of first-step values its second step needs);
 *   1: one launch per step;
 *   0 (default), per level: 5 while a launch on 4 x 4 x 4 blocks (every
 *     batch slot included) has at most one workgroup per compute unit,
 *     else 4 while that holds for 4 x 4 x 8 blocks, else 2.
 * 1 and 2 give bitwise the same result, and so do 3 and 5 for even
 * degrees; 3, 4 and 5 apply the same polynomial with their node sums
 * rounded in another order than 1 and 2 (each bitwise reproducible).
 * FE_EINVAL for other values and for batch slots. */
FE_API fe_status fe_set_coarse_fusion(fe_problem* p, int32_t steps_per_launch);

/* Timing of the hot kernels: with on = 1 every launch of the matrix-free
 * K*u on the finest grid, in all its forms (CG product, residual, smoothing
 * sweep), is bracketed by HIP events on the handle's stream; with on = 2 + m
 * only the launches of form m (1 = CG product, 3 = smoothing sweep,
 * 4 = residual, 5 = last smoothing sweep with r^T z, 6 = Chebyshev step,
 * 0 = plain product), and with m = 7 each coarsest-level Chebyshev solve
 * (its launches of two or three steps, the largest share of a multigrid solve's
 * time, bracketed as one: a launch of a few microseconds is shorter than an
 * event pair's own cost); on = 0 switches it off, other values are
 * FE_EINVAL.
 * fe_kernel_stats returns the number of launches and their summed duration
 * in ms since the last reset, and the mean algorithmic bytes of one launch
 * (each array the kernel reads or writes counted once).  Launches that met
 * the CG stop flag (the iterations of a captured chunk after the solve
 * stopped inside it return at once) are not counted. */
FE_API fe_status fe_set_profiling(fe_problem* p, int32_t on);
FE_API fe_status fe_kernel_stats(fe_problem* p, int32_t reset, int64_t* launches,
                          double* total_ms, double* bytes_per_launch);

/* Cold-cache timing of the profiled launches (measurement only): with buf
 * set (device memory of `bytes` >= 512 MB, 16-byte aligned, owned by the
 * caller and overwritten: every 32-bit word is incremented once per profiled
 * launch), every launch that fe_set_profiling brackets with events is
 * preceded by a kernel that streams once through buf, so the launch finds
 * none of its operands in the 256 MB last-level cache or in the XCDs' L2
 * caches and its timing is that of data coming from HBM.  The time of the
 * streaming kernel itself is outside the event pair.  buf = NULL switches
 * it off.  Captured CG chunks are re-captured on the next solve.
 * FE_EINVAL for a smaller or misaligned buffer. */
FE_API fe_status fe_set_cache_flush(fe_problem* p, void* buf, size_t bytes);

/* Release the handle (the workspace stays the caller's). */
FE_API void fe_destroy(fe_problem* p);

/* ---- Batches: many designs of one configuration in shared launches ----
 * The serving form of the step (continuous batching of design solves).  A
 * batch holds nslots problems of one configuration (multigrid; FE_PREC_FP64
 * or FE_PREC_FP32_IR) in one caller workspace.  Their CG iterations run as
 * one captured HIP graph whose every launch covers all slots (one slot per
 * grid y index); a slot whose CG is stopped (empty, finished, or between
 * refinement steps) costs an early exit, so designs join and leave a batch
 * between replays while the others keep iterating.  Everything else of a
 * slot (setup, solve start, float64 residuals, sensitivity, filter, OC) runs
 * per slot on the batch's stream through the usual calls on its handle. */
typedef struct fe_batch fe_batch;

/* Bytes of device workspace for a batch of nslots (0 if cfg or nslots is
 * invalid for a batch: 1 <= nslots <= 1024). */
FE_API size_t fe_batch_workspace_size(const fe_config* cfg, int32_t nslots);

/* Creates the batch on ws (device, 256-byte aligned, >= the size above; the
 * caller keeps it alive until fe_batch_destroy) with every slot idle.  All
 * work of the batch and its slots is ordered on `stream`.  Errors:
 * FE_EINVAL, FE_ENOMEM (workspace too small), FE_EDEVICE. */
FE_API fe_status fe_batch_create(const fe_config* cfg, int32_t nslots, void* ws, size_t ws_bytes,
                          void* stream, fe_batch** out);

/* (Re)initialises slot `slot` for a new design (supports `fixed`, load `f`,
 * as for fe_setup; f = NULL: no load) and returns its handle, owned by the
 * batch: valid until the slot is set up again or the batch is destroyed,
 * never passed to fe_destroy.  Start its solve with fe_solve_begin; the
 * batch's rounds advance it; fe_solve_step reports (without advancing)
 * whether it finished; then fe_solve_end.  fe_solve and fe_set_mg_params are
 * FE_EINVAL on a slot (the multigrid parameters are the library defaults).
 * FE_EINVAL if the slot's previous solve is still running or a round is
 * open. */
FE_API fe_status fe_batch_setup_slot(fe_batch* b, int32_t slot, const uint8_t* fixed, const double* f,
                              fe_problem** out);

/* One round, in two halves so that several batches (on different streams)
 * overlap: begin enqueues one replay of the batched CG chunk and the state
 * copies; end waits for them and advances every running slot by one stage,
 * returning the number of slots still running.  A slot whose new stage only
 * waits for a short computation whose result the host needs (the float64
 * residual of a refinement step, the final residual and compliance) is
 * advanced again after one wait for the batch's stream, so that it rejoins
 * the next replay, or finishes, within the same call instead of sitting a
 * round out.  A slot that fails stops with its status in fe_solve_end; the
 * first such status is also returned. */
FE_API fe_status fe_batch_round_begin(fe_batch* b);
FE_API fe_status fe_batch_round_end(fe_batch* b, int32_t* running);

/* Whether the open round's work has completed on the device, without
 * waiting (*ready = 1: fe_batch_round_end does not wait for the replay; also 1
 * when no round is open), so that a serving loop can end and restart each
 * batch's rounds as they complete instead of in lockstep. */
FE_API fe_status fe_batch_round_ready(fe_batch* b, int32_t* ready);

/* Releases the batch and its slots' handles (the workspace stays the caller's). */
FE_API void fe_batch_destroy(fe_batch* b);

/* ---- Online neural synthetic gradients (Sec. III-B/C/E, Alg. 1) --------
 * A sample is one block of nb x nb x nb fine elements (the coarse elements
 * of the two-scale scheme, in coarse element order): its input is the
 * block's design variables z (x fastest, then y, then z) followed by the 24
 * displacements u_C of its coarse element (corner order (0,0,0) (1,0,0)
 * (1,1,0) (0,1,0) (0,0,1) (1,0,1) (1,1,1) (0,1,1), 3 dofs each) divided by
 * max |u_C| of that iteration; its target is the exact gradient dJ/dz of
 * the block's elements divided by max |dJ/dz| of that iteration.  A
 * prediction is therefore a gradient up to a positive factor, which the OC
 * update does not see (its multiplier absorbs it).  The network: nb^3 + 24 inputs, four hidden layers of
 * `width` with ReLU, a linear output of nb^3; parameters per layer W
 * (out x in, row-major) then b (out), all layers in one vector of
 * fe_onsg_num_params(nb, width) values.  Float32 arithmetic; the dense
 * products are rocBLAS GEMMs.  All pointers are device memory owned by the
 * caller unless stated; calls are asynchronous on the stream of
 * fe_onsg_create except where stated. */
typedef struct fe_onsg fe_onsg;

/* Parameter count of the network for block size nb and hidden width
 * (0 if nb is not in [1, 16] or width not in [1, 8192]). */
FE_API int64_t fe_onsg_num_params(int32_t nb, int32_t width);

/* Bytes of device workspace for a model of the (nx, ny, nz) grid, block
 * size nb (dividing nx, ny, nz; <= 16), hidden width (1..8192), at most
 * max_samples stored samples and mini-batches of `batch` rows; 0 if an
 * argument is invalid.  Pure host arithmetic. */
FE_API size_t fe_onsg_workspace_size(int32_t nx, int32_t ny, int32_t nz, int32_t nb, int32_t width,
                              int32_t max_samples, int32_t batch);

/* Creates the model in ws (256-byte aligned, >= fe_onsg_workspace_size)
 * with the initial parameters params (float64, rounded to float32) and the
 * stream (hipStream_t, NULL = default).  The
 * rocBLAS handle it creates holds memory of its own until
 * fe_onsg_destroy.  FE_EINVAL / FE_ENOMEM on bad arguments. */
FE_API fe_status fe_onsg_create(int32_t nx, int32_t ny, int32_t nz, int32_t nb, int32_t width,
                         int32_t max_samples, int32_t batch, const double* params,
                         void* ws, size_t ws_bytes, void* stream, fe_onsg** out);

/* Appends the samples of every block of one exact iteration (Alg. 1's
 * training set grows by one iteration): z (nelem design variables), uc
 * (coarse-mesh displacements, 3 (nx/nb + 1)(ny/nb + 1)(nz/nb + 1)), g
 * (nelem exact gradients dJ/dz), float64.  FE_EINVAL when max_samples would
 * be exceeded. */
FE_API fe_status fe_onsg_add_samples(fe_onsg* m, const double* z, const double* uc, const double* g);

/* Number of stored samples (host output, immediate). */
FE_API fe_status fe_onsg_num_samples(const fe_onsg* m, int64_t* n);

/* One model update: `steps` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected, moments restarted), step t on the mini-batch of samples
 * idx[t * batch .. t * batch + batch - 1] (int32, device; an index outside
 * [0, num_samples) is clamped into it), learning rate lr0 halved every
 * halve_every steps, loss = mean squared error over the batch and outputs;
 * losses (float32[steps], device, may be NULL) receives each step's batch
 * loss before its update. */
FE_API fe_status fe_onsg_train(fe_onsg* m, int32_t steps, const int32_t* idx, double lr0, int32_t halve_every,
                        float* losses);

/* Synthetic gradient of every element (float64 g[nelem], device) from the
 * design z and the coarse displacements uc, as laid out above: the
 * network's outputs, in units of the largest gradient of an iteration. */
FE_API fe_status fe_onsg_predict(fe_onsg* m, const double* z, const double* uc, double* g);

/* The current parameters as float64 (device array of the parameter count). */
FE_API fe_status fe_onsg_get_params(const fe_onsg* m, double* params);

/* Waits for the model's stream and releases the handle (ws stays the caller's). */
FE_API void fe_onsg_destroy(fe_onsg* m);

/* Message of the last failure on this thread ("" if none). */
FE_API const char* fe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FE_ABI_H */
