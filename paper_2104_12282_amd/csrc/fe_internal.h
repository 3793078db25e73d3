// Internal declarations of the gfx950 finite-element library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <type_traits>
#include <vector>

#include "fe_abi.h"

#define FE_BLOCK 256
#define FE_MAX_LEVELS 6
#define FE_RED_GRID 4096  // grid of the reduction kernels (partials per slot)
#define FE_OC_PARTIALS 65536  // partial sums an OC update needs (max of FE_RED_GRID and 1024 x 64)
#ifndef FE_IR_FACTOR
#define FE_IR_FACTOR 0.3  // refinement: the inner solve aims at FE_IR_FACTOR x the outer target
#endif
#ifndef FE_IR_FLOOR
#define FE_IR_FLOOR 1e-5  // refinement: tightest relative tolerance asked of a float32 inner solve
#endif
#ifndef FE_IR_FLOOR_BF16
#define FE_IR_FLOOR_BF16 1e-1  // refinement over the bf16 contraction: tightest inner tolerance
#endif
#define FE_CS_OFF 99  // first multigrid level smoothed by Chebyshev steps: none
#ifndef FE_CHEB_TRIPLES
#define FE_CHEB_TRIPLES 1  // automatic coarse form: three steps per launch where 4 x 4 x 4 blocks fit
#endif
#ifndef FE_CHEB3_SHAPE
#define FE_CHEB3_SHAPE 0  // blocks of the three-step launches: 0 automatic, 1: 4x4x4, 2: 2x4x4, 3: 2x2x4 nodes
#endif
#ifndef FE_CS_DEG
#define FE_CS_DEG 6  // default Chebyshev smoothing steps
#endif
#ifndef FE_CS_RATIO
#define FE_CS_RATIO 100.0  // default Chebyshev smoothing interval ratio
#endif
#ifndef FE_IR_PHASE
#define FE_IR_PHASE 5e-3  // refinement with residual replacement: reduction of the residual per phase
#endif
#ifndef FE_IR_RESUME
#define FE_IR_RESUME 1  // refinement: continue the float32 CG with the float64 residual (no restart)
#endif
#ifndef FE_CHEB_FORM
#define FE_CHEB_FORM 0  // default launch form of the coarsest-level Chebyshev steps (0: automatic)
#endif
#define FE_MAX_STENCIL 2304  // density-filter stencil entries (radius <= 8 elements)

// Structured brick grid of one multigrid level.
struct Grid {
  int32_t nx, ny, nz;
  int64_t nelem, nnode, ndof;
};

// Device-resident state of one CG instance.  Scalars are written by the
// last workgroup of a kernel and read by the following kernels, so the loop
// runs with no host round trip per iteration.
struct CgState {
  double rz;      // r^T z of the current iterate
  double alpha;   // step length of the current iteration
  double beta;    // direction update factor
  double rr;      // ||r||^2
  double bb;      // ||b||^2 (right-hand side)
  double tol2;    // stop when rr <= tol2
  double pq;      // p^T K p
  double x_alpha; // folded multigrid CG: step of a deferred x update (x += x_alpha x_dir)
  double rz_new;  // r^T z of the new preconditioned residual (multigrid CG, not yet committed)
  int32_t iter;   // iterations done
  int32_t max_iter;
  int32_t done;   // 1 = stop (converged, capped or broken down)
  int32_t status; // FE_OK, FE_ENOTCONV, FE_EBREAKDOWN
  int32_t iter_next;  // iteration count after the update in flight (multigrid CG)
  uint32_t counter[8];  // arrival counters of the last-block reductions
  void* x_dir;    // the direction of the deferred x update (a vector of the solve's type)
};

// Constants of the element operator in the per-axis sum/difference basis.
// With t = V u_e (V = Walsh transform of the 8 corners, per component),
// Ke u_e = V S t / 64 and S has the sparsity of an isotropic cube:
//   A, B  : normal-strain block of the three linear modes
//   G     : shear pairs of the linear modes
//   C, D  : bilinear-mode pairs, F, H : bilinear triple, J : trilinear mode.
// The stored values already include the 1/64.
struct WalshK {
  double A, B, G, C, D, F, H, J;
};

struct Level {
  Grid g;
  double h;
  // device arrays (inside the workspace)
  double* E64 = nullptr;     // element moduli
  float* E32 = nullptr;
  double* invd64 = nullptr;  // 1 / Jacobi diagonal per node
  float* invd32 = nullptr;
  uint8_t* nmask = nullptr;  // bit c set = dof c of the node is fixed
  // multigrid work vectors (float32 or float64 by precision)
  void* mg_r = nullptr;
  void* mg_z = nullptr;
  void* mg_t = nullptr;
  void* mg_w = nullptr;
  void* mg_q = nullptr;  // levels below the finest: second residual of the fused Chebyshev steps
  void* mg_s = nullptr;  // levels between the finest and the coarsest: third residual
};

struct KStats {
  bool on = false;
  int mode = -1;               // only launches of this form (-1: all)
  std::vector<hipEvent_t> ev;  // pairs
  std::vector<double> bytes;   // algorithmic bytes of each recorded launch
  int64_t pending = 0;         // recorded pairs not yet read
  int64_t launches = 0;
  double total_ms = 0.0;
  double total_bytes = 0.0;
  // cold-cache timing: a caller buffer streamed through (read and written)
  // before every profiled launch, larger than the last-level cache
  uint32_t* flush = nullptr;
  size_t flush_words = 0;
  // while a graph is being captured, event pairs go to the graph's own lists
  std::vector<hipEvent_t>* cap_ev = nullptr;
  std::vector<double>* cap_bytes = nullptr;
};

// One captured chunk of CG iterations (per vector type).
struct GraphChunk {
  hipGraphExec_t exec = nullptr;
  bool prof = false;            // captured with profiling events
  std::vector<hipEvent_t> ev;   // event pairs recorded by each replay
  std::vector<double> bytes;
  int iters = 0;                // CG iterations of the chunk
  int iter0 = 0;                // completed CG iterations when the last replay was launched
};

// The OC update captured as one graph for the arrays and parameters of the
// call it serves; a key met for the first time is launched directly and
// recorded, its second call captures.
struct OcGraph {
  hipGraphExec_t exec = nullptr;
  const void* key[5] = {};
  double volfrac = 0.0, move = 0.0;
  bool seen = false;
};

// Non-blocking solve: a host state machine advanced by fe_solve_step; every
// stage ends with a copy of the few scalars it needs into pinned host memory
// and an event.
struct SolveCtx {
  int stage = 0;
  double rtol = 0.0;
  int max_iters = 0;
  double* u = nullptr;
  int total = 0, outer = 0;
  double prev_rel = 1e300;
  int fresh_inner = 0;          // the inner CG state was just initialised
  bool can_resume = false;      // the next refinement step may continue the float32 CG
  int inner_base = 0;           // refinement iterations before the running float32 CG
  int chunk_iter0 = 0;          // CG iteration at which the last chunk started
  double inner_rr = 0.0;        // ||r||^2 the running float32 CG is scaled by
  double mark_rr = 0.0;         // ||r||^2 of the running CG at iteration mark_iter
  int mark_iter = -1;           // (-1: none yet) -- its convergence rate sizes the next chunk
  double rate = 0.0;            // ||r||^2 ratio per CG iteration last measured (0: none)
  fe_status result = FE_OK;
  fe_solve_info info{};
};

// Brackets the next launch on p->stream with a pair of events when profiling
// is on (returns the slot, or -1).
int kstats_begin(fe_problem* p, double bytes);
void kstats_end(fe_problem* p, int slot);

struct fe_problem {
  fe_config cfg;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int nlev = 1;
  Level L[FE_MAX_LEVELS];

  double ke64_host[576];
  double* ke64 = nullptr;  // dense Ke (device copy)
  float* ke32 = nullptr;
  WalshK wk;               // for h = 1 per level scaled by h
  double ke_diag = 0.0;    // common diagonal entry of Ke (unit modulus, edge h)

  double* f = nullptr;     // load, zero on fixed dofs
  double* invW = nullptr;  // 1 / filter row sums
  double* zpad = nullptr;  // 64 zero bytes: the source of loads outside the mesh
  int nstencil = 0;             // filter stencil: LDS offsets in the filter tile, cone weights
  int* st_lin = nullptr;
  double* st_w = nullptr;
  int st_halo = 0, st_tz = 4;  // the stencil's reach, the filter tile's depth

  // float64 CG vectors
  double *r64 = nullptr, *p64 = nullptr, *q64 = nullptr;
  double* p64b = nullptr;  // second direction buffer (multigrid CG alternates the two)
  // float32 CG vectors (iterative refinement)
  float *x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr;
  float* p32b = nullptr;
  // scratch
  double* tmp64 = nullptr;
  double* partials = nullptr;  // 4 regions of part_stride doubles (see part_region)
  int64_t part_stride = 0;     // doubles per CG region
  int64_t part_gen = 0;        // doubles of the general region

  CgState* st = nullptr;       // device state (two instances: [0] inner, [1] aux)
  double* scal = nullptr;      // 64 device scalars for small results
  double* oc = nullptr;        // OC search state

  // solve state machine, pinned host mirrors, captured CG chunks
  SolveCtx sc;
  CgState* h_st = nullptr;      // pinned
  double* h_scal = nullptr;     // pinned, 4 values
  hipEvent_t done_ev = nullptr;
  hipStream_t cap_stream = nullptr;
  // captured CG chunks per vector type, one per length: q, 2q, 3q, 4q
  // iterations (q = a quarter of the full chunk, an even number)
  GraphChunk chunk64[4], chunk32[4];
  OcGraph ocg;
  GraphChunk* last_replay = nullptr;  // profiled graph replayed since the last harvest
  bool use_graphs = true;
  bool in_batch = false;  // a slot of an fe_batch: its CG chunks run in the batch's replays
  bool start_pending = false;  // batch slot: its CG (re)start awaits the batch's shared first V-cycle
  int mfma_l0 = 0;  // finest-grid float32 K*u: 0 vector ALUs, 1 bf16, 2 split-bf16 matrix cores
  double* x64 = nullptr;        // float64 iterate of the solve (graphs need fixed pointers)
  double ff = 0.0;              // ||f||^2

  // geometric multigrid parameters
  int mg_nu = 1;               // damped Jacobi sweeps before and after the coarse correction
  int mg_coarse_sweeps = 48;   // Chebyshev degree on the coarsest level
  double mg_omega = 0.35;      // Jacobi damping: below 2 / lambda_max(D^-1 Ke) = 2 / 5.32
  double lam_max = 0.0;        // lambda_max(diag(Ke)^-1 Ke): bounds that of D^-1 K on every level
  double cheb_ratio = 5000.0;  // coarse Chebyshev interval [lam_max / ratio, lam_max]
  // Chebyshev smoothing (instead of damped Jacobi) on levels cs_from .. nlev - 2:
  // cs_deg steps before and after the coarse correction on [lam_max / cs_ratio, lam_max]
  int cs_from = FE_CS_OFF;
  int cs_deg = FE_CS_DEG;
  double cs_ratio = FE_CS_RATIO;
  int cheb_per_launch = FE_CHEB_FORM;  // coarse Chebyshev launches: 3 / 4 pairs of steps on 3D tiles of
                                      // 4 x 4 x 4 / 4 x 4 x 8 nodes, 2 pairs on z-marching tiles, 1 one
                                      // step each, 0 chosen per launch
  int f32_from = 1 << 30;      // float64 solves run multigrid levels >= f32_from in float32

  KStats kst;

  // batched launches: while bcount > 1 (a batch's captured CG chunk) every
  // kernel of the chunk runs bcount problems, one per grid y index, whose
  // workspaces lie bstride bytes apart (this problem's is the first)
  int bcount = 1;
  int64_t bstride = 0;
};

// Byte offset of this workgroup's problem in a batched launch, and a pointer
// moved by it (null stays null).
__device__ inline int64_t batch_offset(int64_t wsh) { return (int64_t)blockIdx.y * wsh; }
// Byte arithmetic on a char pointer (not on an integer) keeps the pointer's
// address space visible to the compiler, so shifted pointers still load with
// global (not flat) instructions.
template <typename P>
__device__ inline P* wshift(P* ptr, int64_t off) {
  using B = std::conditional_t<std::is_const<P>::value, const char, char>;
  return ptr ? reinterpret_cast<P*>(reinterpret_cast<B*>(ptr) + off) : ptr;
}

// Partial-sum regions.  Multigrid CG hands each reduction to the next kernel
// (which sums the partials itself), so producer and consumer must not share
// a region: GEN is for one-shot reductions finished by cg_finalize, PQ for
// p^T K p, RR for r^T r, RZ for r^T z.
enum { PART_GEN = 0, PART_PQ = 1, PART_RR = 2, PART_RZ = 3, PART_REGIONS = 4 };
inline double* part_region(const fe_problem* p, int k) {
  return k == PART_GEN ? p->partials : p->partials + p->part_gen + (k - 1) * p->part_stride;
}

// ------------------------------------------------------------------ host
void fe_set_error(const std::string& msg);
int host_hex8_ke(double nu, double E, double h, double* Ke /*576*/);
int host_walsh_constants(const double* Ke, WalshK* wk, double* max_dev);

// ------------------------------------------------------------- launchers
// All launchers enqueue on p->stream and return hipGetLastError().
hipError_t launch_simp(fe_problem* p, int lev, const double* rho);
hipError_t launch_coarsen_modulus(fe_problem* p, int lev);  // E[lev] from E[lev-1]
hipError_t launch_diag(fe_problem* p, int lev);
hipError_t launch_node_mask(fe_problem* p, const uint8_t* fixed);
hipError_t launch_coarsen_mask(fe_problem* p, int lev);
hipError_t launch_mask_load(fe_problem* p, const double* f);
template <typename T>
hipError_t launch_mask_vec(fe_problem* p, int lev, T* v);

// y = K x (masked) on level lev; if st != nullptr also accumulates x^T y and
// finalises alpha = rz / pq into st (CG step).
template <typename T>
hipError_t launch_kxu(fe_problem* p, int lev, const T* x, T* y, CgState* st);

// Operands of one Chebyshev step (mode 6 of the tiled kernel).
template <typename T>
struct ChebStep {
  T* res;      // residual, updated in place
  T* acc;      // iterate, updated in place
  double c1, c2;
  int first;   // iterate starts at zero
};

// The tiled kernel behind launch_kxu: mode 0 y = Kx, 1 CG step (st), 2 y = b64 - Kx
// with ||y||^2 -> out[0] (float64 only), 3 damped Jacobi y = x + omega D^-1 (bT - Kx),
// 4 y = bT - Kx, 5 mode 3 plus r^T z for CG, 6 Chebyshev step with direction x.
// Optional fused input and reduction of a tiled launch.
//   xin 1: the operand is x = s * D^-1 a, formed on the fly (a first Jacobi
//          sweep from zero); owners store it to xout when xout is non-null.
//   xin 2: the operand is the CG direction x = z + beta * pold (z on the
//          first iteration), beta = rz / rz_old with rz summed from the
//          nfold partials at fold; owners store it to xout.
//   fold_rr: before its work every workgroup sums the nfold r^T r partials at
//          fold and takes the convergence decision of the CG update.
//   part: partials region of modes 1 and 5; no_finalize: leave them for the
//          next kernel instead of a one-workgroup finalize.
template <typename T>
struct TileFuse {
  int xin = 0;
  const T* invd = nullptr;  // xin 1
  double s = 0.0;           // xin 1
  const T* pold = nullptr;  // xin 2
  T* xout = nullptr;
  const double* fold = nullptr;
  int nfold = 0;
  bool fold_rr = false;
  double* part = nullptr;
  bool no_finalize = false;
  int* nblocks = nullptr;   // out: workgroups launched
};

template <typename T>
hipError_t launch_kxu_tile(fe_problem* p, int lev, const T* x, const T* E, T* y, CgState* st, int mode,
                           const double* b64, double* out, const T* bT = nullptr,
                           const T* invd = nullptr, double omega = 0.0,
                           const ChebStep<T>* cs = nullptr, const TileFuse<T>* fz = nullptr);
int64_t kxu_tile_blocks(const Grid& g);
// Two Chebyshev steps (mode 6 twice) on level lev in one launch: from the
// direction dk, residual rin and iterate acc (in place) to the direction
// y = d_{k+2} and residual rout (rin and rout must differ); c = c1, c2 of
// step k, then of step k + 1; first: step k starts the iterate.  The result
// is bitwise that of two mode-6 launches.  dscale != 0: d_k is not read but
// formed in the launch as dscale D^-1 r_k (the first direction; only the 3D
// tile forms do, see cheb2_forms_first_direction; hipErrorInvalidValue
// otherwise).
template <typename T>
hipError_t launch_cheb2(fe_problem* p, int lev, const T* dk, T* y, const T* E, const T* invd, const T* rin,
                        T* rout, T* acc, const double (&c)[4], int first, CgState* st, double dscale = 0.0);
template <typename T>
bool cheb2_forms_first_direction(const fe_problem* p, int lev);
// Three steps per launch (4 x 4 x 4 blocks with a three-node halo; float32
// levels whose launch fits one workgroup per compute unit, or form 5 asked
// for): c = c1, c2 of steps k, k + 1, k + 2; otherwise as launch_cheb2.
template <typename T>
bool cheb_triples(const fe_problem* p, int lev);
template <typename T>
hipError_t launch_cheb3(fe_problem* p, int lev, const T* dk, T* y, const T* E, const T* invd, const T* rin,
                        T* rout, T* acc, const double (&c)[6], int first, CgState* st, double dscale = 0.0);
// Number of r^T z partials the level's last smoothing sweep (mode 5) leaves.
template <typename T>
int kxu_rz_partials(const fe_problem* p, int lev);
// Node-centric dense-Ke reference kernel (float64), kept as a second implementation.
hipError_t launch_kxu_dense64(fe_problem* p, const double* x, double* y);

// z = V(r): one symmetric multigrid V-cycle from level l down.  st (may be
// null) skips the launches once CG stopped.
// rz: what the last level-0 sweep does with r^T z -- RZ_NONE nothing,
// RZ_FINISH rz and beta into st (one-workgroup finalize), RZ_PARTIALS leave
// the partials in PART_RZ (kxu_rz_partials of them) for the next direction
// kernel.
// With fold_rr > 0 the first level-0 kernel also takes the convergence
// decision of the CG update from the fold_rr r^T r partials in PART_RR.
enum { RZ_NONE = 0, RZ_FINISH = 1, RZ_PARTIALS = 2 };
template <typename T>
hipError_t launch_vcycle(fe_problem* p, int l, const T* r, T* z, CgState* st, int rz, int fold_rr = 0);

// CG helpers (T = float or double vectors, float64 reductions)
template <typename T>
hipError_t launch_cg_init(fe_problem* p, const T* b, const T* Kx, T* r, T* pvec, CgState* st,
                          int precond_mg);
template <typename T>
hipError_t launch_cg_update(fe_problem* p, T* x, T* r, const T* pvec, const T* q, CgState* st,
                            int precond_mg);
template <typename T>
hipError_t launch_cg_direction(fe_problem* p, const T* r, const T* z, T* pvec, CgState* st);
// Multigrid CG update: alpha = rz_new / p^T q from the npq partials in PART_PQ
// (summed by every workgroup), x += alpha p, r -= alpha q, r^T r partials to
// PART_RR; returns their count in *nrr.
// With r32 given, the updated residual is also written there in float32.
template <typename T>
hipError_t launch_cg_update_mg(fe_problem* p, T* x, T* r, const T* pvec, const T* q, CgState* st, int npq,
                               int* nrr, float* r32 = nullptr, const T* pold = nullptr);
// x += st->x_alpha st->x_dir: the x update a multigrid CG deferred when it
// stopped after an iteration that defers it
template <typename T>
hipError_t launch_cg_flush_x(fe_problem* p, T* x, const CgState* st);
// b = (float)a over the finest grid's dofs
hipError_t launch_narrow(fe_problem* p, const double* a, float* b);

hipError_t launch_cg_state_init(fe_problem* p, CgState* st, double tol_rel, int max_iter);
// Re-arms a stopped CG for residual replacement: not done, status FE_OK,
// stop at ||r||^2 <= tol2 (absolute) or max_iter iterations; the iteration
// count and the committed r^T z are kept.
hipError_t launch_cg_state_resume(fe_problem* p, CgState* st, double tol2, int max_iter);
// Sets g->done (a guard state; batched over p's slots while p->bcount > 1).
hipError_t launch_cg_guard(fe_problem* p, CgState* g, int done);
// One-workgroup scalar update after a kernel that left nb partials:
// op 0 alpha = rz / pq, 1 CG start, 2 CG update and convergence test,
// 3 rz and beta, 4 out[0] = the sum.
enum { FIN_ALPHA = 0, FIN_INIT = 1, FIN_UPDATE = 2, FIN_RZ = 3, FIN_SCALAR = 4 };
hipError_t launch_cg_finalize(fe_problem* p, int op, int nb, int mg, CgState* st, double* out);

// float64 residual r = f - K u (masked) and ||r||^2 into scal[slot]
hipError_t launch_residual64(fe_problem* p, const double* u, double* r, double* scal_slot);
// r32 = r64 * scale (scale = 1/||r64|| read on device from scal)
hipError_t launch_to32_scaled(fe_problem* p, const double* r64, float* r32, const double* nrm2);
hipError_t launch_axpy_from32(fe_problem* p, double* u, const float* d, const double* nrm2);
hipError_t launch_dot64(fe_problem* p, const double* a, const double* b, int64_t n, double* out);

// element kernels
hipError_t launch_sensitivity(fe_problem* p, const double* rho, const double* u, double* dc);
hipError_t launch_filter(fe_problem* p, const double* in, double* out, int transpose);
hipError_t launch_filter_rowsums(fe_problem* p);
hipError_t launch_adjoint_sensitivity(fe_problem* p, const double* rho, const double* u, const double* lam,
                                      double* out);
hipError_t launch_block_mean(fe_problem* p, const double* z, int nb, double* zc);
// u <- u + theta (u - hist), hist <- the old u (finest-grid dofs)
hipError_t launch_extrapolate(fe_problem* p, double* u, double* hist, double theta);
hipError_t launch_oc(fe_problem* p, const double* x, const double* dcx, const double* dv,
                     double volfrac, double move, double* x_new, double* change);
// The same update on `stream` with the library's static per-device scratch
// instead of a problem's workspace (no allocation).
hipError_t launch_oc_noalloc(hipStream_t stream, int64_t n, const double* x, const double* dcx, const double* dv,
                             double volfrac, double move, double* x_new, double* change);

// conversions and fills (fill is a kernel, so it is safe inside captured graphs)
template <typename T>
hipError_t launch_fill(fe_problem* p, T* v, int64_t n, T val);
hipError_t launch_convert_64_32(fe_problem* p, const double* a, float* b, int64_t n);
hipError_t launch_convert_32_64(fe_problem* p, const float* a, double* b, int64_t n);
