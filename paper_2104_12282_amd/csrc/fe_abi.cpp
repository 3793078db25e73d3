// C ABI entry points: validation, workspace layout, setup and the solver
// drivers (float64 PCG and float32 PCG inside float64 iterative refinement).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "fe_internal.h"

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// scal[] slots: value at 2*s, arrival counter of its reduction at 2*s + 1.
enum { SLOT_FF = 0, SLOT_RR = 1, SLOT_C = 2, SLOT_TMP = 3, SLOT_IRS = 4, NSCAL = 128 };
// SLOT_IRS: ||r||^2 of the float64 residual the running float32 inner solve was scaled by

Grid make_grid(int nx, int ny, int nz) {
  Grid g;
  g.nx = nx;
  g.ny = ny;
  g.nz = nz;
  g.nelem = (int64_t)nx * ny * nz;
  g.nnode = (int64_t)(nx + 1) * (ny + 1) * (nz + 1);
  g.ndof = 3 * g.nnode;
  return g;
}

int num_levels(const fe_config* c) { return c->precond == FE_PRECOND_GMG ? c->mg_levels : 1; }

std::string validate(const fe_config* c) {
  if (!c) return "cfg is NULL";
  if (c->nx < 1 || c->ny < 1 || c->nz < 1) return "grid dimensions must be >= 1";
  const int64_t nn = (int64_t)(c->nx + 1) * (c->ny + 1) * (c->nz + 1);
  if (3 * nn >= (int64_t)1 << 31) return "grid too large (3*nodes must fit in int32 range)";
  if (!(c->h > 0.0) || !std::isfinite(c->h)) return "h must be > 0";
  if (!(c->nu > -1.0 && c->nu < 0.5)) return "nu must lie in (-1, 0.5)";
  if (!(c->E0 > 0.0) || !std::isfinite(c->E0)) return "E0 must be > 0";
  if (!(c->Emin > 0.0 && c->Emin < c->E0)) return "Emin must lie in (0, E0)";
  if (!(c->penal >= 1.0) || !std::isfinite(c->penal)) return "penal must be >= 1";
  if (!(c->filter_r > 0.0) || c->filter_r > 8.0) return "filter_r must lie in (0, 8]";
  if (c->precision < FE_PREC_FP64 || c->precision > FE_PREC_BF16X3_IR) return "unknown precision";
  if (c->precond != FE_PRECOND_JACOBI && c->precond != FE_PRECOND_GMG) return "unknown preconditioner";
  if (c->reserved != 0) return "reserved must be 0";
  if (c->precond == FE_PRECOND_GMG) {
    if (c->mg_levels < 2 || c->mg_levels > FE_MAX_LEVELS) return "mg_levels must lie in [2, 6]";
  }
  // the stencil table holds at most 512 offsets
  const int R = (int)std::ceil(c->filter_r);
  int cnt = 0;
  for (int dk = -R; dk <= R; ++dk)
    for (int dj = -R; dj <= R; ++dj)
      for (int di = -R; di <= R; ++di)
        if (c->filter_r - std::sqrt((double)(di * di + dj * dj + dk * dk)) > 0.0) ++cnt;
  if (cnt > FE_MAX_STENCIL) return "filter radius too large";
  return "";
}

// One pass assigns every buffer; with base == nullptr it only measures.
size_t layout(const fe_config* c, fe_problem* p, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = align_up(off);
    char* r = base ? base + off : nullptr;
    off += bytes;
    return r;
  };
  const int nl = num_levels(c);
  const bool f32 = c->precision != FE_PREC_FP64;
  const size_t vbytes = f32 ? sizeof(float) : sizeof(double);  // multigrid vector type
  Grid g0 = make_grid(c->nx, c->ny, c->nz);
  int nx = c->nx, ny = c->ny, nz = c->nz;
  double h = c->h;
  int64_t max_blocks = 0;
  for (int l = 0; l < nl; ++l) {
    Grid g = make_grid(nx, ny, nz);
    Level L;
    L.g = g;
    L.h = h;
    L.E64 = (double*)take(g.nelem * sizeof(double));
    L.E32 = (float*)take(g.nelem * sizeof(float));
    L.invd64 = (double*)take(g.nnode * sizeof(double));
    L.invd32 = (float*)take(g.nnode * sizeof(float));
    L.nmask = (uint8_t*)take(g.nnode);
    if (nl > 1) {
      L.mg_r = take(g.ndof * vbytes);
      L.mg_z = take(g.ndof * vbytes);
      L.mg_t = take(g.ndof * vbytes);
      L.mg_w = take(g.ndof * vbytes);
      if (l > 0) L.mg_q = take(g.ndof * vbytes);
      if (l > 0 && l < nl - 1) L.mg_s = take(g.ndof * vbytes);
    }
    if (p) p->L[l] = L;
    int64_t nb = (g.nnode + FE_BLOCK - 1) / FE_BLOCK;
    if (kxu_tile_blocks(g) > nb) nb = kxu_tile_blocks(g);
    if (nb > max_blocks) max_blocks = nb;
    // the next level has ceil(n / 2) elements of twice the edge per axis: an
    // odd axis ends in a coarse element that overhangs the mesh by one fine
    // element (coarse node I sits on fine node 2I, the last one just past
    // the mesh)
    nx = (nx + 1) / 2;
    ny = (ny + 1) / 2;
    nz = (nz + 1) / 2;
    h *= 2.0;
  }
  double* f = (double*)take(g0.ndof * sizeof(double));
  double* invW = (double*)take(g0.nelem * sizeof(double));
  int* st_lin = (int*)take(FE_MAX_STENCIL * sizeof(int));
  double* st_w = (double*)take(FE_MAX_STENCIL * sizeof(double));
  double* r64 = (double*)take(g0.ndof * sizeof(double));
  double* p64 = (double*)take(g0.ndof * sizeof(double));
  double* p64b = (double*)take(g0.ndof * sizeof(double));
  double* q64 = (double*)take(g0.ndof * sizeof(double));
  double* tmp64 = (double*)take(g0.ndof * sizeof(double));
  double* x64 = (double*)take(g0.ndof * sizeof(double));
  float *x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr, *p32b = nullptr;
  if (f32) {
    x32 = (float*)take(g0.ndof * sizeof(float));
    r32 = (float*)take(g0.ndof * sizeof(float));
    p32 = (float*)take(g0.ndof * sizeof(float));
    p32b = (float*)take(g0.ndof * sizeof(float));
    q32 = (float*)take(g0.ndof * sizeof(float));
  }
  // the general region also holds the 64 per-workgroup partials of the OC
  // passes; the CG regions hold up to 3 partials per workgroup of any
  // reducing launch
  int64_t gen = std::max<int64_t>((int64_t)FE_RED_GRID * 64, max_blocks * 3);
  int64_t stride = std::max<int64_t>((int64_t)FE_RED_GRID, max_blocks) * 3;
  gen = (gen + 63) / 64 * 64;
  stride = (stride + 63) / 64 * 64;
  double* partials = (double*)take((size_t)(gen + stride * (PART_REGIONS - 1)) * sizeof(double));
  CgState* st = (CgState*)take(2 * sizeof(CgState));
  double* scal = (double*)take(NSCAL * sizeof(double));
  double* oc = (double*)take(64 * sizeof(double));
  double* ke64 = (double*)take(576 * sizeof(double));
  float* ke32 = (float*)take(576 * sizeof(float));
  double* zpad = (double*)take(8 * sizeof(double));
  if (p) {
    p->nlev = nl;
    p->f32_from = 0;  // the whole preconditioner in float32
    if (nl > 1) {
      // default coarse Chebyshev for the coarsest grid's longest dimension
      // n: the number of steps a Chebyshev solve needs grows like the square
      // root of the condition number, i.e. like n, and the smallest
      // eigenvalue worth resolving like n^-2 (degree 48 and ratio 5000 at
      // n = 56, measured best there; degree ~ 6n/7 measured best from n = 8
      // to 32)
      const Grid& gc = p->L[nl - 1].g;
      const int n = std::max(gc.nx, std::max(gc.ny, gc.nz));
      p->mg_coarse_sweeps = 2 * std::max(4, std::min(24, (int)std::lround(n * 24.0 / 56.0)));
      p->cheb_ratio = 5000.0 * std::min(1.0, (n / 56.0) * (n / 56.0));
      p->cheb_ratio = std::max(p->cheb_ratio, 50.0);
      // from four levels on, on coarsest grids of 24 elements or more along
      // their longest axis, level 2 and below (but the coarsest) are
      // smoothed by Chebyshev steps: with the coarse correction under them
      // they stand in for the long coarse solve a three-level hierarchy
      // spends on that grid (224 x 112 x 56 loop: 75 CG iterations against
      // 112 with damped Jacobi on four levels and 76 with three levels,
      // 48.7 against 37.8 and 42.4 solves/s); on smaller grids the coarsest
      // solve is short and accurate already and the extra launches did not
      // pay (128 x 64 x 64: 39 against 40 iterations)
      p->cs_from = (nl >= 4 && n >= 24) ? 2 : FE_CS_OFF;
    }
    p->f = f;
    p->invW = invW;
    p->st_lin = st_lin;
    p->st_w = st_w;
    p->r64 = r64;
    p->p64 = p64;
    p->p64b = p64b;
    p->q64 = q64;
    p->tmp64 = tmp64;
    p->x64 = x64;
    p->x32 = x32;
    p->r32 = r32;
    p->p32 = p32;
    p->p32b = p32b;
    p->q32 = q32;
    p->partials = partials;
    p->part_stride = stride;
    p->part_gen = gen;
    p->st = st;
    p->scal = scal;
    p->oc = oc;
    p->ke64 = ke64;
    p->ke32 = ke32;
    p->zpad = zpad;
  }
  return align_up(off);
}

#define HIP_TRY(expr)                                                        \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess) {                                                  \
      fe_set_error(std::string(#expr) + ": " + hipGetErrorString(e_));       \
      return FE_EDEVICE;                                                     \
    }                                                                        \
  } while (0)

#define CHECK_HANDLE(p)                     \
  do {                                      \
    if (!(p)) {                             \
      fe_set_error("problem handle is NULL"); \
      return FE_EINVAL;                     \
    }                                       \
  } while (0)

fe_status read_state(fe_problem* p, CgState* host) {
  HIP_TRY(hipMemcpyAsync(host, p->st, sizeof(CgState), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return FE_OK;
}

fe_status read_scal(fe_problem* p, int slot, double* v) {
  HIP_TRY(hipMemcpyAsync(v, p->scal + 2 * slot, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return FE_OK;
}

// Moduli and Jacobi diagonals of every level for the density rho.
fe_status prepare_operator(fe_problem* p, const double* rho) {
  HIP_TRY(launch_simp(p, 0, rho));
  HIP_TRY(launch_diag(p, 0));
  for (int l = 1; l < p->nlev; ++l) {
    HIP_TRY(launch_coarsen_modulus(p, l));
    HIP_TRY(launch_diag(p, l));
  }
  return FE_OK;
}

constexpr int kChunk = 24;    // Jacobi-PCG iterations per enqueued chunk
constexpr int kChunkMG = 8;   // multigrid-PCG iterations per enqueued chunk (even: the folded
                              // iteration alternates two direction buffers)
constexpr int kMaxOuter = 40; // float64 refinement steps
constexpr bool kResumeInner = FE_IR_RESUME != 0;  // residual replacement instead of restarts

enum { ST_DONE = 0, ST_CG64 = 1, ST_IR_RESID = 2, ST_IR_CG = 3, ST_FINISH = 4 };

template <typename T>
T* second_direction(fe_problem* p);
template <>
double* second_direction<double>(fe_problem* p) { return p->p64b; }
template <>
float* second_direction<float>(fe_problem* p) { return p->p32b; }
template <typename T>
const T* fine_E(fe_problem* p);
template <>
const double* fine_E<double>(fe_problem* p) { return p->L[0].E64; }
template <>
const float* fine_E<float>(fe_problem* p) { return p->L[0].E32; }

// Multigrid CG with its reductions folded into the kernels that consume
// them: three launch groups per iteration instead of seven.
//   1. direction + product: p = z + beta p_old (beta from the r^T z partials
//      of the last V-cycle), q = K p, p^T q partials;
//   2. update: alpha, r -= alpha q, r^T r partials, and x += alpha p every
//      second iteration for two steps (x += alpha_1 p_1 + alpha_2 p_2 while
//      both directions are in their buffers; a stop after the deferring
//      iteration applies the last step with cg_flush_x);
//   3. V-cycle z = M r whose first kernel takes the convergence decision and
//      whose last sweep leaves r^T z partials.
// The direction alternates between two buffers (other workgroups still read
// the old one around their tiles while a workgroup writes the new one).
bool folded_mg(const fe_problem* p) { return p->nlev > 1 && !p->mfma_l0; }

// One CG iteration (iteration `it` of its chunk): q = K p (alpha), x/r update
// and convergence test, the preconditioner (multigrid V-cycle with r^T z
// fused, or Jacobi inside the direction kernel), p = z + beta p.  Every
// kernel is guarded by st->done.
template <typename T>
hipError_t cg_iteration(fe_problem* p, T* x, T* r, T* pv, T* q, int it) {
  const bool mg = p->nlev > 1;
  T* z = mg ? static_cast<T*>(p->L[0].mg_z) : nullptr;
  hipError_t e;
  if (folded_mg(p)) {
    T* pb = second_direction<T>(p);
    T* pold = (it & 1) ? pb : pv;
    T* pnew = (it & 1) ? pv : pb;
    int npq = 0, nrr = 0;
    // chunks have even lengths and start at even positions: an even
    // iteration defers its x update to the odd one after it
    T* xu = (it & 1) ? x : nullptr;
    const T* xp = (it & 1) ? pold : nullptr;
    TileFuse<T> fz;
    fz.xin = 2;
    fz.pold = pold;
    fz.xout = pnew;
    // a float64 solve whose preconditioner runs the finest level in float32
    // too: its V-cycle reads a float32 copy of r and leaves z in float32,
    // which the direction kernel reads as such
    const bool f32_l0 = std::is_same<T, double>::value && p->f32_from == 0;
    float* z32 = static_cast<float*>(p->L[0].mg_w);
    if (f32_l0) fz.xin = 3;
    fz.fold = part_region(p, PART_RZ);
    fz.nfold = f32_l0 ? kxu_rz_partials<float>(p, 0) : kxu_rz_partials<T>(p, 0);
    fz.part = part_region(p, PART_PQ);
    fz.no_finalize = true;
    fz.nblocks = &npq;
    if ((e = launch_kxu_tile<T>(p, 0, f32_l0 ? reinterpret_cast<const T*>(z32) : z, fine_E<T>(p), q, p->st, 1,
                                nullptr, nullptr, nullptr, nullptr, 0.0, nullptr, &fz)) != hipSuccess)
      return e;
    if (f32_l0) {
      float* r32 = static_cast<float*>(p->L[0].mg_r);
      if ((e = launch_cg_update_mg<T>(p, xu, r, pnew, q, p->st, npq, &nrr, r32, xp)) != hipSuccess) return e;
      return launch_vcycle<float>(p, 0, r32, z32, p->st, RZ_PARTIALS, nrr);
    }
    if ((e = launch_cg_update_mg<T>(p, xu, r, pnew, q, p->st, npq, &nrr, nullptr, xp)) != hipSuccess) return e;
    return launch_vcycle<T>(p, 0, r, z, p->st, RZ_PARTIALS, nrr);
  }
  if ((e = launch_kxu<T>(p, 0, pv, q, p->st)) != hipSuccess) return e;
  if ((e = launch_cg_update<T>(p, x, r, pv, q, p->st, mg ? 1 : 0)) != hipSuccess) return e;
  if (mg && (e = launch_vcycle<T>(p, 0, r, z, p->st, RZ_FINISH)) != hipSuccess) return e;
  return launch_cg_direction<T>(p, r, z, pv, p->st);
}

template <typename T>
GraphChunk& chunk_of(fe_problem* p, int v);
template <>
GraphChunk& chunk_of<double>(fe_problem* p, int v) { return p->chunk64[v]; }
template <>
GraphChunk& chunk_of<float>(fe_problem* p, int v) { return p->chunk32[v]; }

void drop_graph(GraphChunk& gc) {
  if (gc.exec) (void)hipGraphExecDestroy(gc.exec);
  gc.exec = nullptr;
  for (hipEvent_t e : gc.ev) (void)hipEventDestroy(e);
  gc.ev.clear();
  gc.bytes.clear();
}

void drop_chunks(fe_problem* p) {
  for (int v = 0; v < 4; ++v) {
    drop_graph(p->chunk64[v]);
    drop_graph(p->chunk32[v]);
  }
}

// Full chunk length; chunk variant v (0..3) runs (v + 1) / 4 of it.  Every
// length is even, so a chunk ends with the direction in the buffer it
// started from.
int full_chunk(const fe_problem* p) { return p->nlev > 1 ? kChunkMG : kChunk; }

// Chunk plan at a chunk boundary of a running CG.  Iterations enqueued past
// the stop run as early exits (tens of launches each, a few microseconds
// apiece) and a chunk that ends short of the stop costs a host round trip,
// so the iterations still needed -- from the residual's rate over the last
// chunk, or the previous phase's rate at the start of one -- pick the
// shortest chunk that covers them with one to spare; far from the stop two
// full chunks go out back to back (one round trip for both).  Returns the
// variant and sets *replays (1 or 2).
int plan_chunk(fe_problem* p, const CgState& hs, int* replays) {
  SolveCtx& sc = p->sc;
  *replays = 1;
  // at the first boundary after a residual replacement, hs.rr is still the
  // recurrence's old value: the mark holds the replaced one
  const bool fresh = hs.iter == sc.mark_iter;
  const double rr = fresh ? sc.mark_rr : hs.rr;
  if (!fresh && sc.mark_iter >= 0 && hs.iter > sc.mark_iter && sc.mark_rr > 0.0 && hs.rr > 0.0)
    sc.rate = std::pow(hs.rr / sc.mark_rr, 1.0 / (double)(hs.iter - sc.mark_iter));
  if (!fresh) {
    sc.mark_rr = hs.rr;
    sc.mark_iter = hs.iter;
  }
  const int full = full_chunk(p);
  if (!(sc.rate > 0.0 && sc.rate < 1.0) || !(hs.tol2 > 0.0) || !(rr > hs.tol2)) return 3;
  const double need = std::log(hs.tol2 / rr) / std::log(sc.rate) + 1.0;
  if (need >= 2.5 * full && !p->kst.on) {  // profiled replays are harvested one at a time
    *replays = 2;
    return 3;
  }
  const int v = (int)std::ceil(need / (full / 4)) - 1;
  return v < 0 ? 0 : v > 3 ? 3 : v;
}

// Enqueues a chunk of CG iterations (variant v: (v + 1) / 4 of the full
// length) on p->stream.  The chunk is captured once per problem, vector type
// and length as a HIP graph (on a private stream, then replayed on
// p->stream); with profiling on, the graph carries its own event pairs
// around each fine-grid K*u launch.
template <typename T>
hipError_t enqueue_chunk(fe_problem* p, T* x, T* r, T* pv, T* q, int v = 3) {
  const int n = (v + 1) * (full_chunk(p) / 4);
  GraphChunk& gc = chunk_of<T>(p, v);
  const bool prof = p->kst.on;
  if (p->use_graphs && p->cap_stream) {
    if (!gc.exec || gc.prof != prof) {
      drop_graph(gc);
      hipStream_t saved = p->stream;
      p->stream = p->cap_stream;
      if (prof) {
        p->kst.cap_ev = &gc.ev;
        p->kst.cap_bytes = &gc.bytes;
      }
      hipError_t e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed);
      for (int it = 0; it < n && e == hipSuccess; ++it) e = cg_iteration<T>(p, x, r, pv, q, it);
      hipGraph_t graph = nullptr;
      hipError_t e2 = hipStreamEndCapture(p->cap_stream, &graph);
      p->stream = saved;
      p->kst.cap_ev = nullptr;
      p->kst.cap_bytes = nullptr;
      if (e == hipSuccess && e2 == hipSuccess && graph)
        e = hipGraphInstantiate(&gc.exec, graph, nullptr, nullptr, 0);
      else
        e = (e != hipSuccess) ? e : e2;
      if (graph) (void)hipGraphDestroy(graph);
      if (e != hipSuccess || !gc.exec) {
        (void)hipGetLastError();
        drop_graph(gc);
        p->use_graphs = false;  // fall back to direct launches from now on
      } else {
        gc.prof = prof;
      }
    }
    if (gc.exec) {
      if (gc.prof) {
        p->last_replay = &gc;
        gc.iters = n;
        gc.iter0 = p->h_st->iter;  // the state copied after the previous stage
      }
      return hipGraphLaunch(gc.exec, p->stream);
    }
  }
  hipError_t e = hipSuccess;
  for (int it = 0; it < n && e == hipSuccess; ++it) e = cg_iteration<T>(p, x, r, pv, q, it);
  return e;
}

// Adds the kernel times the last profiled graph replay recorded (the replay
// has completed: its stage event fired, and the state copied after it is in
// h_st).  Only the iterations that ran count: once CG has stopped inside a
// chunk, the launches of its remaining iterations meet the stop flag and
// return at once, without work.  The launches of one iteration are
// recorded in order, the same number for every iteration.
fe_status harvest_graph_events(fe_problem* p) {
  GraphChunk* gc = p->last_replay;
  p->last_replay = nullptr;
  if (!gc || !gc->exec || !gc->prof || gc->iters < 1) return FE_OK;
  const size_t per_iter = gc->bytes.size() / (size_t)gc->iters;
  const int ran = std::min(gc->iters, std::max(1, p->h_st->iter - gc->iter0));
  for (size_t i = 0; i < per_iter * (size_t)ran; ++i) {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, gc->ev[2 * i], gc->ev[2 * i + 1]));
    p->kst.total_ms += ms;
    p->kst.total_bytes += gc->bytes[i];
    p->kst.launches += 1;
  }
  return FE_OK;
}

// The first V-cycle of a folded multigrid CG (its start, or the restart of a
// refinement step): z = M r, leaving the r^T z partials that the chunk's
// first direction kernel sums.  r and z follow the solve's form: a float64
// solve runs it on the float32 copy of r (all levels float32) or on r
// itself, a refinement's float32 CG on its scaled residual.  guard: the
// state whose stop flag the launches honour.
hipError_t launch_start_vcycle(fe_problem* p, CgState* guard) {
  if (p->cfg.precision == FE_PREC_FP64) {
    if (p->f32_from == 0)
      return launch_vcycle<float>(p, 0, static_cast<float*>(p->L[0].mg_r), static_cast<float*>(p->L[0].mg_w),
                                  guard, RZ_PARTIALS, 0);
    return launch_vcycle<double>(p, 0, p->r64, static_cast<double*>(p->L[0].mg_z), guard, RZ_PARTIALS, 0);
  }
  return launch_vcycle<float>(p, 0, p->r32, static_cast<float*>(p->L[0].mg_z), guard, RZ_PARTIALS, 0);
}

// The first V-cycle now; for a batch slot, armed instead (its second state
// is the guard, cleared) for the V-cycle that the batch runs for all its
// starting slots at once before the next replay.
hipError_t start_vcycle(fe_problem* p) {
  if (p->in_batch) {
    p->start_pending = true;
    return launch_cg_guard(p, p->st + 1, 0);
  }
  return launch_start_vcycle(p, p->st);
}

// r = b - Kx (Kx null: x = 0) and the first preconditioned direction.
template <typename T>
hipError_t enqueue_start(fe_problem* p, const T* b, const T* Kx, T* r, T* pv) {
  const bool mg = p->nlev > 1;
  hipError_t e = launch_cg_init<T>(p, b, Kx, r, pv, p->st, mg ? 1 : 0);
  if (e != hipSuccess || !mg) return e;
  T* z = static_cast<T*>(p->L[0].mg_z);
  // folded: the first direction kernel forms p = z from the r^T z partials
  if (folded_mg(p) && std::is_same<T, double>::value && p->f32_from == 0) {
    float* r32 = static_cast<float*>(p->L[0].mg_r);
    if ((e = launch_narrow(p, reinterpret_cast<const double*>(r), r32)) != hipSuccess) return e;
    return start_vcycle(p);  // on r32, into the float32 z (mg_w)
  }
  if (folded_mg(p)) return start_vcycle(p);  // on r, into z
  if ((e = launch_fill<T>(p, pv, p->L[0].g.ndof, T(0))) != hipSuccess) return e;
  if ((e = launch_vcycle<T>(p, 0, r, z, p->st, RZ_FINISH)) != hipSuccess) return e;
  return launch_cg_direction<T>(p, r, z, pv, p->st);
}

fe_status copy_state(fe_problem* p) {
  // a batch slot's state reaches the host in the batch's one strided copy
  // after each replay (fe_batch_round_begin)
  if (p->in_batch) return FE_OK;
  HIP_TRY(hipMemcpyAsync(p->h_st, p->st, sizeof(CgState), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipEventRecord(p->done_ev, p->stream));
  return FE_OK;
}

fe_status copy_scal(fe_problem* p, int slot, int dst) {
  HIP_TRY(hipMemcpyAsync(p->h_scal + dst, p->scal + 2 * slot, sizeof(double), hipMemcpyDeviceToHost,
                         p->stream));
  return FE_OK;
}

// Final float64 residual and compliance of the returned u.
fe_status enqueue_finish(fe_problem* p, bool need_residual) {
  SolveCtx& sc = p->sc;
  if (need_residual) {
    HIP_TRY(launch_residual64(p, sc.u, p->tmp64, p->scal + 2 * SLOT_RR));
    fe_status s = copy_scal(p, SLOT_RR, 0);
    if (s != FE_OK) return s;
  }
  HIP_TRY(launch_dot64(p, p->f, sc.u, p->L[0].g.ndof, p->scal + 2 * SLOT_C));
  fe_status s = copy_scal(p, SLOT_C, 1);
  if (s != FE_OK) return s;
  HIP_TRY(hipEventRecord(p->done_ev, p->stream));
  sc.stage = ST_FINISH;
  return FE_OK;
}

fe_status enqueue_ir_residual(fe_problem* p) {
  HIP_TRY(launch_residual64(p, p->sc.u, p->r64, p->scal + 2 * SLOT_RR));
  fe_status s = copy_scal(p, SLOT_RR, 0);
  if (s != FE_OK) return s;
  HIP_TRY(hipEventRecord(p->done_ev, p->stream));
  p->sc.stage = ST_IR_RESID;
  return FE_OK;
}

// Advances the solve by one stage; the previous stage's event has completed.
fe_status advance(fe_problem* p) {
  SolveCtx& sc = p->sc;
  fe_status hs0 = harvest_graph_events(p);
  if (hs0 != FE_OK) return hs0;
  switch (sc.stage) {
    case ST_CG64: {
      const CgState hs = *p->h_st;
      if (!hs.done) {
        if (p->in_batch) return FE_OK;  // the batch's next replay runs the chunk
        int reps = 1;
        const int v = plan_chunk(p, hs, &reps);
        for (int k = 0; k < reps; ++k) HIP_TRY(enqueue_chunk<double>(p, p->x64, p->r64, p->p64, p->q64, v));
        return copy_state(p);
      }
      sc.info.iters = hs.iter;
      sc.result = (fe_status)hs.status;
      // an odd count: the last iteration deferred its x update
      if (folded_mg(p) && (hs.iter & 1)) HIP_TRY(launch_cg_flush_x<double>(p, p->x64, p->st));
      HIP_TRY(hipMemcpyAsync(sc.u, p->x64, p->L[0].g.ndof * sizeof(double), hipMemcpyDeviceToDevice,
                             p->stream));
      return enqueue_finish(p, true);
    }
    case ST_IR_RESID: {
      const double rr = p->h_scal[0];
      const double rel = std::sqrt(rr / p->ff);
      sc.info.iters = sc.total;
      sc.info.outer_iters = sc.outer;
      if (!std::isfinite(rel)) {
        sc.result = FE_EBREAKDOWN;
        return enqueue_finish(p, false);
      }
      if (rel <= sc.rtol) {
        sc.result = FE_OK;
        return enqueue_finish(p, false);
      }
      if (sc.outer >= kMaxOuter || sc.total >= sc.max_iters || rel > 0.99 * sc.prev_rel) {
        sc.result = FE_ENOTCONV;
        return enqueue_finish(p, false);
      }
      sc.prev_rel = rel;
      if (sc.can_resume) {
        // Residual replacement: the float32 CG goes on from its last
        // direction with the float64 residual of the refined u in place of
        // its recurrence (the Krylov space is kept; a restart would throw it
        // away).  The system stays scaled by the norm it started with.
        const CgState hs = *p->h_st;
        const double scaled = std::sqrt(rr / sc.inner_rr);  // ||r|| in the inner system's units
        double tol = FE_IR_FACTOR * sc.rtol * std::sqrt(p->ff / sc.inner_rr);
        if (tol < FE_IR_PHASE * scaled) tol = FE_IR_PHASE * scaled;
        HIP_TRY(launch_to32_scaled(p, p->r64, p->r32, p->scal + 2 * SLOT_IRS));
        HIP_TRY(launch_fill<float>(p, p->x32, p->L[0].g.ndof, 0.0f));
        // the chunk's first direction kernel reads the last direction from p32
        const int j = hs.iter - sc.chunk_iter0 - 1;  // chunk position of the last iteration
        if (j >= 0 && (j & 1) == 0)
          HIP_TRY(hipMemcpyAsync(p->p32, p->p32b, p->L[0].g.ndof * sizeof(float), hipMemcpyDeviceToDevice,
                                 p->stream));
        HIP_TRY(launch_cg_state_resume(p, p->st, tol * tol, hs.iter + (sc.max_iters - sc.total)));
        HIP_TRY(start_vcycle(p));
        sc.inner_base = sc.total - hs.iter;
        sc.chunk_iter0 = hs.iter;
        sc.mark_rr = scaled * scaled;  // the replaced residual, in the inner system's units
        sc.mark_iter = hs.iter;
        sc.can_resume = false;
        sc.stage = ST_IR_CG;
        return copy_state(p);
      }
      // inner tolerance: aim a little past the target, within float32 reach;
      // a float32 CG that will go on by residual replacement stops after a
      // reduction of FE_IR_PHASE, while its recurrence still tracks the
      // float64 residual to a small fraction
      // With the bf16 contraction the inner operator itself is off by about
      // a tenth of the residual it works on (8-bit operands, rounded after
      // the brick's rigid motion is removed: a nonlinear perturbation of K),
      // so a refinement step cannot cut the float64 residual by much more
      // than 10: its inner solve stops there too
      double itol = FE_IR_FACTOR * sc.rtol / rel;
      const double floor = p->cfg.precision == FE_PREC_BF16_IR          ? FE_IR_FLOOR_BF16
                           : (kResumeInner && folded_mg(p)) ? FE_IR_PHASE
                                                            : FE_IR_FLOOR;
      if (itol < floor) itol = floor;
      if (itol > 1e-1) itol = 1e-1;
      HIP_TRY(hipMemcpyAsync(p->scal + 2 * SLOT_IRS, p->scal + 2 * SLOT_RR, sizeof(double),
                             hipMemcpyDeviceToDevice, p->stream));
      sc.inner_rr = rr;
      HIP_TRY(launch_to32_scaled(p, p->r64, p->r32, p->scal + 2 * SLOT_IRS));
      HIP_TRY(launch_fill<float>(p, p->x32, p->L[0].g.ndof, 0.0f));
      HIP_TRY(launch_cg_state_init(p, p->st, itol, sc.max_iters - sc.total));
      HIP_TRY(enqueue_start<float>(p, p->r32, nullptr, p->r32, p->p32));
      sc.inner_base = sc.total;
      sc.chunk_iter0 = 0;
      sc.mark_iter = -1;
      sc.stage = ST_IR_CG;
      return copy_state(p);
    }
    case ST_IR_CG: {
      const CgState hs = *p->h_st;
      if (!hs.done) {
        sc.chunk_iter0 = hs.iter;  // the next chunk starts at this iteration
        if (p->in_batch) return FE_OK;  // the batch's next replay runs the chunk
        int reps = 1;
        const int v = plan_chunk(p, hs, &reps);
        for (int k = 0; k < reps; ++k) HIP_TRY(enqueue_chunk<float>(p, p->x32, p->r32, p->p32, p->q32, v));
        return copy_state(p);
      }
      sc.total = sc.inner_base + hs.iter;
      sc.outer += 1;
      sc.info.iters = sc.total;
      sc.info.outer_iters = sc.outer;
      // an odd count since the chunks' parity origin: the last iteration
      // deferred its x update
      if (folded_mg(p) && ((hs.iter - sc.chunk_iter0) & 1)) HIP_TRY(launch_cg_flush_x<float>(p, p->x32, p->st));
      if (hs.iter > 0) HIP_TRY(launch_axpy_from32(p, sc.u, p->x32, p->scal + 2 * SLOT_IRS));
      if (hs.status == FE_EBREAKDOWN && hs.iter == 0) {
        sc.result = FE_EBREAKDOWN;
        return enqueue_finish(p, false);
      }
      // the next refinement step may go on with this Krylov space: a folded
      // multigrid CG that stopped at its tolerance after some iterations
      sc.can_resume = kResumeInner && folded_mg(p) && hs.status == FE_OK && hs.iter > 0 &&
                      hs.iter - sc.chunk_iter0 >= 1;
      return enqueue_ir_residual(p);
    }
    case ST_FINISH: {
      sc.info.rel_res = std::sqrt(p->h_scal[0] / p->ff);
      sc.info.compliance = p->h_scal[1];
      sc.stage = ST_DONE;
      return FE_OK;
    }
    default:
      return FE_OK;
  }
}

fe_status solve_begin(fe_problem* p, const double* rho, double* u, double rtol, int max_iters) {
  if (!rho || !u) {
    fe_set_error("rho and u must not be NULL");
    return FE_EINVAL;
  }
  if (!(rtol > 0.0) || max_iters < 1) {
    fe_set_error("rtol must be > 0 and max_iters >= 1");
    return FE_EINVAL;
  }
  if (p->sc.stage != ST_DONE) {
    fe_set_error("a solve is still in progress on this problem");
    return FE_EINVAL;
  }
  SolveCtx& sc = p->sc;
  sc = SolveCtx();
  sc.rtol = rtol;
  sc.max_iters = max_iters;
  sc.u = u;
  fe_status s = prepare_operator(p, rho);
  if (s != FE_OK) return s;
  HIP_TRY(launch_mask_vec<double>(p, 0, u));
  if (!(p->ff > 0.0)) {  // no load: u = 0 is exact
    HIP_TRY(launch_fill<double>(p, u, p->L[0].g.ndof, 0.0));
    HIP_TRY(hipEventRecord(p->done_ev, p->stream));
    sc.stage = ST_DONE;
    return FE_OK;
  }
  if (p->cfg.precision == FE_PREC_FP64) {
    const int64_t nd = p->L[0].g.ndof;
    HIP_TRY(hipMemcpyAsync(p->x64, u, nd * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(launch_kxu<double>(p, 0, p->x64, p->q64, nullptr));
    HIP_TRY(launch_cg_state_init(p, p->st, rtol, max_iters));
    HIP_TRY(enqueue_start<double>(p, p->f, p->q64, p->r64, p->p64));
    sc.stage = ST_CG64;
    return copy_state(p);
  }
  return enqueue_ir_residual(p);
}

fe_status solve_step(fe_problem* p, int wait, int* done) {
  *done = 0;
  while (p->sc.stage != ST_DONE) {
    if (wait) {
      HIP_TRY(hipEventSynchronize(p->done_ev));
    } else {
      const hipError_t q = hipEventQuery(p->done_ev);
      if (q == hipErrorNotReady) return FE_OK;
      if (q != hipSuccess) {
        fe_set_error(std::string("hipEventQuery: ") + hipGetErrorString(q));
        return FE_EDEVICE;
      }
    }
    fe_status s = advance(p);
    if (s != FE_OK) {
      p->sc.stage = ST_DONE;
      return s;
    }
    if (!wait) break;  // one stage per call when polling
  }
  *done = p->sc.stage == ST_DONE;
  return FE_OK;
}

fe_status solve_end(fe_problem* p, fe_solve_info* info) {
  SolveCtx& sc = p->sc;
  if (sc.stage != ST_DONE) {
    fe_set_error("the solve has not finished");
    return FE_EINVAL;
  }
  if (info) *info = sc.info;
  if (sc.result == FE_ENOTCONV)
    fe_set_error("iteration limit reached (relative residual " + std::to_string(sc.info.rel_res) + ")");
  if (sc.result == FE_EBREAKDOWN) fe_set_error("CG breakdown (p^T K p <= 0 or non-finite value)");
  return sc.result;
}

struct KeTables {
  double ke[576];
  WalshK wk;
  double lam_max;
};

// Ke by Gauss quadrature, its sum/difference-basis constants (checked against
// the full transformed matrix) and lambda_max(Ke) / Ke_dd by power iteration
// (Ke is symmetric positive semi-definite); that ratio bounds
// lambda_max(D^-1 K) for any modulus field.
bool make_ke_tables(double nu, KeTables* t) {
  host_hex8_ke(nu, 1.0, 1.0, t->ke);
  double dev = 0.0;
  host_walsh_constants(t->ke, &t->wk, &dev);
  if (dev > 1e-12) return false;
  double v[24], w[24], lam = 0.0;
  for (int i = 0; i < 24; ++i) v[i] = 1.0 + 0.01 * i * ((i & 1) ? -1.0 : 1.0);
  for (int it = 0; it < 5000; ++it) {
    double nrm = 0.0;
    for (int i = 0; i < 24; ++i) {
      double s2 = 0.0;
      for (int j = 0; j < 24; ++j) s2 += t->ke[i * 24 + j] * v[j];
      w[i] = s2;
      nrm += s2 * s2;
    }
    nrm = std::sqrt(nrm);
    double num = 0.0, den = 0.0;
    for (int i = 0; i < 24; ++i) {
      num += v[i] * w[i];
      den += v[i] * v[i];
    }
    lam = num / den;
    for (int i = 0; i < 24; ++i) v[i] = w[i] / nrm;
  }
  t->lam_max = lam / t->ke[0];
  return true;
}

}  // namespace

// ======================================================================= ABI
extern "C" size_t fe_workspace_size(const fe_config* cfg) {
  if (!validate(cfg).empty()) return 0;
  return layout(cfg, nullptr, nullptr);
}

extern "C" fe_status fe_setup(const fe_config* cfg, const uint8_t* fixed, const double* f, void* ws,
                              size_t ws_bytes, void* stream, fe_problem** out) {
  if (!out) {
    fe_set_error("out is NULL");
    return FE_EINVAL;
  }
  *out = nullptr;
  const std::string why = validate(cfg);
  if (!why.empty()) {
    fe_set_error(why);
    return FE_EINVAL;
  }
  if (!f || !ws) {
    fe_set_error("f and ws must not be NULL");
    return FE_EINVAL;
  }
  if (((uintptr_t)ws) % kAlign) {
    fe_set_error("workspace must be 256-byte aligned");
    return FE_EINVAL;
  }
  const size_t need = layout(cfg, nullptr, nullptr);
  if (ws_bytes < need) {
    fe_set_error("workspace too small: need " + std::to_string(need) + " bytes");
    return FE_ENOMEM;
  }
  fe_problem* p = new (std::nothrow) fe_problem();
  if (!p) {
    fe_set_error("out of host memory");
    return FE_ENOMEM;
  }
  p->cfg = *cfg;
  p->mfma_l0 = cfg->precision == FE_PREC_BF16_IR ? 1 : cfg->precision == FE_PREC_BF16X3_IR ? 2 : 0;
  p->stream = (hipStream_t)stream;
  p->ws = (char*)ws;
  p->ws_bytes = ws_bytes;
  layout(cfg, p, (char*)ws);

  // Ke, its sum/difference-basis constants and lambda_max(diag(Ke)^-1 Ke)
  // (unit modulus, unit edge) depend on nu only: computed once per nu.
  {
    static std::mutex mu;
    static std::vector<std::pair<double, KeTables>> cache;
    std::lock_guard<std::mutex> lock(mu);
    const KeTables* hit = nullptr;
    for (auto& kv : cache)
      if (kv.first == cfg->nu) hit = &kv.second;
    if (!hit) {
      KeTables t;
      if (!make_ke_tables(cfg->nu, &t)) {
        delete p;
        fe_set_error("element stiffness lacks the cube symmetry the kernels rely on");
        return FE_EINVAL;
      }
      cache.emplace_back(cfg->nu, t);
      hit = &cache.back().second;
    }
    std::memcpy(p->ke64_host, hit->ke, sizeof(p->ke64_host));
    p->wk = hit->wk;
    p->lam_max = hit->lam_max;
  }
  p->ke_diag = p->ke64_host[0];
  float ke32h[576];
  for (int i = 0; i < 576; ++i) ke32h[i] = (float)p->ke64_host[i];

  // filter stencil: offsets d with positive cone weight r - |d| (z slowest),
  // as offsets into the LDS tile of the filter kernel (8 x 8 x tz elements
  // plus a halo of the stencil's reach H; tz = 2 when the halo is 7, so that
  // the tile stays within 64 KB)
  const double r = cfg->filter_r;
  const int R = (int)std::ceil(r);
  std::vector<int> soff;
  std::vector<double> w;
  int H = 0;
  for (int dk = -R; dk <= R; ++dk)
    for (int dj = -R; dj <= R; ++dj)
      for (int di = -R; di <= R; ++di) {
        const double wt = r - std::sqrt((double)(di * di + dj * dj + dk * dk));
        if (wt > 0.0) {
          soff.insert(soff.end(), {di, dj, dk});
          w.push_back(wt);
          H = std::max(H, std::max(std::abs(di), std::max(std::abs(dj), std::abs(dk))));
        }
      }
  const int n = (int)w.size();
  const int tz = H <= 6 ? 4 : 2;
  const int LX = 8 + 2 * H;
  std::vector<int> lin(n);
  for (int q = 0; q < n; ++q) lin[q] = (soff[3 * q + 2] * LX + soff[3 * q + 1]) * LX + soff[3 * q];
  p->nstencil = n;
  p->st_halo = H;
  p->st_tz = tz;

  auto fail = [&](hipError_t e, const char* what) {
    fe_set_error(std::string(what) + ": " + hipGetErrorString(e));
    fe_destroy(p);
    return FE_EDEVICE;
  };
  hipError_t e;
  if ((e = hipMemcpyAsync(p->ke64, p->ke64_host, sizeof(p->ke64_host), hipMemcpyHostToDevice, p->stream)))
    return fail(e, "copy Ke");
  if ((e = hipMemcpyAsync(p->ke32, ke32h, sizeof(ke32h), hipMemcpyHostToDevice, p->stream)))
    return fail(e, "copy Ke32");
  if ((e = hipMemcpyAsync(p->st_lin, lin.data(), n * sizeof(int), hipMemcpyHostToDevice, p->stream)))
    return fail(e, "copy stencil");
  if ((e = hipMemcpyAsync(p->st_w, w.data(), n * sizeof(double), hipMemcpyHostToDevice, p->stream)))
    return fail(e, "copy stencil weights");
  if ((e = launch_fill<double>(p, p->scal, NSCAL, 0.0))) return fail(e, "clear scalars");
  if ((e = launch_fill<double>(p, p->zpad, 8, 0.0))) return fail(e, "clear zero pad");
  if ((e = launch_fill<double>(p, (double*)p->st, 2 * sizeof(CgState) / sizeof(double), 0.0)))
    return fail(e, "clear state");
  if ((e = launch_fill<double>(p, p->oc, 64, 0.0))) return fail(e, "clear oc state");
  if ((e = launch_node_mask(p, fixed))) return fail(e, "node mask");
  for (int l = 1; l < p->nlev; ++l)
    if ((e = launch_coarsen_mask(p, l))) return fail(e, "coarse mask");
  if ((e = launch_mask_load(p, f))) return fail(e, "load");
  if ((e = launch_filter_rowsums(p))) return fail(e, "filter row sums");
  if ((e = launch_dot64(p, p->f, p->f, p->L[0].g.ndof, p->scal + 2 * SLOT_FF))) return fail(e, "||f||");
  if ((e = hipHostMalloc((void**)&p->h_st, sizeof(CgState), hipHostMallocDefault))) return fail(e, "pinned state");
  if ((e = hipHostMalloc((void**)&p->h_scal, 4 * sizeof(double), hipHostMallocDefault)))
    return fail(e, "pinned scalars");
  if ((e = hipEventCreateWithFlags(&p->done_ev, hipEventDisableTiming))) return fail(e, "event");
  if ((e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking))) return fail(e, "capture stream");
  if ((e = hipMemcpyAsync(p->h_scal, p->scal + 2 * SLOT_FF, sizeof(double), hipMemcpyDeviceToHost, p->stream)))
    return fail(e, "read ||f||");
  // host copies above read stack arrays: finish them before returning
  if ((e = hipStreamSynchronize(p->stream))) return fail(e, "setup sync");
  p->ff = p->h_scal[0];
  *out = p;
  return FE_OK;
}

extern "C" fe_status fe_apply_K(fe_problem* p, const double* rho, const double* u, double* y,
                                int32_t variant) {
  CHECK_HANDLE(p);
  if (!rho || !u || !y) {
    fe_set_error("rho, u and y must not be NULL");
    return FE_EINVAL;
  }
  const int64_t ndof = p->L[0].g.ndof;
  fe_status s = prepare_operator(p, rho);
  if (s != FE_OK) return s;
  if (variant == 0) {
    HIP_TRY(hipMemcpyAsync(p->tmp64, u, ndof * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(launch_mask_vec<double>(p, 0, p->tmp64));
    HIP_TRY(launch_kxu<double>(p, 0, p->tmp64, y, nullptr));
    return FE_OK;
  }
  if (variant == 1 || variant == 2 || variant == 4) {
    if (p->cfg.precision == FE_PREC_FP64) {
      fe_set_error("float32 and bf16 variants need a problem set up with a reduced precision");
      return FE_EINVAL;
    }
    const int saved = p->mfma_l0;
    p->mfma_l0 = variant == 2 ? 1 : variant == 4 ? 2 : 0;
    HIP_TRY(launch_convert_64_32(p, u, p->x32, ndof));
    HIP_TRY(launch_mask_vec<float>(p, 0, p->x32));
    hipError_t e = launch_kxu<float>(p, 0, p->x32, p->q32, nullptr);
    p->mfma_l0 = saved;
    HIP_TRY(e);
    HIP_TRY(launch_convert_32_64(p, p->q32, y, ndof));
    return FE_OK;
  }
  if (variant == 3) {  // dense-Ke node-centric reference kernel, float64
    HIP_TRY(hipMemcpyAsync(p->tmp64, u, ndof * sizeof(double), hipMemcpyDeviceToDevice, p->stream));
    HIP_TRY(launch_mask_vec<double>(p, 0, p->tmp64));
    HIP_TRY(launch_kxu_dense64(p, p->tmp64, y));
    return FE_OK;
  }
  fe_set_error("unknown K*u variant");
  return FE_EINVAL;
}

extern "C" fe_status fe_solve(fe_problem* p, const double* rho, double* u, double rtol, int32_t max_iters,
                              fe_solve_info* info) {
  CHECK_HANDLE(p);
  if (p->in_batch) {
    fe_set_error("a batch slot solves through fe_solve_begin and the batch's rounds");
    return FE_EINVAL;
  }
  if (info) std::memset(info, 0, sizeof(*info));
  fe_status s = solve_begin(p, rho, u, rtol, max_iters);
  if (s != FE_OK) return s;
  int done = 0;
  s = solve_step(p, 1, &done);
  if (s != FE_OK) return s;
  return solve_end(p, info);
}

extern "C" fe_status fe_solve_begin(fe_problem* p, const double* rho, double* u, double rtol,
                                    int32_t max_iters) {
  CHECK_HANDLE(p);
  return solve_begin(p, rho, u, rtol, max_iters);
}

extern "C" fe_status fe_solve_step(fe_problem* p, int32_t* done) {
  CHECK_HANDLE(p);
  if (!done) {
    fe_set_error("done must not be NULL");
    return FE_EINVAL;
  }
  if (p->in_batch) {  // the batch's rounds advance it
    *done = p->sc.stage == ST_DONE;
    return FE_OK;
  }
  int d = 0;
  fe_status s = solve_step(p, 0, &d);
  *done = d;
  return s;
}

extern "C" fe_status fe_solve_end(fe_problem* p, fe_solve_info* info) {
  CHECK_HANDLE(p);
  return solve_end(p, info);
}

extern "C" fe_status fe_sensitivity(fe_problem* p, const double* rho, const double* u, double* dc,
                                    double* compliance) {
  CHECK_HANDLE(p);
  if (!rho || !u || !dc) {
    fe_set_error("rho, u and dc must not be NULL");
    return FE_EINVAL;
  }
  HIP_TRY(launch_sensitivity(p, rho, u, dc));
  if (compliance) {
    // the reduction counter lives next to the value in scal[]
    HIP_TRY(launch_dot64(p, p->f, u, p->L[0].g.ndof, p->scal + 2 * SLOT_TMP));
    HIP_TRY(hipMemcpyAsync(compliance, p->scal + 2 * SLOT_TMP, sizeof(double), hipMemcpyDeviceToDevice,
                           p->stream));
  }
  return FE_OK;
}

extern "C" fe_status fe_sensitivity_adjoint(fe_problem* p, const double* rho, const double* u, const double* lam,
                                            double* g) {
  CHECK_HANDLE(p);
  if (!rho || !u || !lam || !g) {
    fe_set_error("rho, u, lam and g must not be NULL");
    return FE_EINVAL;
  }
  HIP_TRY(launch_adjoint_sensitivity(p, rho, u, lam, g));
  return FE_OK;
}

extern "C" fe_status fe_set_load(fe_problem* p, const double* f) {
  CHECK_HANDLE(p);
  if (!f) {
    fe_set_error("f must not be NULL");
    return FE_EINVAL;
  }
  if (p->in_batch) {
    fe_set_error("a batch slot takes its load from fe_batch_setup_slot");
    return FE_EINVAL;
  }
  if (p->sc.stage != ST_DONE) {
    fe_set_error("a solve is still in progress on this problem");
    return FE_EINVAL;
  }
  HIP_TRY(launch_mask_load(p, f));
  HIP_TRY(launch_dot64(p, p->f, p->f, p->L[0].g.ndof, p->scal + 2 * SLOT_FF));
  HIP_TRY(hipMemcpyAsync(p->h_scal, p->scal + 2 * SLOT_FF, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->ff = p->h_scal[0];
  return FE_OK;
}

extern "C" fe_status fe_filter(fe_problem* p, const double* in, double* out, int32_t transpose) {
  CHECK_HANDLE(p);
  if (!in || !out || in == out) {
    fe_set_error("in and out must be distinct non-NULL arrays");
    return FE_EINVAL;
  }
  HIP_TRY(launch_filter(p, in, out, transpose ? 1 : 0));
  return FE_OK;
}

namespace {

void drop_oc_graph(OcGraph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g.exec = nullptr;
}

// The OC update is some fifty short launches, most of which return at once
// once the multiplier search has converged; replayed as one graph they cost
// the host a single launch.  The graph bakes in the arrays and parameters, so
// a call with others launches directly and the next call with those captures.
hipError_t enqueue_oc(fe_problem* p, const double* x, const double* dcx, const double* dv, double volfrac,
                      double move, double* x_new, double* change) {
  OcGraph& g = p->ocg;
  const void* key[5] = {x, dcx, dv, x_new, change};
  const bool same = g.seen && std::equal(key, key + 5, g.key) && g.volfrac == volfrac && g.move == move;
  if (!p->use_graphs || !p->cap_stream || !same) {
    drop_oc_graph(g);
    std::copy(key, key + 5, g.key);
    g.volfrac = volfrac;
    g.move = move;
    g.seen = true;
    return launch_oc(p, x, dcx, dv, volfrac, move, x_new, change);
  }
  if (!g.exec) {
    hipStream_t saved = p->stream;
    p->stream = p->cap_stream;
    hipError_t e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed);
    hipGraph_t graph = nullptr;
    if (e == hipSuccess) {
      e = launch_oc(p, x, dcx, dv, volfrac, move, x_new, change);
      const hipError_t e2 = hipStreamEndCapture(p->cap_stream, &graph);
      if (e == hipSuccess) e = e2;
    }
    p->stream = saved;
    if (e == hipSuccess && graph) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess || !g.exec) {
      (void)hipGetLastError();
      drop_oc_graph(g);
      p->use_graphs = false;  // direct launches from now on
      return launch_oc(p, x, dcx, dv, volfrac, move, x_new, change);
    }
  }
  return hipGraphLaunch(g.exec, p->stream);
}

}  // namespace

extern "C" fe_status oc_update(fe_problem* p, const double* x, const double* dcx, const double* dv,
                               double volfrac, double move, double* x_new, double* change) {
  CHECK_HANDLE(p);
  if (!x || !dcx || !dv || !x_new) {
    fe_set_error("x, dcx, dv and x_new must not be NULL");
    return FE_EINVAL;
  }
  if (!(volfrac > 0.0 && volfrac <= 1.0) || !(move > 0.0)) {
    fe_set_error("volfrac must lie in (0, 1] and move must be > 0");
    return FE_EINVAL;
  }
  HIP_TRY(enqueue_oc(p, x, dcx, dv, volfrac, move, x_new, change));
  return FE_OK;
}

extern "C" fe_status oc_update_noalloc(int64_t nelem, const double* x, const double* dcx, const double* dv,
                                       double volfrac, double move, double* x_new, double* change, void* stream) {
  if (!x || !dcx || !dv || !x_new) {
    fe_set_error("x, dcx, dv and x_new must not be NULL");
    return FE_EINVAL;
  }
  if (nelem < 1 || nelem > FE_NOALLOC_MAX_ELEMS) {
    fe_set_error("nelem must lie in [1, " + std::to_string((long long)FE_NOALLOC_MAX_ELEMS) + "]");
    return FE_EINVAL;
  }
  if (!(volfrac > 0.0 && volfrac <= 1.0) || !(move > 0.0)) {
    fe_set_error("volfrac must lie in (0, 1] and move must be > 0");
    return FE_EINVAL;
  }
  HIP_TRY(launch_oc_noalloc(static_cast<hipStream_t>(stream), nelem, x, dcx, dv, volfrac, move, x_new, change));
  return FE_OK;
}

extern "C" fe_status fe_block_mean(fe_problem* p, const double* z, int32_t nb, double* zc) {
  CHECK_HANDLE(p);
  if (!z || !zc || z == zc) {
    fe_set_error("z and zc must be distinct non-NULL arrays");
    return FE_EINVAL;
  }
  const Grid& g = p->L[0].g;
  if (nb < 1 || g.nx % nb || g.ny % nb || g.nz % nb) {
    fe_set_error("nb must be >= 1 and divide nx, ny and nz");
    return FE_EINVAL;
  }
  HIP_TRY(launch_block_mean(p, z, nb, zc));
  return FE_OK;
}

extern "C" fe_status fe_extrapolate(fe_problem* p, double* u, double* u_hist, double theta) {
  CHECK_HANDLE(p);
  if (!u || !u_hist || u == u_hist) {
    fe_set_error("u and u_hist must be distinct non-NULL arrays");
    return FE_EINVAL;
  }
  if (!(theta >= 0.0 && theta <= 4.0)) {
    fe_set_error("theta must be in [0, 4]");
    return FE_EINVAL;
  }
  HIP_TRY(launch_extrapolate(p, u, u_hist, theta));
  return FE_OK;
}

extern "C" fe_status fe_set_mg_params(fe_problem* p, int32_t nu, int32_t coarse_sweeps, double omega,
                                      double coarse_ratio) {
  CHECK_HANDLE(p);
  if (p->in_batch) {
    fe_set_error("batch slots share the batch's multigrid parameters (the library defaults)");
    return FE_EINVAL;
  }
  if (nu < 1 || nu > 8 || coarse_sweeps < 1 || coarse_sweeps > 10000 || !(omega > 0.0 && omega < 1.0) ||
      !(coarse_ratio >= 2.0 && coarse_ratio <= 1e12)) {
    fe_set_error("need 1 <= nu <= 8, 1 <= coarse_sweeps <= 10000, 0 < omega < 1, 2 <= coarse_ratio <= 1e12");
    return FE_EINVAL;
  }
  if (omega * p->lam_max >= 2.0) {
    fe_set_error("omega must stay below 2 / lambda_max(diag(Ke)^-1 Ke) = " + std::to_string(2.0 / p->lam_max) +
                 " for the smoother to be convergent");
    return FE_EINVAL;
  }
  p->mg_nu = nu;
  p->mg_coarse_sweeps = coarse_sweeps;
  p->mg_omega = omega;
  p->cheb_ratio = coarse_ratio;
  drop_chunks(p);  // the captured chunks bake these in
  return FE_OK;
}

extern "C" fe_status fe_set_mg_smoother(fe_problem* p, int32_t cheb_from_level, int32_t degree, double ratio) {
  CHECK_HANDLE(p);
  if (p->in_batch) {
    fe_set_error("batch slots share the batch's multigrid parameters (the library defaults)");
    return FE_EINVAL;
  }
  const bool off = cheb_from_level == 0;
  if (!off && (cheb_from_level < 1 || cheb_from_level > p->nlev - 2 || degree < 1 || degree > 64 ||
               !(ratio >= 2.0 && ratio <= 1e6))) {
    fe_set_error("need cheb_from_level = 0 (off) or 1 <= cheb_from_level <= levels - 2 with 1 <= degree <= 64 "
                 "and 2 <= ratio <= 1e6");
    return FE_EINVAL;
  }
  p->cs_from = off ? FE_CS_OFF : cheb_from_level;
  if (!off) {
    p->cs_deg = degree;
    p->cs_ratio = ratio;
  }
  drop_chunks(p);  // the captured chunks bake these in
  return FE_OK;
}

extern "C" fe_status fe_get_mg_smoother(const fe_problem* p, int32_t* cheb_from_level, int32_t* degree,
                                        double* ratio) {
  CHECK_HANDLE(p);
  const bool on = p->cs_from >= 1 && p->cs_from <= p->nlev - 2;
  if (cheb_from_level) *cheb_from_level = on ? p->cs_from : 0;
  if (degree) *degree = p->cs_deg;
  if (ratio) *ratio = p->cs_ratio;
  return FE_OK;
}

extern "C" fe_status fe_set_float32_levels(fe_problem* p, int32_t first_level) {
  CHECK_HANDLE(p);
  if (p->in_batch) {
    fe_set_error("batch slots share the batch's multigrid parameters (the library defaults)");
    return FE_EINVAL;
  }
  if (first_level < 0 || first_level > p->nlev) {
    fe_set_error("first_level must lie in [0, number of levels]");
    return FE_EINVAL;
  }
  p->f32_from = first_level;
  drop_chunks(p);  // the captured chunks bake the path in
  return FE_OK;
}

extern "C" fe_status fe_get_mg_params(const fe_problem* p, int32_t* nu, int32_t* coarse_sweeps, double* omega,
                                      double* coarse_ratio) {
  CHECK_HANDLE(p);
  if (nu) *nu = p->mg_nu;
  if (coarse_sweeps) *coarse_sweeps = p->mg_coarse_sweeps;
  if (omega) *omega = p->mg_omega;
  if (coarse_ratio) *coarse_ratio = p->cheb_ratio;
  return FE_OK;
}

extern "C" fe_status fe_set_coarse_fusion(fe_problem* p, int32_t steps_per_launch) {
  CHECK_HANDLE(p);
  if (p->in_batch) {
    fe_set_error("batch slots share the batch's multigrid parameters (the library defaults)");
    return FE_EINVAL;
  }
  if (steps_per_launch < 0 || steps_per_launch > 5) {
    fe_set_error("the coarse launch form must be 0, 1, 2, 3, 4 or 5");
    return FE_EINVAL;
  }
  p->cheb_per_launch = steps_per_launch;
  drop_chunks(p);
  return FE_OK;
}

extern "C" fe_status fe_set_profiling(fe_problem* p, int32_t on) {
  CHECK_HANDLE(p);
  if (on < 0 || on > 9) {
    fe_set_error("profiling selector must be 0, 1 or 2 + form (form 0..7)");
    return FE_EINVAL;
  }
  p->kst.on = on != 0;
  p->kst.mode = on >= 2 ? on - 2 : -1;
  return FE_OK;
}

extern "C" fe_status fe_set_cache_flush(fe_problem* p, void* buf, size_t bytes) {
  CHECK_HANDLE(p);
  if (buf && (bytes < ((size_t)512 << 20) || ((uintptr_t)buf) % 16)) {
    fe_set_error("the cold-cache buffer must be 16-byte aligned and at least 512 MB");
    return FE_EINVAL;
  }
  p->kst.flush = buf ? static_cast<uint32_t*>(buf) : nullptr;
  p->kst.flush_words = buf ? bytes / sizeof(uint32_t) : 0;
  // captured chunks carry the flush launches only if captured with it
  drop_chunks(p);
  return FE_OK;
}

extern "C" fe_status fe_kernel_stats(fe_problem* p, int32_t reset, int64_t* launches, double* total_ms,
                                     double* bytes_per_launch) {
  CHECK_HANDLE(p);
  KStats& ks = p->kst;
  if (ks.pending) {
    HIP_TRY(hipStreamSynchronize(p->stream));
    for (int64_t i = 0; i < ks.pending; ++i) {
      float ms = 0.0f;
      HIP_TRY(hipEventElapsedTime(&ms, ks.ev[2 * i], ks.ev[2 * i + 1]));
      ks.total_ms += ms;
      ks.total_bytes += ks.bytes[i];
    }
    ks.launches += ks.pending;
    ks.pending = 0;
  }
  if (launches) *launches = ks.launches;
  if (total_ms) *total_ms = ks.total_ms;
  if (bytes_per_launch) *bytes_per_launch = ks.launches ? ks.total_bytes / (double)ks.launches : 0.0;
  if (reset) {
    ks.launches = 0;
    ks.total_ms = 0.0;
    ks.total_bytes = 0.0;
  }
  return FE_OK;
}

extern "C" void fe_destroy(fe_problem* p) {
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  drop_chunks(p);
  drop_oc_graph(p->ocg);
  for (hipEvent_t e : p->kst.ev) (void)hipEventDestroy(e);
  if (p->done_ev) (void)hipEventDestroy(p->done_ev);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->h_st) (void)hipHostFree(p->h_st);
  if (p->h_scal) (void)hipHostFree(p->h_scal);
  delete p;
}

// ------------------------------------------------------------------ batches
// A batch holds nslots problems of one configuration in one workspace, slot
// s at byte s * stride; their CG chunks run as one captured graph whose
// kernels take one problem per grid y index (pointers moved by the stride).
// A slot whose CG is stopped (idle, finished, or in another stage) turns
// every workgroup of its y index into an early exit, so problems join and
// leave between replays.
struct fe_batch {
  fe_config cfg;
  int nslots = 0;
  size_t stride = 0;
  char* ws = nullptr;
  double* zero_f = nullptr;  // zero load of the idle slots
  size_t st_off = 0;         // offset of the CG state inside a slot
  hipStream_t stream = nullptr;
  std::vector<fe_problem*> slot;
  hipGraphExec_t chunk = nullptr;
  hipEvent_t ev = nullptr;
  CgState* h_states = nullptr;  // pinned: every slot's CG state after the round's replay (one copy)
  bool open = false;      // a round was begun and not yet ended
  bool replayed = false;  // the open round replayed the chunk (h_states is filled)
};

namespace {

// New supports and load on a problem of the same configuration (the parts
// of fe_setup that depend on the design, not on the configuration).
fe_status reinit_design(fe_problem* p, const uint8_t* fixed, const double* f) {
  HIP_TRY(launch_fill<double>(p, (double*)p->st, 2 * sizeof(CgState) / sizeof(double), 0.0));
  HIP_TRY(launch_node_mask(p, fixed));
  for (int l = 1; l < p->nlev; ++l) HIP_TRY(launch_coarsen_mask(p, l));
  HIP_TRY(launch_mask_load(p, f));
  HIP_TRY(launch_dot64(p, p->f, p->f, p->L[0].g.ndof, p->scal + 2 * SLOT_FF));
  HIP_TRY(hipMemcpyAsync(p->h_scal, p->scal + 2 * SLOT_FF, sizeof(double), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  p->ff = p->h_scal[0];
  p->sc = SolveCtx();
  return FE_OK;
}

std::string batch_validate(const fe_config* cfg, int nslots) {
  const std::string why = validate(cfg);
  if (!why.empty()) return why;
  if (nslots < 1 || nslots > 1024) return "nslots must lie in [1, 1024]";
  if (cfg->precond != FE_PRECOND_GMG) return "batches need the multigrid preconditioner";
  if (cfg->precision != FE_PREC_FP64 && cfg->precision != FE_PREC_FP32_IR)
    return "batches run FE_PREC_FP64 or FE_PREC_FP32_IR";
  return "";
}

size_t batch_stride(const fe_config* cfg) { return align_up(layout(cfg, nullptr, nullptr)); }

size_t batch_zero_bytes(const fe_config* cfg) {
  return align_up((size_t)3 * (cfg->nx + 1) * (cfg->ny + 1) * (cfg->nz + 1) * sizeof(double));
}

// Stops the CG state at slot s (its workgroups exit at once in a replay),
// and its guard of the shared first V-cycle (the second state).
fe_status batch_stop_slot(fe_batch* b, int s) {
  CgState cs[2];
  std::memset(cs, 0, sizeof(cs));
  cs[0].done = cs[1].done = 1;
  cs[0].status = cs[1].status = FE_OK;
  HIP_TRY(hipMemcpyAsync(b->ws + (size_t)s * b->stride + b->st_off, cs, sizeof(cs), hipMemcpyHostToDevice,
                         b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));  // the source is on this stack
  return FE_OK;
}

template <typename T>
fe_status batch_capture(fe_batch* b) {
  fe_problem* t = b->slot[0];
  T *x, *r, *pv, *q;
  if (std::is_same<T, double>::value) {
    x = reinterpret_cast<T*>(t->x64);
    r = reinterpret_cast<T*>(t->r64);
    pv = reinterpret_cast<T*>(t->p64);
    q = reinterpret_cast<T*>(t->q64);
  } else {
    x = reinterpret_cast<T*>(t->x32);
    r = reinterpret_cast<T*>(t->r32);
    pv = reinterpret_cast<T*>(t->p32);
    q = reinterpret_cast<T*>(t->q32);
  }
  const bool prof = t->kst.on;
  t->kst.on = false;
  t->bcount = b->nslots;
  t->bstride = (int64_t)b->stride;
  hipStream_t saved = t->stream;
  t->stream = t->cap_stream;
  hipError_t e = hipStreamBeginCapture(t->cap_stream, hipStreamCaptureModeRelaxed);
  for (int it = 0; it < kChunkMG && e == hipSuccess; ++it) e = cg_iteration<T>(t, x, r, pv, q, it);
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(t->cap_stream, &graph);
  t->stream = saved;
  t->bcount = 1;
  t->bstride = 0;
  t->kst.on = prof;
  if (e == hipSuccess && e2 == hipSuccess && graph) e = hipGraphInstantiate(&b->chunk, graph, nullptr, nullptr, 0);
  else if (e == hipSuccess) e = e2;
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess || !b->chunk) {
    (void)hipGetLastError();
    b->chunk = nullptr;
    fe_set_error(std::string("batch chunk capture: ") + hipGetErrorString(e));
    return FE_EDEVICE;
  }
  return FE_OK;
}

bool in_cg_stage(const fe_problem* h) { return h && (h->sc.stage == ST_CG64 || h->sc.stage == ST_IR_CG); }

// The slots that (re)started their CG since the last replay share one first
// V-cycle before the next: every slot's launches run, those whose guard is
// set leave at once; then every guard is set again.
fe_status batch_start_vcycles(fe_batch* b) {
  bool starting = false;
  for (int s = 0; s < b->nslots; ++s)
    if (b->slot[s] && b->slot[s]->start_pending) {
      starting = true;
      b->slot[s]->start_pending = false;
    }
  if (!starting) return FE_OK;
  fe_problem* t = b->slot[0];
  const bool prof = t->kst.on;
  t->kst.on = false;
  t->bcount = b->nslots;
  t->bstride = (int64_t)b->stride;
  hipError_t e = launch_start_vcycle(t, t->st + 1);
  if (e == hipSuccess) e = launch_cg_guard(t, t->st + 1, 1);
  t->bcount = 1;
  t->bstride = 0;
  t->kst.on = prof;
  if (e != hipSuccess) {
    fe_set_error(std::string("batched first V-cycle: ") + hipGetErrorString(e));
    return FE_EDEVICE;
  }
  return FE_OK;
}

}  // namespace

extern "C" size_t fe_batch_workspace_size(const fe_config* cfg, int32_t nslots) {
  if (!batch_validate(cfg, nslots).empty()) return 0;
  return (size_t)nslots * batch_stride(cfg) + batch_zero_bytes(cfg);
}

extern "C" fe_status fe_batch_create(const fe_config* cfg, int32_t nslots, void* ws, size_t ws_bytes,
                                     void* stream, fe_batch** out) {
  if (!out) {
    fe_set_error("out is NULL");
    return FE_EINVAL;
  }
  *out = nullptr;
  const std::string why = batch_validate(cfg, nslots);
  if (!why.empty()) {
    fe_set_error(why);
    return FE_EINVAL;
  }
  if (!ws || ((uintptr_t)ws) % kAlign) {
    fe_set_error("ws must be a 256-byte aligned device pointer");
    return FE_EINVAL;
  }
  const size_t need = fe_batch_workspace_size(cfg, nslots);
  if (ws_bytes < need) {
    fe_set_error("batch workspace too small: need " + std::to_string(need) + " bytes");
    return FE_ENOMEM;
  }
  fe_batch* b = new (std::nothrow) fe_batch();
  if (!b) {
    fe_set_error("out of host memory");
    return FE_ENOMEM;
  }
  b->cfg = *cfg;
  b->nslots = nslots;
  b->stride = batch_stride(cfg);
  b->ws = static_cast<char*>(ws);
  b->zero_f = reinterpret_cast<double*>(b->ws + (size_t)nslots * b->stride);
  b->stream = (hipStream_t)stream;
  b->slot.assign(nslots, nullptr);
  auto fail = [&](fe_status st) {
    fe_batch_destroy(b);
    return st;
  };
  hipError_t e = hipMemsetAsync(b->zero_f, 0, batch_zero_bytes(cfg), b->stream);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_states, (size_t)nslots * sizeof(CgState), hipHostMallocDefault);
  if (e != hipSuccess) {
    fe_set_error(std::string("batch setup: ") + hipGetErrorString(e));
    return fail(FE_EDEVICE);
  }
  for (int s = 0; s < nslots; ++s) {
    fe_problem* h = nullptr;
    const fe_status st = fe_setup(cfg, nullptr, b->zero_f, b->ws + (size_t)s * b->stride, b->stride, stream, &h);
    if (st != FE_OK) return fail(st);
    h->in_batch = true;
    b->slot[s] = h;
    if (s == 0) b->st_off = (size_t)(reinterpret_cast<char*>(h->st) - b->ws);
    const fe_status ss = batch_stop_slot(b, s);
    if (ss != FE_OK) return fail(ss);
  }
  *out = b;
  return FE_OK;
}

extern "C" fe_status fe_batch_setup_slot(fe_batch* b, int32_t slot, const uint8_t* fixed, const double* f,
                                         fe_problem** out) {
  if (!b || !out || slot < 0 || slot >= b->nslots) {
    fe_set_error("invalid batch, slot or out");
    return FE_EINVAL;
  }
  *out = nullptr;
  if (b->open) {
    fe_set_error("end the open round before setting up a slot");
    return FE_EINVAL;
  }
  fe_problem* old = b->slot[slot];
  if (old && old->sc.stage != ST_DONE) {
    fe_set_error("the slot's solve is still running");
    return FE_EINVAL;
  }
  if (old) {
    // same configuration: keep the handle, its Ke, filter and multigrid
    // tables and its host resources; reset only the design's own data
    const fe_status st = reinit_design(old, fixed, f ? f : b->zero_f);
    if (st == FE_OK) {
      const fe_status ss = batch_stop_slot(b, slot);
      if (ss != FE_OK) return ss;
      *out = old;
      return FE_OK;
    }
    fe_destroy(old);
  }
  b->slot[slot] = nullptr;
  fe_problem* h = nullptr;
  fe_status st = fe_setup(&b->cfg, fixed, f ? f : b->zero_f, b->ws + (size_t)slot * b->stride, b->stride,
                          b->stream, &h);
  if (st != FE_OK) {
    (void)batch_stop_slot(b, slot);  // the region keeps a stopped state for the replays
    return st;
  }
  h->in_batch = true;
  b->slot[slot] = h;
  st = batch_stop_slot(b, slot);  // until its solve begins
  if (st != FE_OK) return st;
  *out = h;
  return FE_OK;
}

extern "C" fe_status fe_batch_round_begin(fe_batch* b) {
  if (!b) {
    fe_set_error("batch is NULL");
    return FE_EINVAL;
  }
  if (b->open) {
    fe_set_error("a round is already open");
    return FE_EINVAL;
  }
  bool any = false;
  for (fe_problem* h : b->slot) any = any || in_cg_stage(h);
  if (any) {
    if (!b->slot[0]) {
      fe_set_error("slot 0 has no problem");
      return FE_EINVAL;
    }
    if (!b->chunk) {
      const fe_status st = b->cfg.precision == FE_PREC_FP64 ? batch_capture<double>(b) : batch_capture<float>(b);
      if (st != FE_OK) return st;
    }
    const fe_status sv = batch_start_vcycles(b);
    if (sv != FE_OK) return sv;
    HIP_TRY(hipGraphLaunch(b->chunk, b->stream));
    // every slot's state in one strided copy (the states sit stride bytes apart)
    HIP_TRY(hipMemcpy2DAsync(b->h_states, sizeof(CgState), b->ws + b->st_off, b->stride, sizeof(CgState),
                             (size_t)b->nslots, hipMemcpyDeviceToHost, b->stream));
  }
  HIP_TRY(hipEventRecord(b->ev, b->stream));
  b->open = true;
  b->replayed = any;
  return FE_OK;
}

extern "C" fe_status fe_batch_round_end(fe_batch* b, int32_t* running) {
  if (!b || !b->open) {
    fe_set_error("no open round");
    return FE_EINVAL;
  }
  b->open = false;
  HIP_TRY(hipEventSynchronize(b->ev));
  fe_status first_err = FE_OK;
  auto take = [&](fe_problem* h) {
    const fe_status st = advance(h);
    if (st != FE_OK) {
      h->sc.stage = ST_DONE;
      h->sc.result = st;
      if (first_err == FE_OK) first_err = st;
    }
  };
  // a stage that only waits for a short computation whose result the host
  // needs (the float64 residual of a refinement step, the final residual and
  // compliance)
  auto waits_short = [](const fe_problem* h) {
    return h && (h->sc.stage == ST_IR_RESID || h->sc.stage == ST_FINISH);
  };
  bool again = false;
  for (int s = 0; s < b->nslots; ++s) {
    fe_problem* h = b->slot[s];
    if (!h || h->sc.stage == ST_DONE) continue;
    if (b->replayed && in_cg_stage(h)) *h->h_st = b->h_states[s];
    take(h);
    again = again || waits_short(h);
  }
  // such stages are taken now, after one wait for the stream, so the slot
  // rejoins the next replay (or is free) instead of sitting a round out
  for (int pass = 0; again && pass < 3; ++pass) {
    HIP_TRY(hipStreamSynchronize(b->stream));
    again = false;
    for (int s = 0; s < b->nslots; ++s) {
      fe_problem* h = b->slot[s];
      if (!waits_short(h)) continue;
      take(h);
      again = again || waits_short(h);
    }
  }
  int n = 0;
  for (int s = 0; s < b->nslots; ++s)
    if (b->slot[s] && b->slot[s]->sc.stage != ST_DONE) ++n;
  if (running) *running = n;
  return first_err;
}

extern "C" fe_status fe_batch_round_ready(fe_batch* b, int32_t* ready) {
  if (!b || !ready) {
    fe_set_error("batch and ready must not be NULL");
    return FE_EINVAL;
  }
  if (!b->open) {
    *ready = 1;
    return FE_OK;
  }
  const hipError_t q = hipEventQuery(b->ev);
  if (q == hipErrorNotReady) {
    *ready = 0;
    return FE_OK;
  }
  HIP_TRY(q);
  *ready = 1;
  return FE_OK;
}

extern "C" void fe_batch_destroy(fe_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (fe_problem* h : b->slot)
    if (h) fe_destroy(h);
  if (b->chunk) (void)hipGraphExecDestroy(b->chunk);
  if (b->ev) (void)hipEventDestroy(b->ev);
  if (b->h_states) (void)hipHostFree(b->h_states);
  delete b;
}
