// C ABI entry points: validation, workspace layout, setup and the solver
// drivers (float64 PCG and float32 PCG inside float64 iterative refinement).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "fe_internal.h"

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// scal[] slots: value at 2*s, arrival counter of its reduction at 2*s + 1.
enum { SLOT_FF = 0, SLOT_RR = 1, SLOT_C = 2, SLOT_TMP = 3, NSCAL = 128 };

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
  if (!(c->filter_r > 0.0) || c->filter_r > 7.0) return "filter_r must lie in (0, 7]";
  if (c->precision < FE_PREC_FP64 || c->precision > FE_PREC_BF16_IR) return "unknown precision";
  if (c->precond != FE_PRECOND_JACOBI && c->precond != FE_PRECOND_GMG) return "unknown preconditioner";
  if (c->reserved != 0) return "reserved must be 0";
  if (c->precond == FE_PRECOND_GMG) {
    if (c->mg_levels < 2 || c->mg_levels > FE_MAX_LEVELS) return "mg_levels must lie in [2, 6]";
    const int d = 1 << (c->mg_levels - 1);
    if (c->nx % d || c->ny % d || c->nz % d)
      return "grid dimensions must be divisible by 2^(mg_levels-1) for multigrid";
  }
  // the stencil table holds at most 512 offsets
  const int R = (int)std::ceil(c->filter_r);
  int cnt = 0;
  for (int dk = -R; dk <= R; ++dk)
    for (int dj = -R; dj <= R; ++dj)
      for (int di = -R; di <= R; ++di)
        if (c->filter_r - std::sqrt((double)(di * di + dj * dj + dk * dk)) > 0.0) ++cnt;
  if (cnt > 512) return "filter radius too large";
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
    }
    if (p) p->L[l] = L;
    int64_t nb = (g.nnode + FE_BLOCK - 1) / FE_BLOCK;
    if (kxu_tile_blocks(g) > nb) nb = kxu_tile_blocks(g);
    if (nb > max_blocks) max_blocks = nb;
    nx /= 2;
    ny /= 2;
    nz /= 2;
    h *= 2.0;
  }
  double* f = (double*)take(g0.ndof * sizeof(double));
  double* invW = (double*)take(g0.nelem * sizeof(double));
  int4* st_off = (int4*)take(512 * sizeof(int4));
  double* st_w = (double*)take(512 * sizeof(double));
  double* r64 = (double*)take(g0.ndof * sizeof(double));
  double* p64 = (double*)take(g0.ndof * sizeof(double));
  double* q64 = (double*)take(g0.ndof * sizeof(double));
  double* tmp64 = (double*)take(g0.ndof * sizeof(double));
  float *x32 = nullptr, *r32 = nullptr, *p32 = nullptr, *q32 = nullptr;
  if (f32) {
    x32 = (float*)take(g0.ndof * sizeof(float));
    r32 = (float*)take(g0.ndof * sizeof(float));
    p32 = (float*)take(g0.ndof * sizeof(float));
    q32 = (float*)take(g0.ndof * sizeof(float));
  }
  size_t npart = (size_t)FE_RED_GRID * 64;
  if ((size_t)max_blocks * 2 > npart) npart = (size_t)max_blocks * 2;
  double* partials = (double*)take(npart * sizeof(double));
  CgState* st = (CgState*)take(2 * sizeof(CgState));
  double* scal = (double*)take(NSCAL * sizeof(double));
  double* oc = (double*)take(64 * sizeof(double));
  double* ke64 = (double*)take(576 * sizeof(double));
  float* ke32 = (float*)take(576 * sizeof(float));
  if (p) {
    p->nlev = nl;
    p->f = f;
    p->invW = invW;
    p->st_off = st_off;
    p->st_w = st_w;
    p->r64 = r64;
    p->p64 = p64;
    p->q64 = q64;
    p->tmp64 = tmp64;
    p->x32 = x32;
    p->r32 = r32;
    p->p32 = p32;
    p->q32 = q32;
    p->partials = partials;
    p->st = st;
    p->scal = scal;
    p->oc = oc;
    p->ke64 = ke64;
    p->ke32 = ke32;
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

constexpr int kChunk = 24;    // Jacobi-PCG iterations enqueued between host checks
constexpr int kChunkMG = 8;   // multigrid-PCG iterations enqueued between host checks

// Preconditioned CG on level 0 with vectors of type T, from the state set by
// cg_start.  Returns the CgState at exit.
template <typename T>
fe_status cg_loop(fe_problem* p, T* x, T* r, T* pv, T* q, CgState* out) {
  const bool mg = p->nlev > 1;
  T* z = mg ? static_cast<T*>(p->L[0].mg_z) : nullptr;
  const int chunk = mg ? kChunkMG : kChunk;
  for (;;) {
    for (int it = 0; it < chunk; ++it) {
      HIP_TRY(launch_kxu<T>(p, 0, pv, q, p->st));
      HIP_TRY(launch_cg_update<T>(p, x, r, pv, q, p->st, mg ? 1 : 0));
      if (mg) HIP_TRY(launch_vcycle<T>(p, 0, r, z, p->st, true));
      HIP_TRY(launch_cg_direction<T>(p, r, z, pv, p->st));
    }
    fe_status s = read_state(p, out);
    if (s != FE_OK) return s;
    if (out->done) return FE_OK;
  }
}

// r = b - Kx (Kx null: x = 0), first preconditioned direction, convergence
// test of the start point.
template <typename T>
fe_status cg_start(fe_problem* p, const T* b, const T* Kx, T* r, T* pv, CgState* hs) {
  const bool mg = p->nlev > 1;
  HIP_TRY(launch_cg_init<T>(p, b, Kx, r, pv, p->st, mg ? 1 : 0));
  if (mg) {
    T* z = static_cast<T*>(p->L[0].mg_z);
    HIP_TRY(launch_fill<T>(p, pv, p->L[0].g.ndof, T(0)));
    HIP_TRY(launch_vcycle<T>(p, 0, r, z, p->st, true));
    HIP_TRY(launch_cg_direction<T>(p, r, z, pv, p->st));
  }
  return read_state(p, hs);
}

fe_status solve_fp64(fe_problem* p, double* u, double rtol, int max_iters, fe_solve_info* info) {
  HIP_TRY(launch_kxu<double>(p, 0, u, p->q64, nullptr));
  HIP_TRY(launch_cg_state_init(p, p->st, rtol, max_iters));
  CgState hs;
  fe_status s = cg_start<double>(p, p->f, p->q64, p->r64, p->p64, &hs);
  if (s != FE_OK) return s;
  if (!hs.done) {
    s = cg_loop<double>(p, u, p->r64, p->p64, p->q64, &hs);
    if (s != FE_OK) return s;
  }
  info->iters = hs.iter;
  info->outer_iters = 0;
  return (fe_status)hs.status;
}

// float32 PCG on K d = r / ||r|| inside float64 refinement u += ||r|| d.
fe_status solve_ir(fe_problem* p, double* u, double rtol, int max_iters, fe_solve_info* info,
                   double ff) {
  int total = 0, outer = 0;
  fe_status result = FE_ENOTCONV;
  const int max_outer = 40;
  double prev_rel = 1e300;
  for (;;) {
    HIP_TRY(launch_residual64(p, u, p->r64, p->scal + 2 * SLOT_RR));
    double rr;
    fe_status s = read_scal(p, SLOT_RR, &rr);
    if (s != FE_OK) return s;
    const double rel = std::sqrt(rr / ff);
    if (!std::isfinite(rel)) {
      result = FE_EBREAKDOWN;
      break;
    }
    if (rel <= rtol) {
      result = FE_OK;
      break;
    }
    if (outer >= max_outer || total >= max_iters || rel > 0.99 * prev_rel) {
      result = FE_ENOTCONV;
      break;
    }
    prev_rel = rel;
    // inner tolerance: aim a little past the target, within float32 reach
    double itol = 0.3 * rtol / rel;
    if (itol < 1e-5) itol = 1e-5;
    if (itol > 1e-1) itol = 1e-1;
    HIP_TRY(launch_to32_scaled(p, p->r64, p->r32, p->scal + 2 * SLOT_RR));
    HIP_TRY(launch_fill<float>(p, p->x32, p->L[0].g.ndof, 0.0f));
    HIP_TRY(launch_cg_state_init(p, p->st, itol, max_iters - total));
    CgState hs;
    s = cg_start<float>(p, p->r32, nullptr, p->r32, p->p32, &hs);
    if (s != FE_OK) return s;
    if (!hs.done) {
      s = cg_loop<float>(p, p->x32, p->r32, p->p32, p->q32, &hs);
      if (s != FE_OK) return s;
    }
    total += hs.iter;
    ++outer;
    if (hs.iter > 0) HIP_TRY(launch_axpy_from32(p, u, p->x32, p->scal + 2 * SLOT_RR));
    if (hs.status == FE_EBREAKDOWN && hs.iter == 0) {
      result = FE_EBREAKDOWN;
      break;
    }
  }
  info->iters = total;
  info->outer_iters = outer;
  return result;
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
  p->stream = (hipStream_t)stream;
  p->ws = (char*)ws;
  p->ws_bytes = ws_bytes;
  layout(cfg, p, (char*)ws);

  // Ke and its sum/difference-basis constants (unit modulus, unit edge)
  host_hex8_ke(cfg->nu, 1.0, 1.0, p->ke64_host);
  double dev = 0.0;
  host_walsh_constants(p->ke64_host, &p->wk, &dev);
  if (dev > 1e-12) {
    delete p;
    fe_set_error("element stiffness lacks the cube symmetry the kernels rely on");
    return FE_EINVAL;
  }
  p->ke_diag = p->ke64_host[0];
  {
    // lambda_max(Ke) / Ke_dd by power iteration (Ke is symmetric positive
    // semi-definite); it bounds lambda_max(D^-1 K) for any modulus field
    double v[24], w[24], lam = 0.0;
    for (int i = 0; i < 24; ++i) v[i] = 1.0 + 0.01 * i * ((i & 1) ? -1.0 : 1.0);
    for (int it = 0; it < 5000; ++it) {
      double nrm = 0.0;
      for (int i = 0; i < 24; ++i) {
        double s2 = 0.0;
        for (int j = 0; j < 24; ++j) s2 += p->ke64_host[i * 24 + j] * v[j];
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
    p->lam_max = lam / p->ke_diag;
  }
  float ke32h[576];
  for (int i = 0; i < 576; ++i) ke32h[i] = (float)p->ke64_host[i];

  // filter stencil: offsets with positive cone weight r - |d|
  int4 off[512];
  double w[512];
  int n = 0;
  const double r = cfg->filter_r;
  const int R = (int)std::ceil(r);
  for (int dk = -R; dk <= R; ++dk)
    for (int dj = -R; dj <= R; ++dj)
      for (int di = -R; di <= R; ++di) {
        const double wt = r - std::sqrt((double)(di * di + dj * dj + dk * dk));
        if (wt > 0.0) {
          off[n] = make_int4(di, dj, dk, 0);
          w[n] = wt;
          ++n;
        }
      }
  p->nstencil = n;

  auto fail = [&](hipError_t e, const char* what) {
    fe_set_error(std::string(what) + ": " + hipGetErrorString(e));
    delete p;
    return FE_EDEVICE;
  };
  hipError_t e;
  if ((e = hipMemcpyAsync(p->ke64, p->ke64_host, sizeof(p->ke64_host), hipMemcpyHostToDevice, p->stream)))
    return fail(e, "copy Ke");
  if ((e = hipMemcpyAsync(p->ke32, ke32h, sizeof(ke32h), hipMemcpyHostToDevice, p->stream)))
    return fail(e, "copy Ke32");
  if ((e = hipMemcpyAsync(p->st_off, off, n * sizeof(int4), hipMemcpyHostToDevice, p->stream)))
    return fail(e, "copy stencil");
  if ((e = hipMemcpyAsync(p->st_w, w, n * sizeof(double), hipMemcpyHostToDevice, p->stream)))
    return fail(e, "copy stencil weights");
  if ((e = launch_fill<double>(p, p->scal, NSCAL, 0.0))) return fail(e, "clear scalars");
  if ((e = launch_fill<double>(p, (double*)p->st, 2 * sizeof(CgState) / sizeof(double), 0.0)))
    return fail(e, "clear state");
  if ((e = launch_fill<double>(p, p->oc, 64, 0.0))) return fail(e, "clear oc state");
  if ((e = launch_node_mask(p, fixed))) return fail(e, "node mask");
  for (int l = 1; l < p->nlev; ++l)
    if ((e = launch_coarsen_mask(p, l))) return fail(e, "coarse mask");
  if ((e = launch_mask_load(p, f))) return fail(e, "load");
  if ((e = launch_filter_rowsums(p))) return fail(e, "filter row sums");
  if ((e = launch_dot64(p, p->f, p->f, p->L[0].g.ndof, p->scal + 2 * SLOT_FF))) return fail(e, "||f||");
  // host copies above read stack arrays: finish them before returning
  if ((e = hipStreamSynchronize(p->stream))) return fail(e, "setup sync");
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
  if (variant == 1) {
    if (p->cfg.precision == FE_PREC_FP64) {
      fe_set_error("float32 variant needs a problem set up with a reduced precision");
      return FE_EINVAL;
    }
    HIP_TRY(launch_convert_64_32(p, u, p->x32, ndof));
    HIP_TRY(launch_mask_vec<float>(p, 0, p->x32));
    HIP_TRY(launch_kxu<float>(p, 0, p->x32, p->q32, nullptr));
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
  if (!rho || !u) {
    fe_set_error("rho and u must not be NULL");
    return FE_EINVAL;
  }
  if (!(rtol > 0.0) || max_iters < 1) {
    fe_set_error("rtol must be > 0 and max_iters >= 1");
    return FE_EINVAL;
  }
  fe_solve_info local;
  if (!info) info = &local;
  std::memset(info, 0, sizeof(*info));
  fe_status s = prepare_operator(p, rho);
  if (s != FE_OK) return s;
  HIP_TRY(launch_mask_vec<double>(p, 0, u));
  double ff;
  s = read_scal(p, SLOT_FF, &ff);
  if (s != FE_OK) return s;
  if (!(ff > 0.0)) {  // no load: u = 0 is exact
    HIP_TRY(launch_fill<double>(p, u, p->L[0].g.ndof, 0.0));
    HIP_TRY(hipStreamSynchronize(p->stream));
    return FE_OK;
  }
  fe_status res;
  if (p->cfg.precision == FE_PREC_FP64)
    res = solve_fp64(p, u, rtol, max_iters, info);
  else
    res = solve_ir(p, u, rtol, max_iters, info, ff);
  if (res == FE_EDEVICE || res == FE_EINVAL) return res;
  // true float64 residual and compliance of the returned u
  HIP_TRY(launch_residual64(p, u, p->tmp64, p->scal + 2 * SLOT_RR));
  HIP_TRY(launch_dot64(p, p->f, u, p->L[0].g.ndof, p->scal + 2 * SLOT_C));
  double rr, c;
  s = read_scal(p, SLOT_RR, &rr);
  if (s != FE_OK) return s;
  s = read_scal(p, SLOT_C, &c);
  if (s != FE_OK) return s;
  info->rel_res = std::sqrt(rr / ff);
  info->compliance = c;
  if (res == FE_ENOTCONV)
    fe_set_error("iteration limit reached (relative residual " + std::to_string(info->rel_res) + ")");
  if (res == FE_EBREAKDOWN) fe_set_error("CG breakdown (p^T K p <= 0 or non-finite value)");
  return res;
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

extern "C" fe_status fe_filter(fe_problem* p, const double* in, double* out, int32_t transpose) {
  CHECK_HANDLE(p);
  if (!in || !out || in == out) {
    fe_set_error("in and out must be distinct non-NULL arrays");
    return FE_EINVAL;
  }
  HIP_TRY(launch_filter(p, in, out, transpose ? 1 : 0));
  return FE_OK;
}

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
  HIP_TRY(launch_oc(p, x, dcx, dv, volfrac, move, x_new, change));
  return FE_OK;
}

extern "C" fe_status fe_set_mg_params(fe_problem* p, int32_t nu, int32_t coarse_sweeps, double omega) {
  CHECK_HANDLE(p);
  if (nu < 1 || nu > 8 || coarse_sweeps < 1 || coarse_sweeps > 10000 || !(omega > 0.0 && omega < 1.0)) {
    fe_set_error("need 1 <= nu <= 8, 1 <= coarse_sweeps <= 10000, 0 < omega < 1");
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
  return FE_OK;
}

extern "C" fe_status fe_set_profiling(fe_problem* p, int32_t on) {
  CHECK_HANDLE(p);
  p->kst.on = on != 0;
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
  if (p->stream) hipStreamSynchronize(p->stream);
  for (hipEvent_t e : p->kst.ev) hipEventDestroy(e);
  delete p;
}
