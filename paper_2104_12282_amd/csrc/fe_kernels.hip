// Element, node and vector kernels of the FE step (gfx950, wave64).
#include <hip/hip_runtime.h>

#include <mutex>

#include "fe_internal.h"
#include "fe_reduce.h"

namespace {

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int red_grid(int64_t n) {
  int64_t g = ceil_div(n, FE_BLOCK);
  if (g > FE_RED_GRID) g = FE_RED_GRID;
  if (g < 1) g = 1;
  return (int)g;
}

// Corner offsets of the brick in the fixed local order.
__constant__ int c_cx[8] = {0, 1, 1, 0, 0, 1, 1, 0};
__constant__ int c_cy[8] = {0, 0, 1, 1, 0, 0, 1, 1};
__constant__ int c_cz[8] = {0, 0, 0, 0, 1, 1, 1, 1};

// ------------------------------------------------------------------ SIMP
template <typename T>
__global__ void __launch_bounds__(FE_BLOCK) simp_kernel(const double* __restrict__ rho, int64_t n,
                                                        double E0, double Emin, double penal,
                                                        double* __restrict__ E64,
                                                        float* __restrict__ E32) {
  for (int64_t e = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * FE_BLOCK) {
    const double r = rho[e];
    const double E = Emin + pow(r, penal) * (E0 - Emin);
    if (E64) E64[e] = E;
    if (E32) E32[e] = (float)E;
  }
}

// Coarse modulus: mean of the 8 fine children of each coarse element, a
// child past the mesh (the overhanging last element of an odd axis) counting
// as void: the rediscretised element then carries the stiffness of the part
// of it that lies in the mesh, as the Galerkin product of the prolongation
// would.
__global__ void __launch_bounds__(FE_BLOCK) coarsen_modulus_kernel(Grid fg, Grid cg,
                                                                   const double* __restrict__ Ef,
                                                                   double* __restrict__ Ec64,
                                                                   float* __restrict__ Ec32) {
  for (int64_t e = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; e < cg.nelem;
       e += (int64_t)gridDim.x * FE_BLOCK) {
    const int i = (int)(e % cg.nx), j = (int)((e / cg.nx) % cg.ny), k = (int)(e / ((int64_t)cg.nx * cg.ny));
    double s = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int fi = 2 * i + c_cx[c], fj = 2 * j + c_cy[c], fk = 2 * k + c_cz[c];
      if (fi < fg.nx && fj < fg.ny && fk < fg.nz) s += Ef[fi + (int64_t)fg.nx * (fj + (int64_t)fg.ny * fk)];
    }
    const double E = s / 8.0;
    if (Ec64) Ec64[e] = E;
    if (Ec32) Ec32[e] = (float)E;
  }
}

// --------------------------------------------------------------- masks
__global__ void __launch_bounds__(FE_BLOCK) node_mask_kernel(Grid g, const uint8_t* __restrict__ fixed,
                                                             uint8_t* __restrict__ nmask) {
  for (int64_t n = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; n < g.nnode;
       n += (int64_t)gridDim.x * FE_BLOCK) {
    uint8_t m = 0;
    if (fixed) {
      for (int c = 0; c < 3; ++c) m |= (fixed[3 * n + c] ? 1 : 0) << c;
    } else {
      m = (n % (g.nx + 1)) == 0 ? 7 : 0;
    }
    nmask[n] = m;
  }
}

// A coarse node is fixed in component c when the fine node at the same place
// is; a coarse node just past the mesh (odd axis) takes the last fine node's.
__global__ void __launch_bounds__(FE_BLOCK) coarsen_mask_kernel(Grid fg, Grid cg,
                                                                const uint8_t* __restrict__ fm,
                                                                uint8_t* __restrict__ cm) {
  for (int64_t n = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; n < cg.nnode;
       n += (int64_t)gridDim.x * FE_BLOCK) {
    const int i = (int)(n % (cg.nx + 1)), j = (int)((n / (cg.nx + 1)) % (cg.ny + 1)),
              k = (int)(n / ((int64_t)(cg.nx + 1) * (cg.ny + 1)));
    const int fi = min(2 * i, fg.nx), fj = min(2 * j, fg.ny), fk = min(2 * k, fg.nz);
    cm[n] = fm[fi + (int64_t)(fg.nx + 1) * (fj + (int64_t)(fg.ny + 1) * fk)];
  }
}

__global__ void __launch_bounds__(FE_BLOCK) mask_load_kernel(Grid g, const double* __restrict__ fin,
                                                             const uint8_t* __restrict__ nmask,
                                                             double* __restrict__ fout) {
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < g.ndof;
       d += (int64_t)gridDim.x * FE_BLOCK) {
    const int64_t n = d / 3;
    const int c = (int)(d - 3 * n);
    fout[d] = ((nmask[n] >> c) & 1) ? 0.0 : fin[d];
  }
}

template <typename T>
__global__ void __launch_bounds__(FE_BLOCK) mask_vec_kernel(Grid g, const uint8_t* __restrict__ nmask,
                                                            T* __restrict__ v) {
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < g.ndof;
       d += (int64_t)gridDim.x * FE_BLOCK) {
    const int64_t n = d / 3;
    const int c = (int)(d - 3 * n);
    if ((nmask[n] >> c) & 1) v[d] = T(0);
  }
}

// ---------------------------------------------------------- Jacobi diag
// All 24 diagonal entries of Ke are equal (cube, isotropic), so
// diag K at node n = kdiag * sum of the moduli of the elements around n.
__global__ void __launch_bounds__(FE_BLOCK) diag_kernel(Grid g, const double* __restrict__ E,
                                                        double kdiag, double* __restrict__ invd64,
                                                        float* __restrict__ invd32) {
  for (int64_t n = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; n < g.nnode;
       n += (int64_t)gridDim.x * FE_BLOCK) {
    const int i = (int)(n % (g.nx + 1)), j = (int)((n / (g.nx + 1)) % (g.ny + 1)),
              k = (int)(n / ((int64_t)(g.nx + 1) * (g.ny + 1)));
    double s = 0.0;
    for (int c = 0; c < 8; ++c) {
      const int ei = i - c_cx[c], ej = j - c_cy[c], ek = k - c_cz[c];
      if (ei >= 0 && ei < g.nx && ej >= 0 && ej < g.ny && ek >= 0 && ek < g.nz)
        s += E[ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek)];
    }
    const double d = 1.0 / (kdiag * s);
    if (invd64) invd64[n] = d;
    if (invd32) invd32[n] = (float)d;
  }
}

// ------------------------------------------------ K * x, dense reference
// Node-centric, dense Ke: node n sums, over the (up to) 8 bricks around it,
// E_e * (row block of Ke for n's corner) * u_e.  Kept as a second, plainly
// written implementation of the operator (float64).  Inputs must be zero on
// fixed dofs; outputs are zeroed there.
__global__ void __launch_bounds__(FE_BLOCK) kxu_dense_kernel(Grid g, const double* __restrict__ x,
                                                             const double* __restrict__ E,
                                                             const uint8_t* __restrict__ nmask,
                                                             const double* __restrict__ ke, double kscale,
                                                             double* __restrict__ y) {
  __shared__ double sKe[576];
  for (int i = threadIdx.x; i < 576; i += FE_BLOCK) sKe[i] = ke[i] * kscale;
  __syncthreads();
  const int64_t n = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x;
  if (n >= g.nnode) return;
  const int i = (int)(n % (g.nx + 1)), j = (int)((n / (g.nx + 1)) % (g.ny + 1)),
            k = (int)(n / ((int64_t)(g.nx + 1) * (g.ny + 1)));
  double acc[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < 8; ++a) {
    const int ei = i - c_cx[a], ej = j - c_cy[a], ek = k - c_cz[a];
    if (ei < 0 || ei >= g.nx || ej < 0 || ej >= g.ny || ek < 0 || ek >= g.nz) continue;
    const double Ee = E[ei + (int64_t)g.nx * (ej + (int64_t)g.ny * ek)];
    double ue[24];
#pragma unroll
    for (int bb = 0; bb < 8; ++bb) {
      const int64_t nb = (ei + c_cx[bb]) + (int64_t)(g.nx + 1) * ((ej + c_cy[bb]) + (int64_t)(g.ny + 1) * (ek + c_cz[bb]));
      ue[3 * bb + 0] = x[3 * nb + 0];
      ue[3 * bb + 1] = x[3 * nb + 1];
      ue[3 * bb + 2] = x[3 * nb + 2];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double* row = &sKe[(3 * a + c) * 24];
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 24; ++q) s += row[q] * ue[q];
      acc[c] += Ee * s;
    }
  }
  const uint8_t m = nmask[n];
#pragma unroll
  for (int c = 0; c < 3; ++c) y[3 * n + c] = ((m >> c) & 1) ? 0.0 : acc[c];
}

// ------------------------------------------------------------- CG pieces
// r = b - Kx (Kx may be null: x = 0), z = D^-1 r, p = z, and rz, rr, bb.
template <typename T>
__global__ void __launch_bounds__(FE_BLOCK) cg_init_kernel(Grid g, const T* __restrict__ b,
                                                           const T* __restrict__ Kx, T* __restrict__ r,
                                                           T* __restrict__ p, const T* __restrict__ invd,
                                                           double* partials, int mg) {
  double acc[3] = {0.0, 0.0, 0.0};  // rz, rr, bb
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < g.ndof;
       d += (int64_t)gridDim.x * FE_BLOCK) {
    const T bv = b[d];
    const T rv = Kx ? (T)(bv - Kx[d]) : bv;
    r[d] = rv;
    if (!mg) {
      const T zv = rv * invd[d / 3];
      p[d] = zv;
      acc[0] += (double)rv * (double)zv;
    }
    acc[1] += (double)rv * (double)rv;
    acc[2] += (double)bv * (double)bv;
  }
  block_partials<3>(acc, partials);
}

// x += alpha p, r -= alpha q, (Jacobi) rz = r^T D^-1 r, rr = r^T r; then the
// convergence test.  With mg = 1 (the unfolded multigrid CG, which the
// matrix-core problems use) the V-cycle's last sweep forms rz.
template <typename T>
__global__ void __launch_bounds__(FE_BLOCK) cg_update_kernel(Grid g, T* __restrict__ x, T* __restrict__ r,
                                                             const T* __restrict__ p, const T* __restrict__ q,
                                                             const T* __restrict__ invd, CgState* st,
                                                             double* partials, int mg) {
  if (st->done) return;
  const T alpha = (T)st->alpha;
  double acc[2] = {0.0, 0.0};
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < g.ndof;
       d += (int64_t)gridDim.x * FE_BLOCK) {
    x[d] += alpha * p[d];
    const T rv = r[d] - alpha * q[d];
    r[d] = rv;
    if (!mg) acc[0] += (double)rv * (double)rv * (double)invd[d / 3];
    acc[1] += (double)rv * (double)rv;
  }
  block_partials<2>(acc, partials);
}

// Multigrid CG update.  Every workgroup sums the p^T q partials the direction
// kernel left (same order, same value), alpha = rz_new / p^T q; workgroup 0
// commits rz and the step.  Then r -= alpha q with r^T r partials for the
// convergence test the next kernel takes, and the iterate's update, made for
// two iterations at once: with x null it is deferred (workgroup 0 records
// alpha and p in st), with x given the deferred step is applied with this
// one, x += x_alpha p_old + alpha p, while the previous direction p_old is
// still in its buffer (x is read and written once per two iterations).
template <typename T>
__global__ void __launch_bounds__(FE_BLOCK) cg_update_mg_kernel(Grid g, T* __restrict__ x, T* __restrict__ r,
                                                                const T* __restrict__ p,
                                                                const T* __restrict__ q, CgState* st,
                                                                const double* __restrict__ pq_part, int npq,
                                                                double* partials, int64_t wsh,
                                                                float* __restrict__ r32,
                                                                const T* __restrict__ pold) {
  if (wsh) {  // batched launch: this workgroup's problem
    const int64_t o = batch_offset(wsh);
    x = wshift(x, o);
    r = wshift(r, o);
    p = wshift(p, o);
    pold = wshift(pold, o);
    q = wshift(q, o);
    st = wshift(st, o);
    pq_part = wshift(pq_part, o);
    partials = wshift(partials, o);
    r32 = wshift(r32, o);
  }
  if (st->done) return;
  __shared__ double sh[FE_BLOCK / 64];
  __shared__ double tot;
  double v = 0.0;
  for (int i = threadIdx.x; i < npq; i += FE_BLOCK) v += pq_part[i];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < FE_BLOCK / 64; ++w) t += sh[w];
    tot = t;
  }
  __syncthreads();
  const double pq = tot, rz = st->rz_new;
  const bool bad = !(pq > 0.0) || !finite_d(pq);
  // the deferred step (written by the previous update launch, not by this one)
  const T xa = x ? (T)st->x_alpha : T(0);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->pq = pq;
    if (!x && !bad) {
      st->x_alpha = rz / pq;
      st->x_dir = const_cast<T*>(p);
    }
    if (bad) {
      st->status = FE_EBREAKDOWN;
      st->done = 1;
    } else {
      st->alpha = rz / pq;
      st->rz = rz;
      st->iter_next = st->iter + 1;
    }
  }
  if (bad) return;
  const T alpha = (T)(rz / pq);
  double acc[1] = {0.0};
  const bool upd_x = x != nullptr;
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < g.ndof;
       d += (int64_t)gridDim.x * FE_BLOCK) {
    if (upd_x) {
      T xv = x[d];
      xv += xa * pold[d];
      xv += alpha * p[d];
      x[d] = xv;
    }
    const T rv = r[d] - alpha * q[d];
    r[d] = rv;
    if (r32) r32[d] = (float)rv;  // the residual a float32 preconditioner reads
    acc[0] += (double)rv * (double)rv;
  }
  block_partials<1>(acc, partials);
}

// x += x_alpha x_dir (the update a multigrid CG deferred before it stopped)
template <typename T>
__global__ void __launch_bounds__(FE_BLOCK) cg_flush_x_kernel(int64_t n, T* __restrict__ x, const CgState* st) {
  const T* __restrict__ p = static_cast<const T*>(st->x_dir);
  const T alpha = (T)st->x_alpha;
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < n; d += (int64_t)gridDim.x * FE_BLOCK)
    x[d] += alpha * p[d];
}

// b = (float)a
__global__ void __launch_bounds__(FE_BLOCK) narrow_kernel(int64_t n, const double* __restrict__ a,
                                                          float* __restrict__ b, int64_t wsh) {
  if (wsh) {
    const int64_t o = batch_offset(wsh);
    a = wshift(a, o);
    b = wshift(b, o);
  }
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < n; d += (int64_t)gridDim.x * FE_BLOCK)
    b[d] = (float)a[d];
}

// Scalar updates of CG, one workgroup, after the kernel that left nb partials.

__global__ void __launch_bounds__(FE_BLOCK) cg_finalize_kernel(int op, int nb, int mg,
                                                               const double* __restrict__ partials,
                                                               CgState* st, double* out) {
  if (op != FIN_SCALAR && op != FIN_INIT && st->done) return;
  if (op == FIN_INIT) {
    double acc[3];
    reduce_partials<3>(acc, partials, nb);
    if (threadIdx.x == 0) {
      st->rz = acc[0];
      st->rr = acc[1];
      st->bb = acc[2];
      st->tol2 = st->tol2 * acc[2];  // tol2 held rtol^2 until now
      st->iter = 0;
      st->status = FE_OK;
      st->done = (acc[1] <= st->tol2) ? 1 : 0;
      if (!finite_d(acc[1])) {
        st->status = FE_EBREAKDOWN;
        st->done = 1;
      }
    }
  } else if (op == FIN_UPDATE) {
    double acc[2];
    reduce_partials<2>(acc, partials, nb);
    if (threadIdx.x == 0) {
      st->iter += 1;
      st->rr = acc[1];
      if (!mg) {
        st->beta = acc[0] / st->rz;
        st->rz = acc[0];
      }
      if (!finite_d(acc[1])) {
        st->status = FE_EBREAKDOWN;
        st->done = 1;
      } else if (acc[1] <= st->tol2) {
        st->status = FE_OK;
        st->done = 1;
      } else if (st->iter >= st->max_iter) {
        st->status = FE_ENOTCONV;
        st->done = 1;
      }
    }
  } else {
    double acc[1];
    reduce_partials<1>(acc, partials, nb);
    if (threadIdx.x == 0) {
      const double v = acc[0];
      if (op == FIN_ALPHA) {
        st->pq = v;
        if (!(v > 0.0) || !finite_d(v)) {
          st->status = FE_EBREAKDOWN;
          st->done = 1;
        } else {
          st->alpha = st->rz / v;
        }
      } else if (op == FIN_RZ) {
        st->beta = st->iter == 0 ? 0.0 : v / st->rz;
        st->rz = v;
        if (!finite_d(v) || !(v > 0.0)) {
          st->status = FE_EBREAKDOWN;
          st->done = 1;
        }
      } else {
        out[0] = v;
      }
    }
  }
}

// p = z + beta p, z = D^-1 r when z is null (Jacobi).
template <typename T>
__global__ void __launch_bounds__(FE_BLOCK) cg_direction_kernel(Grid g, const T* __restrict__ r,
                                                                const T* __restrict__ z,
                                                                const T* __restrict__ invd,
                                                                T* __restrict__ p, CgState* st) {
  if (st->done) return;
  const T beta = (T)st->beta;
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < g.ndof;
       d += (int64_t)gridDim.x * FE_BLOCK) {
    const T zv = z ? z[d] : r[d] * invd[d / 3];
    p[d] = zv + beta * p[d];
  }
}

__global__ void cg_state_resume_kernel(CgState* st, double tol2, int max_iter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->tol2 = tol2;
    st->max_iter = max_iter;
    st->done = 0;
    st->status = FE_OK;
  }
}

__global__ void cg_guard_kernel(CgState* g, int done, int64_t wsh) {
  if (wsh) g = wshift(g, batch_offset(wsh));
  if (threadIdx.x == 0) g->done = done;
}

__global__ void cg_state_init_kernel(CgState* st, double tol_rel, int max_iter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->rz = st->alpha = st->beta = st->rr = st->bb = st->pq = 0.0;
    st->tol2 = tol_rel * tol_rel;
    st->iter = 0;
    st->max_iter = max_iter;
    st->done = 0;
    st->status = FE_OK;
    for (int i = 0; i < 8; ++i) st->counter[i] = 0;
  }
}

// --------------------------------------------------- refinement helpers
__global__ void __launch_bounds__(FE_BLOCK) to32_scaled_kernel(int64_t n, const double* __restrict__ a,
                                                               float* __restrict__ b,
                                                               const double* __restrict__ nrm2) {
  const double s = 1.0 / sqrt(*nrm2);
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < n;
       d += (int64_t)gridDim.x * FE_BLOCK)
    b[d] = (float)(a[d] * s);
}

__global__ void __launch_bounds__(FE_BLOCK) axpy_from32_kernel(int64_t n, double* __restrict__ u,
                                                               const float* __restrict__ dvec,
                                                               const double* __restrict__ nrm2) {
  const double s = sqrt(*nrm2);
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < n;
       d += (int64_t)gridDim.x * FE_BLOCK)
    u[d] += (double)dvec[d] * s;
}

__global__ void __launch_bounds__(FE_BLOCK) dot64_kernel(int64_t n, const double* __restrict__ a,
                                                         const double* __restrict__ b, double* partials,
                                                         double* out) {
  double acc[1] = {0.0};
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < n;
       d += (int64_t)gridDim.x * FE_BLOCK)
    acc[0] += a[d] * b[d];
  block_partials<1>(acc, partials);
}

template <typename T>
__global__ void __launch_bounds__(FE_BLOCK) fill_kernel(int64_t n, T* __restrict__ v, T val) {
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < n;
       d += (int64_t)gridDim.x * FE_BLOCK)
    v[d] = val;
}

template <typename A, typename B>
__global__ void __launch_bounds__(FE_BLOCK) convert_kernel(int64_t n, const A* __restrict__ a,
                                                           B* __restrict__ b) {
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < n;
       d += (int64_t)gridDim.x * FE_BLOCK)
    b[d] = (B)a[d];
}

// ------------------------------------------------------- sensitivity
// dc_e = -p rho^(p-1) (E0 - Emin) u_e^T Ke u_e, with u_e^T Ke u_e = t^T S t
// in the per-axis sum/difference basis (t = Walsh transform of the corners).
__device__ inline void bfly(double& a, double& b) {
  const double s = a + b, d = a - b;
  a = s;
  b = d;
}

__device__ inline void walsh8(double (&v)[8]) {
  // corners in local order 000 100 110 010 001 101 111 011
  bfly(v[0], v[1]); bfly(v[3], v[2]); bfly(v[4], v[5]); bfly(v[7], v[6]);  // x
  bfly(v[0], v[3]); bfly(v[1], v[2]); bfly(v[4], v[7]); bfly(v[5], v[6]);  // y
  bfly(v[0], v[4]); bfly(v[1], v[5]); bfly(v[2], v[6]); bfly(v[3], v[7]);  // z
}

__global__ void __launch_bounds__(FE_BLOCK) sensitivity_kernel(Grid g, const double* __restrict__ rho,
                                                               const double* __restrict__ u,
                                                               WalshK wk, double penal, double dE,
                                                               double* __restrict__ dc) {
  for (int64_t e = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; e < g.nelem;
       e += (int64_t)gridDim.x * FE_BLOCK) {
    const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((int64_t)g.nx * g.ny));
    double t[3][8];
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int64_t n = (i + c_cx[a]) + (int64_t)(g.nx + 1) * ((j + c_cy[a]) + (int64_t)(g.ny + 1) * (k + c_cz[a]));
      t[0][a] = u[3 * n];
      t[1][a] = u[3 * n + 1];
      t[2][a] = u[3 * n + 2];
    }
    walsh8(t[0]);
    walsh8(t[1]);
    walsh8(t[2]);
    enum { X = 0, Y = 1, Z = 2 };
    // modes: 1=100 2=110 3=010 4=001 5=101 6=111 7=011
    double en = 0.0;
    // linear modes, normal block
    const double n1 = t[X][1], n2 = t[Y][3], n3 = t[Z][4];
    en += wk.A * (n1 * n1 + n2 * n2 + n3 * n3) + 2.0 * wk.B * (n1 * n2 + n1 * n3 + n2 * n3);
    // shear pairs (rank one)
    const double s1 = t[Y][1] + t[X][3], s2 = t[Z][1] + t[X][4], s3 = t[Z][3] + t[Y][4];
    en += wk.G * (s1 * s1 + s2 * s2 + s3 * s3);
    // bilinear pairs
    en += wk.C * (t[X][2] * t[X][2] + t[Z][7] * t[Z][7]) + 2.0 * wk.D * t[X][2] * t[Z][7];
    en += wk.C * (t[Y][2] * t[Y][2] + t[Z][5] * t[Z][5]) + 2.0 * wk.D * t[Y][2] * t[Z][5];
    en += wk.C * (t[X][5] * t[X][5] + t[Y][7] * t[Y][7]) + 2.0 * wk.D * t[X][5] * t[Y][7];
    // bilinear triple
    const double a3 = t[Z][2], b3 = t[Y][5], c3 = t[X][7];
    en += wk.F * (a3 * a3 + b3 * b3 + c3 * c3) + 2.0 * wk.H * (a3 * b3 + a3 * c3 + b3 * c3);
    // trilinear mode
    en += wk.J * (t[X][6] * t[X][6] + t[Y][6] * t[Y][6] + t[Z][6] * t[Z][6]);
    const double r = rho[e];
    dc[e] = -penal * pow(r, penal - 1.0) * dE * en;
  }
}

// The state-equation term of the general adjoint gradient:
// out_e = -p rho^(p-1) (E0 - Emin) lam_e^T Ke u_e, the symmetric bilinear form
// of the factorised Ke (the quadratic form above with one operand from u and
// one from lam, each cross term taken in both orders).
__device__ inline void load_walsh(const Grid& g, const double* __restrict__ v, int i, int j, int k,
                                  double (&t)[3][8]) {
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int64_t n = (i + c_cx[a]) + (int64_t)(g.nx + 1) * ((j + c_cy[a]) + (int64_t)(g.ny + 1) * (k + c_cz[a]));
    t[0][a] = v[3 * n];
    t[1][a] = v[3 * n + 1];
    t[2][a] = v[3 * n + 2];
  }
  walsh8(t[0]);
  walsh8(t[1]);
  walsh8(t[2]);
}

__global__ void __launch_bounds__(FE_BLOCK) adjoint_sensitivity_kernel(Grid g, const double* __restrict__ rho,
                                                                       const double* __restrict__ u,
                                                                       const double* __restrict__ lam,
                                                                       WalshK wk, double penal, double dE,
                                                                       double* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; e < g.nelem;
       e += (int64_t)gridDim.x * FE_BLOCK) {
    const int i = (int)(e % g.nx), j = (int)((e / g.nx) % g.ny), k = (int)(e / ((int64_t)g.nx * g.ny));
    double t[3][8], s[3][8];
    load_walsh(g, u, i, j, k, t);
    load_walsh(g, lam, i, j, k, s);
    enum { X = 0, Y = 1, Z = 2 };
    double en = 0.0;
    // linear modes, normal block
    const double n1 = t[X][1], n2 = t[Y][3], n3 = t[Z][4];
    const double m1 = s[X][1], m2 = s[Y][3], m3 = s[Z][4];
    en += wk.A * (n1 * m1 + n2 * m2 + n3 * m3) +
          wk.B * (n1 * m2 + n2 * m1 + n1 * m3 + n3 * m1 + n2 * m3 + n3 * m2);
    // shear pairs (rank one)
    en += wk.G * ((t[Y][1] + t[X][3]) * (s[Y][1] + s[X][3]) + (t[Z][1] + t[X][4]) * (s[Z][1] + s[X][4]) +
                  (t[Z][3] + t[Y][4]) * (s[Z][3] + s[Y][4]));
    // bilinear pairs
    en += wk.C * (t[X][2] * s[X][2] + t[Z][7] * s[Z][7]) + wk.D * (t[X][2] * s[Z][7] + t[Z][7] * s[X][2]);
    en += wk.C * (t[Y][2] * s[Y][2] + t[Z][5] * s[Z][5]) + wk.D * (t[Y][2] * s[Z][5] + t[Z][5] * s[Y][2]);
    en += wk.C * (t[X][5] * s[X][5] + t[Y][7] * s[Y][7]) + wk.D * (t[X][5] * s[Y][7] + t[Y][7] * s[X][5]);
    // bilinear triple
    const double a3 = t[Z][2], b3 = t[Y][5], c3 = t[X][7];
    const double a4 = s[Z][2], b4 = s[Y][5], c4 = s[X][7];
    en += wk.F * (a3 * a4 + b3 * b4 + c3 * c4) + wk.H * (a3 * b4 + b3 * a4 + a3 * c4 + c3 * a4 + b3 * c4 + c3 * b4);
    // trilinear mode
    en += wk.J * (t[X][6] * s[X][6] + t[Y][6] * s[Y][6] + t[Z][6] * s[Z][6]);
    out[e] = -penal * pow(rho[e], penal - 1.0) * dE * en;
  }
}

// ------------------------------------------------------------ filter
// Density filter by LDS tiles.  A workgroup of 8 x 8 x tz threads owns an
// 8 x 8 x tz brick of elements; it copies the brick and a halo of H elements
// (the stencil's reach; zero outside the mesh, which truncates the cone at
// the boundary) into LDS, then each thread sums the stencil over LDS.  The
// stencil is a table of LDS offsets and cone weights r - |d| (only d with
// positive weight, z slowest), built on the host for the tile shape; entry q
// goes to partial sum q mod 8 (eight LDS reads in flight), and the partial
// sums are added pairwise in a fixed order.  Modes:
//   0  out = P in:    out_i = invW_i sum_j w_ij in_j
//   1  out = P^T in:  out_j = sum_i w_ij invW_i in_i
//   2  out = invW:    1 / sum_j w_ij (row sums of the truncated cone)
struct FilterTile {
  int n;            // stencil entries
  const int* lin;   // LDS offset of each entry
  const double* w;  // its weight
  int H, tz;        // halo, brick depth
  int tbx, tby;     // bricks along x, y
};

template <int MODE>
__global__ void __launch_bounds__(256) filter_tile_kernel(Grid g, FilterTile ft, const double* __restrict__ invW,
                                                          const double* __restrict__ in,
                                                          double* __restrict__ out) {
  extern __shared__ double tile[];
  const int LX = 8 + 2 * ft.H, LY = LX, LZ = ft.tz + 2 * ft.H;
  const int bx = blockIdx.x % ft.tbx, t1 = blockIdx.x / ft.tbx;
  const int by = t1 % ft.tby, bz = t1 / ft.tby;
  const int i0 = bx * 8 - ft.H, j0 = by * 8 - ft.H, k0 = bz * ft.tz - ft.H;
  const int nthr = 64 * ft.tz;
  const int tid = threadIdx.x + 8 * (threadIdx.y + 8 * threadIdx.z);
  for (int t = tid; t < LX * LY * LZ; t += nthr) {
    const int li = t % LX, lj = (t / LX) % LY, lk = t / (LX * LY);
    const int i = i0 + li, j = j0 + lj, k = k0 + lk;
    double v = 0.0;
    if (i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz) {
      const int64_t f = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
      v = MODE == 0 ? in[f] : MODE == 1 ? invW[f] * in[f] : 1.0;
    }
    tile[t] = v;
  }
  __syncthreads();
  const int i = bx * 8 + (int)threadIdx.x, j = by * 8 + (int)threadIdx.y, k = bz * ft.tz + (int)threadIdx.z;
  if (i >= g.nx || j >= g.ny || k >= g.nz) return;
  const double* c = tile + ((threadIdx.z + ft.H) * LY + threadIdx.y + ft.H) * LX + threadIdx.x + ft.H;
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int q = 0;
  for (; q + 8 <= ft.n; q += 8) {
#pragma unroll
    for (int m = 0; m < 8; ++m) a[m] += ft.w[q + m] * c[ft.lin[q + m]];
  }
  for (int m = 0; q < ft.n; ++q, ++m) a[m] += ft.w[q] * c[ft.lin[q]];
  const double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  const int64_t e = i + (int64_t)g.nx * (j + (int64_t)g.ny * k);
  out[e] = MODE == 0 ? acc * invW[e] : MODE == 1 ? acc : 1.0 / acc;
}

// ------------------------------------------------------------------ OC
// In s = 1/sqrt(lambda) the update is x_new = clamp(a s, lo, hi) with
// a = x sqrt(max(0, -dcx) / dv); the volume sum(dv x_new) is continuous and
// non-decreasing in s.  Each pass evaluates the volume at OC_NC points inside
// the current bracket [s_lo, s_hi] and keeps the sub-interval that contains
// the target, until the bracket on lambda is relatively 1e-12 wide (the
// oracle's bisection tolerance).  A target above the largest reachable
// volume leaves s = s_hi (every element with a > 0 at its upper bound).
#define OC_NC 64
struct OcState {
  double s_lo, s_hi, target, lam;
  int32_t done, pass, pad0, pad1;
};

__device__ inline void oc_elem(const double* x, const double* dcx, const double* dv, int64_t e,
                               double move, double& a, double& lo, double& hi, double& w) {
  const double xe = x[e];
  w = dv[e];
  a = xe * sqrt(fmax(0.0, -dcx[e]) / w);
  lo = fmax(0.0, xe - move);
  hi = fmin(1.0, xe + move);
}

__global__ void __launch_bounds__(FE_BLOCK) oc_prep_kernel(int64_t n, const double* __restrict__ x,
                                                           const double* __restrict__ dcx,
                                                           const double* __restrict__ dv, double move,
                                                           double* partials) {
  // s_max: beyond it every element with a > 0 sits at hi.
  double smax = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * FE_BLOCK) {
    double a, lo, hi, w;
    oc_elem(x, dcx, dv, e, move, a, lo, hi, w);
    // a can be subnormal for long-void elements: keep the bound finite (such
    // elements reach their upper bound only beyond s = 1e300)
    if (a > 0.0) smax = fmax(smax, fmin(hi / a, 1e300));
  }
  block_partial_max(smax, partials);
}

__global__ void __launch_bounds__(FE_BLOCK) oc_prep_finalize(int nb, const double* __restrict__ partials,
                                                             double target, OcState* os) {
  const double smax = reduce_partials_max(partials, nb);
  if (threadIdx.x == 0) {
    os->s_lo = 0.0;
    os->s_hi = smax * (1.0 + 1e-15);
    os->target = target;
    os->pass = 0;
    // no element with a > 0: every element sits at its lower bound for any s
    os->done = smax > 0.0 ? 0 : 1;
  }
}

// Candidate c of the current bracket [s_lo, s_hi].  While s_lo = 0 they step
// down from s_hi by factors of 2^16 (the volume is flat below the smallest
// a-scale, which can be 1e-300 for void elements, so the multiplier may lie
// many decades below s_hi); while s_hi / s_lo is large they are spaced
// geometrically, and once the bracket is narrow, evenly.
__device__ inline double oc_candidate(const OcState* os, int c) {
  const double lo = os->s_lo, hi = os->s_hi;
  if (lo == 0.0) return hi * exp2(-16.0 * (double)(OC_NC - c));
  if (hi > 1.5 * lo) return lo * exp2(log2(hi / lo) * (double)(c + 1) / (double)(OC_NC + 1));
  return lo + (hi - lo) * (double)(c + 1) / (double)(OC_NC + 1);
}

// One pass over the elements evaluates the volume at the OC_NC candidates.
// Over the candidate range [s_0, s_last] an element is either pinned at lo or
// at hi (contributing a constant), free (contributing w a s, linear in s), or
// crosses a bound inside the range; only the last kind is evaluated candidate
// by candidate.  Those elements are packed into LDS, where the lane of
// candidate c in each wave sums them in element order.  Once the bracket is
// narrow few elements cross a bound and a pass costs one read of x, dc, dv.
__global__ void __launch_bounds__(FE_BLOCK) oc_pass_kernel(int64_t n, const double* __restrict__ x,
                                                           const double* __restrict__ dcx,
                                                           const double* __restrict__ dv, double move,
                                                           const OcState* os, double* partials) {
  if (os->done) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int cand = tid & (OC_NC - 1);
  const int sub = tid / OC_NC;  // 0..3
  const double sc = oc_candidate(os, cand);
  const double s_first = oc_candidate(os, 0), s_last = oc_candidate(os, OC_NC - 1);
  __shared__ double sa[FE_BLOCK], slo[FE_BLOCK], shi[FE_BLOCK], sw[FE_BLOCK];
  __shared__ int wcount[FE_BLOCK / 64];
  double cst = 0.0, lin = 0.0, vol = 0.0;
  for (int64_t base = blockIdx.x * (int64_t)FE_BLOCK; base < n; base += (int64_t)gridDim.x * FE_BLOCK) {
    const int64_t e = base + tid;
    bool cross = false;
    double a = 0.0, lo = 0.0, hi = 0.0, w = 0.0;
    if (e < n) {
      oc_elem(x, dcx, dv, e, move, a, lo, hi, w);
      const double v0 = a * s_first, v1 = a * s_last;
      if (v1 <= lo)
        cst += w * fmin(lo, hi);
      else if (v0 >= hi)
        cst += w * hi;
      else if (v0 >= lo && v1 <= hi)
        lin += w * a;
      else
        cross = true;
    }
    const uint64_t m = __ballot(cross);
    if (lane == 0) wcount[wv] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
    for (int k = 0; k < FE_BLOCK / 64; ++k) {
      const int c = wcount[k];
      off += k < wv ? c : 0;
      tot += c;
    }
    if (cross) {
      const int pos = off + __popcll(m & ((1ull << lane) - 1ull));
      sa[pos] = a;
      slo[pos] = lo;
      shi[pos] = hi;
      sw[pos] = w;
    }
    __syncthreads();
    for (int q = sub; q < tot; q += FE_BLOCK / OC_NC) vol += sw[q] * fmin(fmax(sa[q] * sc, slo[q]), shi[q]);
    __syncthreads();
  }
  // block sums of the constant and linear parts (fixed tree), and of the four
  // sub-sums of each candidate (fixed order)
  __shared__ double part[FE_BLOCK], pc[FE_BLOCK], pl[FE_BLOCK];
  part[tid] = vol;
  pc[tid] = cst;
  pl[tid] = lin;
  __syncthreads();
  for (int h = FE_BLOCK / 2; h > 0; h >>= 1) {
    if (tid < h) {
      pc[tid] += pc[tid + h];
      pl[tid] += pl[tid + h];
    }
    __syncthreads();
  }
  if (tid < OC_NC) {
    double s = 0.0;
    for (int q = 0; q < FE_BLOCK / OC_NC; ++q) s += part[q * OC_NC + tid];
    partials[(size_t)blockIdx.x * OC_NC + tid] = (pc[0] + pl[0] * sc) + s;
  }
}

// Sums the per-workgroup partials of a pass: thread (c, q) adds those of
// candidate c from every OC_FIN_Q-th workgroup starting at q, in workgroup
// order, its loads issued OC_FIN_BATCH at a time; the OC_FIN_Q sums are then
// added in q order (a fixed order throughout).
#define OC_FIN_Q 16
#define OC_FIN_BATCH 16
__global__ void __launch_bounds__(OC_NC * OC_FIN_Q) oc_pass_finalize(int nb, const double* __restrict__ partials,
                                                                    OcState* os) {
  if (os->done) return;
  const int c = threadIdx.x % OC_NC, q = threadIdx.x / OC_NC;
  double s = 0.0;
  int b = q;
  for (; b + (OC_FIN_BATCH - 1) * OC_FIN_Q < nb; b += OC_FIN_BATCH * OC_FIN_Q) {
    double v[OC_FIN_BATCH];
#pragma unroll
    for (int k = 0; k < OC_FIN_BATCH; ++k) v[k] = partials[(size_t)(b + k * OC_FIN_Q) * OC_NC + c];
#pragma unroll
    for (int k = 0; k < OC_FIN_BATCH; ++k) s += v[k];
  }
  for (; b < nb; b += OC_FIN_Q) s += partials[(size_t)b * OC_NC + c];
  __shared__ double part[OC_NC * OC_FIN_Q];
  __shared__ double vols[OC_NC];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < OC_NC) {
    double v = 0.0;
    for (int k = 0; k < OC_FIN_Q; ++k) v += part[k * OC_NC + threadIdx.x];
    vols[threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // first candidate whose volume reaches the target
    int k = 0;
    while (k < OC_NC && vols[k] < os->target) ++k;
    const double lo_new = (k == 0) ? os->s_lo : oc_candidate(os, k - 1);
    const double hi_new = (k == OC_NC) ? os->s_hi : oc_candidate(os, k);
    os->s_lo = lo_new;
    os->s_hi = hi_new;
    os->pass += 1;
    // bracket on lambda = 1/s^2 relatively 1e-12 wide  <=>  on s about 5e-13
    if (hi_new - lo_new <= 5e-13 * (hi_new + lo_new)) os->done = 1;
  }
}

__global__ void __launch_bounds__(FE_BLOCK) oc_final_kernel(int64_t n, const double* x,
                                                            const double* __restrict__ dcx,
                                                            const double* __restrict__ dv, double move,
                                                            const OcState* os, double* x_new,
                                                            double* partials) {
  const double s = 0.5 * (os->s_lo + os->s_hi);
  double ch = 0.0;
  for (int64_t e = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * FE_BLOCK) {
    double a, lo, hi, w;
    oc_elem(x, dcx, dv, e, move, a, lo, hi, w);
    const double xo = x[e];
    const double xn = fmin(fmax(a * s, lo), hi);
    x_new[e] = xn;
    ch = fmax(ch, fabs(xn - xo));
  }
  block_partial_max(ch, partials);
}

__global__ void __launch_bounds__(FE_BLOCK) oc_final_finalize(int nb, const double* __restrict__ partials,
                                                              OcState* os, double* change) {
  const double ch = reduce_partials_max(partials, nb);
  if (threadIdx.x == 0) {
    const double s = 0.5 * (os->s_lo + os->s_hi);
    os->lam = 1.0 / (s * s);
    if (change) *change = ch;
  }
}

// ------------------------------------------------------------ two-scale
// Block means of the design variables: one thread per coarse element sums
// the nb^3 fine elements of its block (z level slowest, x fastest) and
// divides by nb^3.
__global__ void __launch_bounds__(FE_BLOCK) block_mean_kernel(int nx, int ny, int nb, int cx, int cy, int64_t nc,
                                                              const double* __restrict__ z,
                                                              double* __restrict__ zc) {
  const double cnt = (double)nb * (double)nb * (double)nb;
  for (int64_t ec = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; ec < nc; ec += (int64_t)gridDim.x * FE_BLOCK) {
    const int64_t I = ec % cx, t = ec / cx;
    const int64_t J = t % cy, K = t / cy;
    double s = 0.0;
    for (int c = 0; c < nb; ++c)
      for (int b = 0; b < nb; ++b) {
        const double* row = z + nb * I + (int64_t)nx * (nb * J + b + (int64_t)ny * (nb * K + c));
        for (int a = 0; a < nb; ++a) s += row[a];
      }
    zc[ec] = s / cnt;
  }
}

}  // namespace

// =================================================================== launchers
static inline Grid G(fe_problem* p, int lev) { return p->L[lev].g; }

hipError_t launch_simp(fe_problem* p, int lev, const double* rho) {
  const Grid g = G(p, lev);
  hipLaunchKernelGGL(simp_kernel<double>, dim3(red_grid(g.nelem) * 4), dim3(FE_BLOCK), 0, p->stream, rho,
                     g.nelem, p->cfg.E0, p->cfg.Emin, p->cfg.penal, p->L[lev].E64, p->L[lev].E32);
  return hipGetLastError();
}

hipError_t launch_coarsen_modulus(fe_problem* p, int lev) {
  hipLaunchKernelGGL(coarsen_modulus_kernel, dim3(red_grid(G(p, lev).nelem) * 4), dim3(FE_BLOCK), 0,
                     p->stream, G(p, lev - 1), G(p, lev), p->L[lev - 1].E64, p->L[lev].E64, p->L[lev].E32);
  return hipGetLastError();
}

hipError_t launch_diag(fe_problem* p, int lev) {
  const Grid g = G(p, lev);
  hipLaunchKernelGGL(diag_kernel, dim3(red_grid(g.nnode) * 4), dim3(FE_BLOCK), 0, p->stream, g,
                     p->L[lev].E64, p->ke_diag * p->L[lev].h, p->L[lev].invd64, p->L[lev].invd32);
  return hipGetLastError();
}

hipError_t launch_node_mask(fe_problem* p, const uint8_t* fixed) {
  const Grid g = G(p, 0);
  hipLaunchKernelGGL(node_mask_kernel, dim3(red_grid(g.nnode) * 4), dim3(FE_BLOCK), 0, p->stream, g,
                     fixed, p->L[0].nmask);
  return hipGetLastError();
}

hipError_t launch_coarsen_mask(fe_problem* p, int lev) {
  hipLaunchKernelGGL(coarsen_mask_kernel, dim3(red_grid(G(p, lev).nnode) * 4), dim3(FE_BLOCK), 0,
                     p->stream, G(p, lev - 1), G(p, lev), p->L[lev - 1].nmask, p->L[lev].nmask);
  return hipGetLastError();
}

hipError_t launch_mask_load(fe_problem* p, const double* f) {
  const Grid g = G(p, 0);
  hipLaunchKernelGGL(mask_load_kernel, dim3(red_grid(g.ndof) * 4), dim3(FE_BLOCK), 0, p->stream, g, f,
                     p->L[0].nmask, p->f);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mask_vec(fe_problem* p, int lev, T* v) {
  const Grid g = G(p, lev);
  hipLaunchKernelGGL(mask_vec_kernel<T>, dim3(red_grid(g.ndof) * 4), dim3(FE_BLOCK), 0, p->stream, g,
                     p->L[lev].nmask, v);
  return hipGetLastError();
}
template hipError_t launch_mask_vec<double>(fe_problem*, int, double*);
template hipError_t launch_mask_vec<float>(fe_problem*, int, float*);

template <typename T>
static const T* level_E(fe_problem* p, int lev);
template <>
const double* level_E<double>(fe_problem* p, int lev) { return p->L[lev].E64; }
template <>
const float* level_E<float>(fe_problem* p, int lev) { return p->L[lev].E32; }
template <typename T>
static const T* level_invd(fe_problem* p, int lev);
template <>
const double* level_invd<double>(fe_problem* p, int lev) { return p->L[lev].invd64; }
template <>
const float* level_invd<float>(fe_problem* p, int lev) { return p->L[lev].invd32; }

// Streams once through the cold-cache buffer (one read and one write per
// word), so whatever the next launch reads comes from HBM: the buffer is
// larger than the 256 MB last-level cache and the 4 MB L2 of every XCD.
__global__ void cache_flush_kernel(uint32_t* __restrict__ buf, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < n; i += stride) {
    if (i + 4 <= n) {
      uint4 v = *reinterpret_cast<const uint4*>(buf + i);
      v.x += 1u;
      *reinterpret_cast<uint4*>(buf + i) = v;
    } else {
      for (int64_t k = i; k < n; ++k) buf[k] += 1u;
    }
  }
}

int kstats_begin(fe_problem* p, double bytes) {
  KStats& ks = p->kst;
  if (!ks.on) return -1;
  if (ks.flush && ks.flush_words) {
    hipLaunchKernelGGL(cache_flush_kernel, dim3(8192), dim3(256), 0, p->stream, ks.flush,
                       (int64_t)ks.flush_words);
  }
  if (ks.cap_ev) {  // inside a graph capture: the graph owns the pair
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return -1;
    }
    ks.cap_ev->push_back(a);
    ks.cap_ev->push_back(b);
    ks.cap_bytes->push_back(bytes);
    // external: captured as an event-record node that records on every replay
    (void)hipEventRecordWithFlags(a, p->stream, hipEventRecordExternal);
    return (int)ks.cap_bytes->size() - 1;
  }
  const size_t slot = (size_t)ks.pending;
  if (2 * slot + 2 > ks.ev.size()) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      return -1;
    }
    ks.ev.push_back(a);
    ks.ev.push_back(b);
  }
  if (slot + 1 > ks.bytes.size()) ks.bytes.resize(slot + 1);
  ks.bytes[slot] = bytes;
  (void)hipEventRecord(ks.ev[2 * slot], p->stream);
  return (int)slot;
}

void kstats_end(fe_problem* p, int slot) {
  if (slot < 0) return;
  KStats& ks = p->kst;
  if (ks.cap_ev) {
    (void)hipEventRecordWithFlags((*ks.cap_ev)[2 * (size_t)slot + 1], p->stream, hipEventRecordExternal);
    return;
  }
  (void)hipEventRecord(ks.ev[2 * (size_t)slot + 1], p->stream);
  ks.pending += 1;
}

template <typename T>
hipError_t launch_kxu(fe_problem* p, int lev, const T* x, T* y, CgState* st) {
  return launch_kxu_tile<T>(p, lev, x, level_E<T>(p, lev), y, st, st ? 1 : 0, nullptr, nullptr);
}
template hipError_t launch_kxu<double>(fe_problem*, int, const double*, double*, CgState*);
template hipError_t launch_kxu<float>(fe_problem*, int, const float*, float*, CgState*);

hipError_t launch_residual64(fe_problem* p, const double* u, double* r, double* scal_slot) {
  return launch_kxu_tile<double>(p, 0, u, p->L[0].E64, r, nullptr, 2, p->f, scal_slot);
}

hipError_t launch_kxu_dense64(fe_problem* p, const double* x, double* y) {
  const Grid g = G(p, 0);
  const int nb = (int)ceil_div(g.nnode, FE_BLOCK);
  hipLaunchKernelGGL(kxu_dense_kernel, dim3(nb), dim3(FE_BLOCK), 0, p->stream, g, x, p->L[0].E64,
                     p->L[0].nmask, p->ke64, p->L[0].h, y);
  return hipGetLastError();
}

hipError_t launch_cg_finalize(fe_problem* p, int op, int nb, int mg, CgState* st, double* out) {
  hipLaunchKernelGGL(cg_finalize_kernel, dim3(1), dim3(FE_BLOCK), 0, p->stream, op, nb, mg, p->partials, st,
                     out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_init(fe_problem* p, const T* b, const T* Kx, T* r, T* pvec, CgState* st, int mg) {
  const Grid g = G(p, 0);
  const int nb = red_grid(g.ndof);
  hipLaunchKernelGGL(cg_init_kernel<T>, dim3(nb), dim3(FE_BLOCK), 0, p->stream, g, b, Kx, r, pvec,
                     level_invd<T>(p, 0), p->partials, mg);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_cg_finalize(p, FIN_INIT, nb, mg, st, nullptr);
}
template hipError_t launch_cg_init<double>(fe_problem*, const double*, const double*, double*, double*,
                                           CgState*, int);
template hipError_t launch_cg_init<float>(fe_problem*, const float*, const float*, float*, float*,
                                          CgState*, int);

template <typename T>
hipError_t launch_cg_update(fe_problem* p, T* x, T* r, const T* pvec, const T* q, CgState* st, int mg) {
  const Grid g = G(p, 0);
  const int nb = red_grid(g.ndof);
  hipLaunchKernelGGL(cg_update_kernel<T>, dim3(nb), dim3(FE_BLOCK), 0, p->stream, g, x, r, pvec, q,
                     level_invd<T>(p, 0), st, p->partials, mg);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_cg_finalize(p, FIN_UPDATE, nb, mg, st, nullptr);
}
template hipError_t launch_cg_update<double>(fe_problem*, double*, double*, const double*, const double*,
                                             CgState*, int);
template hipError_t launch_cg_update<float>(fe_problem*, float*, float*, const float*, const float*,
                                            CgState*, int);

// few workgroups: the next kernel's every workgroup sums these partials
constexpr int kUpdateMgGrid = 1024;

template <typename T>
hipError_t launch_cg_update_mg(fe_problem* p, T* x, T* r, const T* pvec, const T* q, CgState* st, int npq,
                               int* nrr, float* r32, const T* pold) {
  if (x && !pold) return hipErrorInvalidValue;  // applying the deferred step needs its direction
  const Grid g = G(p, 0);
  int nb = red_grid(g.ndof);
  if (nb > kUpdateMgGrid) nb = kUpdateMgGrid;
  hipLaunchKernelGGL(cg_update_mg_kernel<T>, dim3(nb, p->bcount), dim3(FE_BLOCK), 0, p->stream, g, x, r, pvec, q,
                     st, part_region(p, PART_PQ), npq, part_region(p, PART_RR),
                     p->bcount > 1 ? p->bstride : (int64_t)0, r32, pold);
  *nrr = nb;
  return hipGetLastError();
}
template hipError_t launch_cg_update_mg<double>(fe_problem*, double*, double*, const double*, const double*,
                                                CgState*, int, int*, float*, const double*);
template hipError_t launch_cg_update_mg<float>(fe_problem*, float*, float*, const float*, const float*,
                                               CgState*, int, int*, float*, const float*);

template <typename T>
hipError_t launch_cg_flush_x(fe_problem* p, T* x, const CgState* st) {
  const int64_t n = G(p, 0).ndof;
  hipLaunchKernelGGL(cg_flush_x_kernel<T>, dim3(red_grid(n) * 2), dim3(FE_BLOCK), 0, p->stream, n, x, st);
  return hipGetLastError();
}
template hipError_t launch_cg_flush_x<double>(fe_problem*, double*, const CgState*);
template hipError_t launch_cg_flush_x<float>(fe_problem*, float*, const CgState*);

hipError_t launch_narrow(fe_problem* p, const double* a, float* b) {
  const int64_t n = G(p, 0).ndof;
  hipLaunchKernelGGL(narrow_kernel, dim3(red_grid(n) * 2, p->bcount), dim3(FE_BLOCK), 0, p->stream, n, a, b,
                     p->bcount > 1 ? p->bstride : (int64_t)0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_direction(fe_problem* p, const T* r, const T* z, T* pvec, CgState* st) {
  const Grid g = G(p, 0);
  hipLaunchKernelGGL(cg_direction_kernel<T>, dim3(red_grid(g.ndof) * 2), dim3(FE_BLOCK), 0, p->stream, g,
                     r, z, level_invd<T>(p, 0), pvec, st);
  return hipGetLastError();
}
template hipError_t launch_cg_direction<double>(fe_problem*, const double*, const double*, double*,
                                                CgState*);
template hipError_t launch_cg_direction<float>(fe_problem*, const float*, const float*, float*, CgState*);

hipError_t launch_cg_state_resume(fe_problem* p, CgState* st, double tol2, int max_iter) {
  hipLaunchKernelGGL(cg_state_resume_kernel, dim3(1), dim3(64), 0, p->stream, st, tol2, max_iter);
  return hipGetLastError();
}

hipError_t launch_cg_guard(fe_problem* p, CgState* g, int done) {
  hipLaunchKernelGGL(cg_guard_kernel, dim3(1, p->bcount), dim3(64), 0, p->stream, g, done,
                     p->bcount > 1 ? p->bstride : (int64_t)0);
  return hipGetLastError();
}

hipError_t launch_cg_state_init(fe_problem* p, CgState* st, double tol_rel, int max_iter) {
  hipLaunchKernelGGL(cg_state_init_kernel, dim3(1), dim3(64), 0, p->stream, st, tol_rel, max_iter);
  return hipGetLastError();
}

hipError_t launch_to32_scaled(fe_problem* p, const double* r64, float* r32, const double* nrm2) {
  const int64_t n = G(p, 0).ndof;
  hipLaunchKernelGGL(to32_scaled_kernel, dim3(red_grid(n) * 2), dim3(FE_BLOCK), 0, p->stream, n, r64, r32,
                     nrm2);
  return hipGetLastError();
}

hipError_t launch_axpy_from32(fe_problem* p, double* u, const float* d, const double* nrm2) {
  const int64_t n = G(p, 0).ndof;
  hipLaunchKernelGGL(axpy_from32_kernel, dim3(red_grid(n) * 2), dim3(FE_BLOCK), 0, p->stream, n, u, d,
                     nrm2);
  return hipGetLastError();
}

hipError_t launch_dot64(fe_problem* p, const double* a, const double* b, int64_t n, double* out) {
  const int nb = red_grid(n);
  hipLaunchKernelGGL(dot64_kernel, dim3(nb), dim3(FE_BLOCK), 0, p->stream, n, a, b, p->partials, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_cg_finalize(p, FIN_SCALAR, nb, 0, nullptr, out);
}

template <typename T>
hipError_t launch_fill(fe_problem* p, T* v, int64_t n, T val) {
  hipLaunchKernelGGL(fill_kernel<T>, dim3(red_grid(n) * 2), dim3(FE_BLOCK), 0, p->stream, n, v, val);
  return hipGetLastError();
}
template hipError_t launch_fill<double>(fe_problem*, double*, int64_t, double);
template hipError_t launch_fill<float>(fe_problem*, float*, int64_t, float);

hipError_t launch_convert_64_32(fe_problem* p, const double* a, float* b, int64_t n) {
  hipLaunchKernelGGL((convert_kernel<double, float>), dim3(red_grid(n) * 2), dim3(FE_BLOCK), 0, p->stream,
                     n, a, b);
  return hipGetLastError();
}

hipError_t launch_convert_32_64(fe_problem* p, const float* a, double* b, int64_t n) {
  hipLaunchKernelGGL((convert_kernel<float, double>), dim3(red_grid(n) * 2), dim3(FE_BLOCK), 0, p->stream,
                     n, a, b);
  return hipGetLastError();
}

hipError_t launch_sensitivity(fe_problem* p, const double* rho, const double* u, double* dc) {
  const Grid g = G(p, 0);
  WalshK wk = p->wk;
  const double h = p->L[0].h;
  wk.A *= h; wk.B *= h; wk.G *= h; wk.C *= h; wk.D *= h; wk.F *= h; wk.H *= h; wk.J *= h;
  hipLaunchKernelGGL(sensitivity_kernel, dim3(red_grid(g.nelem) * 4), dim3(FE_BLOCK), 0, p->stream, g, rho,
                     u, wk, p->cfg.penal, p->cfg.E0 - p->cfg.Emin, dc);
  return hipGetLastError();
}

hipError_t launch_adjoint_sensitivity(fe_problem* p, const double* rho, const double* u, const double* lam,
                                      double* out) {
  const Grid g = G(p, 0);
  WalshK wk = p->wk;
  const double h = p->L[0].h;
  wk.A *= h; wk.B *= h; wk.G *= h; wk.C *= h; wk.D *= h; wk.F *= h; wk.H *= h; wk.J *= h;
  hipLaunchKernelGGL(adjoint_sensitivity_kernel, dim3(red_grid(g.nelem) * 4), dim3(FE_BLOCK), 0, p->stream, g,
                     rho, u, lam, wk, p->cfg.penal, p->cfg.E0 - p->cfg.Emin, out);
  return hipGetLastError();
}

template <int MODE>
static hipError_t launch_filter_tile(fe_problem* p, const double* in, double* out) {
  const Grid g = G(p, 0);
  FilterTile ft;
  ft.n = p->nstencil;
  ft.lin = p->st_lin;
  ft.w = p->st_w;
  ft.H = p->st_halo;
  ft.tz = p->st_tz;
  ft.tbx = (g.nx + 7) / 8;
  ft.tby = (g.ny + 7) / 8;
  const int tbz = (g.nz + ft.tz - 1) / ft.tz;
  const int L = 8 + 2 * ft.H;
  const size_t lds = (size_t)L * L * (ft.tz + 2 * ft.H) * sizeof(double);
  hipLaunchKernelGGL(filter_tile_kernel<MODE>, dim3(ft.tbx * ft.tby * tbz), dim3(8, 8, ft.tz), lds, p->stream, g, ft,
                     p->invW, in, out);
  return hipGetLastError();
}

hipError_t launch_filter_rowsums(fe_problem* p) { return launch_filter_tile<2>(p, nullptr, p->invW); }

hipError_t launch_filter(fe_problem* p, const double* in, double* out, int transpose) {
  return transpose ? launch_filter_tile<1>(p, in, out) : launch_filter_tile<0>(p, in, out);
}

// u <- u + theta (u - hist) and hist <- the old u, per dof
__global__ void __launch_bounds__(FE_BLOCK) extrapolate_kernel(int64_t n, double* __restrict__ u,
                                                               double* __restrict__ hist, double theta) {
  for (int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x; d < n; d += (int64_t)gridDim.x * FE_BLOCK) {
    const double v = u[d];
    u[d] = v + theta * (v - hist[d]);
    hist[d] = v;
  }
}

hipError_t launch_extrapolate(fe_problem* p, double* u, double* hist, double theta) {
  const int64_t n = G(p, 0).ndof;
  hipLaunchKernelGGL(extrapolate_kernel, dim3(red_grid(n) * 2), dim3(FE_BLOCK), 0, p->stream, n, u, hist, theta);
  return hipGetLastError();
}

hipError_t launch_block_mean(fe_problem* p, const double* z, int nb, double* zc) {
  const Grid g = G(p, 0);
  const int cx = g.nx / nb, cy = g.ny / nb;
  const int64_t nc = (int64_t)cx * cy * (g.nz / nb);
  hipLaunchKernelGGL(block_mean_kernel, dim3(red_grid(nc) * 4), dim3(FE_BLOCK), 0, p->stream, g.nx, g.ny, nb, cx,
                     cy, nc, z, zc);
  return hipGetLastError();
}

namespace {

// The OC launch sequence on a given stream with the given scratch: partials
// holds at least FE_OC_PARTIALS doubles (the block partials of the prep and
// final passes, then 64 per workgroup of the candidate passes; they are
// used one launch pair at a time), os one OcState.  Every partial and every
// field of os is written before it is read, so the scratch needs no clearing.
hipError_t launch_oc_on(hipStream_t stream, double* partials, OcState* os, int64_t n, const double* x,
                        const double* dcx, const double* dv, double volfrac, double move, double* x_new,
                        double* change) {
  const double target = volfrac * (double)n;
  const int nb = red_grid(n);
  // the candidate passes keep 64 partials per workgroup: at most 1024 workgroups
  const int nbp = nb < 1024 ? nb : 1024;
  hipLaunchKernelGGL(oc_prep_kernel, dim3(nb), dim3(FE_BLOCK), 0, stream, n, x, dcx, dv, move, partials);
  hipLaunchKernelGGL(oc_prep_finalize, dim3(1), dim3(FE_BLOCK), 0, stream, nb, partials, target, os);
  for (int pass = 0; pass < 24; ++pass) {  // passes after convergence return at once
    hipLaunchKernelGGL(oc_pass_kernel, dim3(nbp), dim3(FE_BLOCK), 0, stream, n, x, dcx, dv, move, os, partials);
    hipLaunchKernelGGL(oc_pass_finalize, dim3(1), dim3(OC_NC * OC_FIN_Q), 0, stream, nbp, partials, os);
  }
  hipLaunchKernelGGL(oc_final_kernel, dim3(nb), dim3(FE_BLOCK), 0, stream, n, x, dcx, dv, move, os, x_new,
                     partials);
  hipLaunchKernelGGL(oc_final_finalize, dim3(1), dim3(FE_BLOCK), 0, stream, nb, partials, os, change);
  return hipGetLastError();
}

// Scratch of the allocation-free OC entry point: FE_OC_PARTIALS partial sums
// followed by the search state.  Each GPU holds its own copy for the life of
// the process; host code reaches it only through the address
// hipGetSymbolAddress returns on that GPU (the array's name is a host-side
// stand-in, not a device address).
constexpr int64_t kOcScratchDoubles = FE_OC_PARTIALS + (int64_t)(sizeof(OcState) + 7) / 8;
static_assert(FE_OC_PARTIALS >= FE_RED_GRID && FE_OC_PARTIALS >= 1024 * OC_NC, "OC partials do not fit");
static __device__ __align__(256) double scratch[kOcScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of this GPU's scratch, looked up once per device with
// that device current (the caller's current device).
hipError_t oc_scratch_address(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

hipError_t launch_oc(fe_problem* p, const double* x, const double* dcx, const double* dv, double volfrac,
                     double move, double* x_new, double* change) {
  return launch_oc_on(p->stream, p->partials, reinterpret_cast<OcState*>(p->oc), G(p, 0).nelem, x, dcx, dv,
                      volfrac, move, x_new, change);
}

hipError_t launch_oc_noalloc(hipStream_t stream, int64_t n, const double* x, const double* dcx, const double* dv,
                             double volfrac, double move, double* x_new, double* change) {
  double* base = nullptr;
  const hipError_t e = oc_scratch_address(&base);
  if (e != hipSuccess) return e;
  return launch_oc_on(stream, base, reinterpret_cast<OcState*>(base + FE_OC_PARTIALS), n, x, dcx, dv, volfrac,
                      move, x_new, change);
}
