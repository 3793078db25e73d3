// Geometric multigrid pieces: grid transfers and the first Jacobi sweep.
//
// Level l+1 halves every grid dimension of level l (element edge doubles).
// Prolongation P is trilinear interpolation from coarse to fine nodes, with
// the rows and columns of fixed dofs removed; restriction is its transpose,
// which keeps the V-cycle symmetric so it can precondition CG.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "fe_internal.h"

namespace {

inline int64_t wsh_of(const fe_problem* p) { return p->bcount > 1 ? p->bstride : 0; }

inline int nblocks(int64_t n) {
  int64_t g = (n + FE_BLOCK - 1) / FE_BLOCK;
  return (int)(g < 1 ? 1 : g);
}

// Division of a node index by a fixed divisor as a multiply and a shift
// (Granlund and Montgomery, "Division by invariant integers using
// multiplication", 1994, Thm. 4.2 with 31-bit numerators): with 2^l >= d and
// m = floor(2^(31+l) / d) + 1 < 2^32, floor(n m / 2^(31+l)) = floor(n / d)
// for every 0 <= n < 2^31.  Node indices qualify: the set-up rejects grids of
// 2^31 / 3 nodes or more.  It replaces the 64-bit divisions (a long chain of
// vector instructions in front of every load) of the node-indexed transfers.
struct FastDiv {
  uint32_t d, m, s;
};
struct NodeDiv {
  FastDiv x, xy;  // by nx + 1 and (nx + 1) (ny + 1)
};

inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while (((uint64_t)1 << l) < d) ++l;
  FastDiv f;
  f.d = d;
  f.s = 31 + l;
  f.m = (uint32_t)((((uint64_t)1 << (31 + l)) / d) + 1);
  return f;
}

inline NodeDiv node_div(const Grid& g) {
  NodeDiv nd;
  nd.x = make_fastdiv((uint32_t)(g.nx + 1));
  nd.xy = make_fastdiv((uint32_t)((g.nx + 1) * (g.ny + 1)));
  return nd;
}

__device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f) { return (uint32_t)(((uint64_t)n * f.m) >> f.s); }

// (i, j, k) of node n < 2^31
__device__ inline void node_ijk(uint32_t n, const NodeDiv& nd, int& i, int& j, int& k) {
  const uint32_t kk = fdiv(n, nd.xy), rem = n - kk * nd.xy.d, jj = fdiv(rem, nd.x);
  i = (int)(rem - jj * nd.x.d);
  j = (int)jj;
  k = (int)kk;
}

// z = omega D^-1 r (the first sweep from z = 0; fixed dofs have r = 0).
// A non-null st guards every kernel of the cycle: nothing is stored once CG
// stopped.
template <typename T>
__global__ void __launch_bounds__(FE_BLOCK) jacobi0_kernel(int64_t ndof, const T* __restrict__ r,
                                                           const T* __restrict__ invd, T omega,
                                                           T* __restrict__ z, const CgState* st, int64_t wsh) {
  if (wsh) {  // batched launch: this workgroup's problem
    const int64_t o = batch_offset(wsh);
    r = wshift(r, o);
    invd = wshift(invd, o);
    z = wshift(z, o);
    st = wshift(st, o);
  }
  const int64_t d = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x;
  if (d >= ndof) return;
  const T v = omega * invd[d / 3] * r[d];
  if (st && st->done) return;  // read after the loads: no round trip in front of them
  z[d] = v;
}

// r_c = P^T t_f: coarse node (I,J,K) collects the fine nodes 2I+a, 2J+b, 2K+c
// (a, b, c in {-1, 0, 1}) with weight prod (a == 0 ? 1 : 1/2).
// The coarse level may hold a narrower type (TC) than the fine one (T): the
// sum is formed in T and rounded once.
template <typename T, typename TC = T>
__global__ void __launch_bounds__(FE_BLOCK) restrict_kernel(Grid fg, Grid cg, NodeDiv cd,
                                                            const T* __restrict__ tf,
                                                            const uint8_t* __restrict__ cmask,
                                                            TC* __restrict__ rc, const CgState* st, int64_t wsh,
                                                            const TC* __restrict__ invd_c, TC omega,
                                                            TC* __restrict__ d0) {
  if (wsh) {  // batched launch: this workgroup's problem
    const int64_t o = batch_offset(wsh);
    tf = wshift(tf, o);
    cmask = wshift(cmask, o);
    rc = wshift(rc, o);
    st = wshift(st, o);
    invd_c = wshift(invd_c, o);
    d0 = wshift(d0, o);
  }
  const int64_t n64 = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x;
  if (n64 >= cg.nnode) return;
  // node and dof indices fit 31 bits; signed, so that the three components'
  // loads of a node merge into one (no wrap-around between them)
  const int n = (int)n64;
  int I, J, K;
  node_ijk((uint32_t)n, cd, I, J, K);
  const int fsx = fg.nx + 1, fsxy = (fg.nx + 1) * (fg.ny + 1);
  // All 27 fine neighbours are loaded unconditionally (one off the mesh
  // reads a clamped node and gets weight 0), so the loads issue back to back
  // instead of one branch and one round trip each; a zero term leaves the
  // sum unchanged.
  T v[27][3], w[27];
#pragma unroll
  for (int c = -1; c <= 1; ++c) {
    const int k = 2 * K + c;
    const bool kin = k >= 0 && k <= fg.nz;
    const int kc = min(max(k, 0), fg.nz);
#pragma unroll
    for (int b = -1; b <= 1; ++b) {
      const int j = 2 * J + b;
      const bool jin = j >= 0 && j <= fg.ny;
      const int jc = min(max(j, 0), fg.ny);
#pragma unroll
      for (int a = -1; a <= 1; ++a) {
        const int i = 2 * I + a;
        const bool in = kin && jin && i >= 0 && i <= fg.nx;
        const int ic = min(max(i, 0), fg.nx);
        const int q = 9 * (c + 1) + 3 * (b + 1) + (a + 1);
        const int f = 3 * (ic + fsx * jc + fsxy * kc);
        w[q] = in ? (c ? T(0.5) : T(1)) * (b ? T(0.5) : T(1)) * (a ? T(0.5) : T(1)) : T(0);
        v[q][0] = tf[f];
        v[q][1] = tf[f + 1];
        v[q][2] = tf[f + 2];
      }
    }
  }
  T acc[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int q = 0; q < 27; ++q) {
    acc[0] += w[q] * v[q][0];
    acc[1] += w[q] * v[q][1];
    acc[2] += w[q] * v[q][2];
  }
  const uint8_t m = cmask[n];
  const TC dn = d0 ? invd_c[n] : TC(0);
  if (st && st->done) return;  // read after the loads: no round trip in front of them
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const TC v = ((m >> q) & 1) ? TC(0) : (TC)acc[q];
    rc[3 * n + q] = v;
    // the coarsest level's first Chebyshev direction omega D^-1 r, formed as
    // the separate first-direction launch forms it
    if (d0) d0[3 * n + q] = omega * dn * v;
  }
}

// out_f = z_f + P z_c (out may alias z: each thread touches only its own node).
// With rf given, z_f is the first Jacobi sweep from zero, formed here as
// (omega D^-1) r_f exactly as the launch that used it formed it, instead of
// being stored there and read back.
template <typename T, typename TC = T>
__global__ void __launch_bounds__(FE_BLOCK) prolong_add_kernel(Grid fg, Grid cg, NodeDiv fd, const T* zf,
                                                               const TC* __restrict__ zc,
                                                               const uint8_t* __restrict__ fmask, T* out,
                                                               const T* __restrict__ rf, const T* __restrict__ invd,
                                                               T omega, const CgState* st, int64_t wsh) {
  if (wsh) {  // batched launch: this workgroup's problem
    const int64_t o = batch_offset(wsh);
    zf = wshift(zf, o);
    zc = wshift(zc, o);
    fmask = wshift(fmask, o);
    out = wshift(out, o);
    rf = wshift(rf, o);
    invd = wshift(invd, o);
    st = wshift(st, o);
  }
  const int64_t n64 = blockIdx.x * (int64_t)FE_BLOCK + threadIdx.x;
  if (n64 >= fg.nnode) return;
  const int n = (int)n64;  // node and dof indices fit 31 bits (signed: merged loads)
  int i, j, k;
  node_ijk((uint32_t)n, fd, i, j, k);
  // coarse neighbours along each axis: one (even index) or two (odd index)
  const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1, k1 = (k + 1) >> 1;
  const T wi = (i & 1) ? T(0.5) : T(1), wj = (j & 1) ? T(0.5) : T(1), wk = (k & 1) ? T(0.5) : T(1);
  const int csx = cg.nx + 1, csxy = (cg.nx + 1) * (cg.ny + 1);
  // the 8 corner loads are issued unconditionally: along an even axis the
  // second neighbour is the first one again, with weight 0
  const int ii[2] = {i0, i1}, jj[2] = {j0, j1}, kk[2] = {k0, k1};
  const T w = wi * wj * wk;
  T v[8][3], wq[8];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int q = 4 * c + 2 * b + a;
        const bool used = (c == 0 || (k & 1)) && (b == 0 || (j & 1)) && (a == 0 || (i & 1));
        const int cq = 3 * (ii[a] + csx * jj[b] + csxy * kk[c]);
        wq[q] = used ? w : T(0);
        v[q][0] = (T)zc[cq];
        v[q][1] = (T)zc[cq + 1];
        v[q][2] = (T)zc[cq + 2];
      }
  T acc[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    acc[0] += wq[q] * v[q][0];
    acc[1] += wq[q] * v[q][1];
    acc[2] += wq[q] * v[q][2];
  }
  const uint8_t m = fmask[n];
  T zv[3];
  if (rf) {
    const T s = omega * invd[n];
#pragma unroll
    for (int q = 0; q < 3; ++q) zv[q] = s * rf[3 * n + q];
  } else {
#pragma unroll
    for (int q = 0; q < 3; ++q) zv[q] = zf[3 * n + q];
  }
  if (st && st->done) return;  // read after the loads: no round trip in front of them
#pragma unroll
  for (int q = 0; q < 3; ++q) out[3 * n + q] = ((m >> q) & 1) ? T(0) : zv[q] + acc[q];
}

template <typename T>
const T* lev_invd(const Level& L);
template <>
const double* lev_invd<double>(const Level& L) { return L.invd64; }
template <>
const float* lev_invd<float>(const Level& L) { return L.invd32; }
template <typename T>
const T* lev_E(const Level& L);
template <>
const double* lev_E<double>(const Level& L) { return L.E64; }
template <>
const float* lev_E<float>(const Level& L) { return L.E32; }

// Pre-smoothing on level l: n damped Jacobi sweeps from z = 0, then the
// residual t = r - K z.  The first sweep (z = omega D^-1 r, pointwise) is
// formed inside the next tiled launch instead of a launch of its own: for
// n = 1 inside the residual launch (which also stores z), otherwise inside
// the second sweep.  With fold_rr > 0 that first launch also takes the CG
// convergence decision.  Level 0 of a matrix-core problem keeps the
// separate first sweep, so that its tiled launches stay on matrix cores.
template <typename T>
hipError_t presmooth(fe_problem* p, int l, const T* r, T* z, T* t, int n, CgState* st, int fold_rr) {
  const Level& L = p->L[l];
  const double om = p->mg_omega;
  TileFuse<T> fz;
  fz.fold = fold_rr > 0 ? part_region(p, PART_RR) : nullptr;
  fz.nfold = fold_rr;
  fz.fold_rr = fold_rr > 0;
  const bool fuse = !(l == 0 && p->mfma_l0) || fold_rr > 0;
  hipError_t e = hipSuccess;
  if (!fuse) {
    T* a = (n % 2) ? z : t;  // first target chosen so the last sweep lands in z
    T* b = (n % 2) ? t : z;
    hipLaunchKernelGGL(jacobi0_kernel<T>, dim3(nblocks(L.g.ndof), p->bcount), dim3(FE_BLOCK), 0, p->stream,
                       L.g.ndof, r, lev_invd<T>(L), (T)om, a, st, wsh_of(p));
    e = hipGetLastError();
    for (int s = 1; s < n && e == hipSuccess; ++s) {
      e = launch_kxu_tile<T>(p, l, a, lev_E<T>(L), b, st, 3, nullptr, nullptr, r, lev_invd<T>(L), om);
      T* tmp = a;
      a = b;
      b = tmp;
    }
    if (e != hipSuccess) return e;
    return launch_kxu_tile<T>(p, l, z, lev_E<T>(L), t, st, 4, nullptr, nullptr, r, nullptr, 0.0);
  }
  fz.xin = 1;
  fz.invd = lev_invd<T>(L);
  fz.s = om;
  if (n == 1) {  // t = r - K z with z = omega D^-1 r (not stored: the prolongation forms it again)
    return launch_kxu_tile<T>(p, l, r, lev_E<T>(L), t, st, 4, nullptr, nullptr, r, nullptr, 0.0, nullptr, &fz);
  }
  // sweeps 2 .. n ping-pong between t and z so that the last lands in z
  T* a = (n % 2) ? t : z;
  T* b = (n % 2) ? z : t;
  e = launch_kxu_tile<T>(p, l, r, lev_E<T>(L), a, st, 3, nullptr, nullptr, r, lev_invd<T>(L), om, nullptr, &fz);
  for (int s = 2; s < n && e == hipSuccess; ++s) {
    e = launch_kxu_tile<T>(p, l, a, lev_E<T>(L), b, st, 3, nullptr, nullptr, r, lev_invd<T>(L), om);
    T* tmp = a;
    a = b;
    b = tmp;
  }
  if (e != hipSuccess) return e;
  return launch_kxu_tile<T>(p, l, z, lev_E<T>(L), t, st, 4, nullptr, nullptr, r, nullptr, 0.0);
}

// Chebyshev interval [lam_max / ratio, 1.02 lam_max] of the coarsest level: its centre.
static inline double cheb_theta(const fe_problem* p) {
  const double b = 1.02 * p->lam_max, a = b / p->cheb_ratio;
  return 0.5 * (b + a);
}

// `deg` steps of Jacobi-preconditioned Chebyshev iteration on the interval
// [b / ratio, b], b = 1.02 lam_max (lam_max bounds the spectrum of D^-1 K
// from above), for A z = r: from z = 0 (first) or adding to z.  The result
// is a fixed polynomial in D^-1 K applied to D^-1 r: linear, symmetric and
// (since the Chebyshev residual polynomial stays inside (0, 1) below the
// interval and below 1 in magnitude on it) positive definite.  The
// iteration's residual starts from r_src and moves between r_a and r_b
// (the first launch reads r_src and writes r_a; r_src is overwritten only
// if it is r_b); *r_end receives the buffer holding the final residual.
template <typename T>
hipError_t cheb_run(fe_problem* p, int l, T* r_src, T* r_a, T* r_b, T* z, T* d0, T* d1, int deg, double ratio,
                    bool first, CgState* st, bool d0_ready, T** r_end) {
  const bool keep_src = r_src != r_b;
  const Level& L = p->L[l];
  const double b = 1.02 * p->lam_max, a = b / ratio;
  const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
  double rho = 1.0 / sigma;
  // d0 = D^-1 r / theta: formed by the restriction when d0_ready, else by
  // the first launch of pairs on 3D tiles, else by a launch of its own
  const bool pairs = p->cheb_per_launch != 1 && deg >= 2;
  double dscale = 0.0;
  if (!d0_ready && pairs && cheb2_forms_first_direction<T>(p, l))
    dscale = 1.0 / theta;
  else if (!d0_ready)
    hipLaunchKernelGGL(jacobi0_kernel<T>, dim3(nblocks(L.g.ndof), p->bcount), dim3(FE_BLOCK), 0, p->stream,
                       L.g.ndof, r_src, lev_invd<T>(L), (T)(1.0 / theta), d0, st, wsh_of(p));
  hipError_t e = hipGetLastError();
  T* rin = r_src;
  T* rout = r_a;
  // profiling form 7: one event pair around a coarsest-level solve's
  // launches; the algorithmic bytes of each launch (one, two or three steps) read
  // d_k, r_k, the iterate, D^-1, the fixed-dof mask and E and write the
  // residual, the iterate and the next direction, each array once
  int prof = -1;
  if (p->kst.on && p->kst.mode == 7 && p->bcount == 1 && l == p->nlev - 1) {
    const int launches = p->cheb_per_launch == 1 ? deg : cheb_triples<T>(p, l) ? (deg == 4 ? 2 : (deg + 2) / 3)
                                                                                : (deg + 1) / 2;
    prof = kstats_begin(p, (double)launches * ((double)sizeof(T) * (19.0 * (double)L.g.nnode + (double)L.g.nelem) +
                                               (double)L.g.nnode));
  }
  const bool triples = cheb_triples<T>(p, l);
  for (int k = 0; k < deg && e == hipSuccess;) {
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    if (triples && k + 3 <= deg && deg - k != 4) {
      // steps k .. k + 2 in one launch (four left: two pairs)
      const double rho2 = 1.0 / (2.0 * sigma - rho1);
      const double rho3 = 1.0 / (2.0 * sigma - rho2);
      const double c[6] = {rho1 * rho,  2.0 * rho1 / delta, rho2 * rho1,
                           2.0 * rho2 / delta, rho3 * rho2, 2.0 * rho3 / delta};
      e = launch_cheb3<T>(p, l, d0, d1, lev_E<T>(L), lev_invd<T>(L), rin, rout, z, c, first && k == 0, st,
                          k == 0 ? dscale : 0.0);
      rho = rho3;
      rin = rout;
      rout = rin == r_a ? r_b : r_a;
      k += 3;
    } else if (p->cheb_per_launch != 1 && k + 2 <= deg && rout) {
      // steps k and k + 1 in one launch; the residual moves to the other buffer
      const double rho2 = 1.0 / (2.0 * sigma - rho1);
      const double c[4] = {rho1 * rho, 2.0 * rho1 / delta, rho2 * rho1, 2.0 * rho2 / delta};
      e = launch_cheb2<T>(p, l, d0, d1, lev_E<T>(L), lev_invd<T>(L), rin, rout, z, c, first && k == 0, st,
                          k == 0 ? dscale : 0.0);
      rho = rho2;
      rin = rout;
      rout = rin == r_a ? r_b : r_a;
      k += 2;
    } else {
      // one step, its residual updated in place (a kept r_src is copied out first)
      if (keep_src && rin == r_src) {
        e = hipMemcpyAsync(rout, rin, L.g.ndof * sizeof(T), hipMemcpyDeviceToDevice, p->stream);
        if (e != hipSuccess) break;
        rin = rout;
        rout = rin == r_a ? r_b : r_a;
      }
      ChebStep<T> cs;
      cs.res = rin;
      cs.acc = z;
      cs.c1 = rho1 * rho;
      cs.c2 = 2.0 * rho1 / delta;
      cs.first = first && k == 0;
      e = launch_kxu_tile<T>(p, l, d0, lev_E<T>(L), d1, st, 6, nullptr, nullptr, nullptr, lev_invd<T>(L), 0.0,
                             &cs);
      rho = rho1;
      k += 1;
    }
    std::swap(d0, d1);
  }
  kstats_end(p, prof);
  if (r_end) *r_end = rin;
  return e;
}

// Coarsest-level solve: `deg` steps from z = 0 on [lam_max / cheb_ratio,
// lam_max].  r and the level's mg_q buffer are overwritten.
template <typename T>
hipError_t chebyshev_solve(fe_problem* p, int l, T* r, T* z, T* d0, T* d1, int deg, CgState* st, bool d0_ready) {
  return cheb_run<T>(p, l, r, static_cast<T*>(p->L[l].mg_q), r, z, d0, d1, deg, p->cheb_ratio, true, st, d0_ready,
                     nullptr);
}

}  // namespace

template <typename T>
hipError_t launch_vcycle(fe_problem* p, int l, const T* r, T* z, CgState* st, int rz, int fold_rr);

namespace {
// V-cycle on a level between the finest and the coarsest with Chebyshev
// smoothing: cs_deg steps from z = 0 (their residual is the one restricted),
// the coarse correction, the residual r - K z, and cs_deg steps more on it
// added to z.  Both smoothers are the same polynomial in D^-1 K applied to
// D^-1 (symmetric), so the cycle stays symmetric.  r is kept.
template <typename T>
hipError_t cheb_smoothed_cycle(fe_problem* p, int l, const T* r, T* z, CgState* st) {
  const Level& L = p->L[l];
  T* t = static_cast<T*>(L.mg_t);
  T* w = static_cast<T*>(L.mg_w);
  T* q = static_cast<T*>(L.mg_q);
  T* s = static_cast<T*>(L.mg_s);
  T* res = nullptr;
  hipError_t e = cheb_run<T>(p, l, const_cast<T*>(r), q, s, z, t, w, p->cs_deg, p->cs_ratio, true, st, false, &res);
  if (e != hipSuccess) return e;
  const Level& C = p->L[l + 1];
  const bool last = l + 1 == p->nlev - 1;
  // the next level may run in float32 under a float64 one (as in launch_vcycle)
  using TC = typename std::conditional<std::is_same<T, double>::value, float, T>::type;
  if (std::is_same<T, double>::value && l + 1 >= p->f32_from) {
    TC* rc = static_cast<TC*>(C.mg_r);
    TC* zc = static_cast<TC*>(C.mg_z);
    hipLaunchKernelGGL((restrict_kernel<T, TC>), dim3(nblocks(C.g.nnode), p->bcount), dim3(FE_BLOCK), 0,
                       p->stream, L.g, C.g, node_div(C.g), res, C.nmask, rc, st, wsh_of(p), last ? C.invd32 : nullptr,
                       (TC)(1.0 / cheb_theta(p)), last ? static_cast<TC*>(C.mg_t) : nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_vcycle<TC>(p, l + 1, rc, zc, st, RZ_NONE, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL((prolong_add_kernel<T, TC>), dim3(nblocks(L.g.nnode), p->bcount), dim3(FE_BLOCK), 0,
                       p->stream, L.g, C.g, node_div(L.g), z, zc, L.nmask, z, nullptr, nullptr, (T)0, st, wsh_of(p));
  } else {
    T* rc = static_cast<T*>(C.mg_r);
    T* zc = static_cast<T*>(C.mg_z);
    hipLaunchKernelGGL(restrict_kernel<T>, dim3(nblocks(C.g.nnode), p->bcount), dim3(FE_BLOCK), 0, p->stream,
                       L.g, C.g, node_div(C.g), res, C.nmask, rc, st, wsh_of(p), last ? lev_invd<T>(C) : nullptr,
                       (T)(1.0 / cheb_theta(p)), last ? static_cast<T*>(C.mg_t) : nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_vcycle<T>(p, l + 1, rc, zc, st, RZ_NONE, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL(prolong_add_kernel<T>, dim3(nblocks(L.g.nnode), p->bcount), dim3(FE_BLOCK), 0, p->stream,
                       L.g, C.g, node_div(L.g), z, zc, L.nmask, z, nullptr, nullptr, (T)0, st, wsh_of(p));
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = launch_kxu_tile<T>(p, l, z, lev_E<T>(L), q, st, 4, nullptr, nullptr, r, nullptr, 0.0)) != hipSuccess)
    return e;
  return cheb_run<T>(p, l, q, s, q, z, t, w, p->cs_deg, p->cs_ratio, false, st, false, nullptr);
}
}  // namespace

// z = V(r): one symmetric V-cycle on levels l .. nlev-1 (pre- and
// post-smoothing with mg_nu damped Jacobi sweeps, a Chebyshev solve of
// degree mg_coarse_sweeps on the coarsest level).  st (may be null) guards
// the launches; rz and fold_rr as declared in the internal header.
template <typename T>
hipError_t launch_vcycle(fe_problem* p, int l, const T* r, T* z, CgState* st, int rz, int fold_rr) {
  const Level& L = p->L[l];
  T* t = static_cast<T*>(L.mg_t);
  if (l == p->nlev - 1)  // r is this level's own restricted residual: free to overwrite
    return chebyshev_solve<T>(p, l, const_cast<T*>(r), z, t, static_cast<T*>(L.mg_w), p->mg_coarse_sweeps, st,
                              l > 0);
  if (l > 0 && l >= p->cs_from) return cheb_smoothed_cycle<T>(p, l, r, z, st);
  // z from the pre-smoothing sweeps, t = r - K z restricted to the next level
  hipError_t e = presmooth<T>(p, l, r, z, t, p->mg_nu, st, l == 0 ? fold_rr : 0);
  if (e != hipSuccess) return e;
  const Level& C = p->L[l + 1];
  T* rc = static_cast<T*>(C.mg_r);
  T* zc = static_cast<T*>(C.mg_z);
  // the restriction to the coarsest level also forms its first Chebyshev direction
  const bool last = l + 1 == p->nlev - 1;
  // a float64 hierarchy may run its levels from f32_from on in float32 (their
  // buffers are sized for float64 and hold the float32 values)
  const bool narrow = std::is_same<T, double>::value && l + 1 >= p->f32_from;
  const int nu = p->mg_nu;
  const bool z_implicit = nu == 1 && (!(l == 0 && p->mfma_l0) || (l == 0 && fold_rr > 0));
  T* a = (nu % 2) ? t : z;
  if (narrow) {
    float* rcf = static_cast<float*>(C.mg_r);
    float* zcf = static_cast<float*>(C.mg_z);
    hipLaunchKernelGGL((restrict_kernel<T, float>), dim3(nblocks(C.g.nnode), p->bcount), dim3(FE_BLOCK), 0,
                       p->stream, L.g, C.g, node_div(C.g), t, C.nmask, rcf, st, wsh_of(p), last ? C.invd32 : nullptr,
                       (float)(1.0 / cheb_theta(p)), last ? static_cast<float*>(C.mg_t) : nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_vcycle<float>(p, l + 1, rcf, zcf, st, RZ_NONE, 0)) != hipSuccess) return e;
    hipLaunchKernelGGL((prolong_add_kernel<T, float>), dim3(nblocks(L.g.nnode), p->bcount), dim3(FE_BLOCK), 0,
                       p->stream, L.g, C.g, node_div(L.g), z, zcf, L.nmask, a, z_implicit ? r : nullptr,
                       z_implicit ? lev_invd<T>(L) : nullptr, (T)p->mg_omega, st, wsh_of(p));
  } else {
    hipLaunchKernelGGL(restrict_kernel<T>, dim3(nblocks(C.g.nnode), p->bcount), dim3(FE_BLOCK), 0, p->stream, L.g,
                       C.g, node_div(C.g), t, C.nmask, rc, st, wsh_of(p), last ? lev_invd<T>(C) : nullptr,
                       (T)(1.0 / cheb_theta(p)), last ? static_cast<T*>(C.mg_t) : nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_vcycle<T>(p, l + 1, rc, zc, st, RZ_NONE, 0)) != hipSuccess) return e;
    // post-smoothing, arranged so the last sweep writes z; with one fused
    // pre-smoothing sweep z was not stored and the prolongation forms it
    hipLaunchKernelGGL(prolong_add_kernel<T>, dim3(nblocks(L.g.nnode), p->bcount), dim3(FE_BLOCK), 0, p->stream,
                       L.g, C.g, node_div(L.g), z, zc, L.nmask, a, z_implicit ? r : nullptr,
                       z_implicit ? lev_invd<T>(L) : nullptr, (T)p->mg_omega, st, wsh_of(p));
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  T* b = (a == t) ? z : t;
  for (int s = 0; s < nu; ++s) {
    const bool last = rz != RZ_NONE && l == 0 && s == nu - 1;
    TileFuse<T> fz;
    if (last && rz == RZ_PARTIALS) {
      fz.part = part_region(p, PART_RZ);
      fz.no_finalize = true;
    }
    e = launch_kxu_tile<T>(p, l, a, lev_E<T>(L), b, st, last ? 5 : 3, nullptr, nullptr, r, lev_invd<T>(L),
                           p->mg_omega, nullptr, (last && rz == RZ_PARTIALS) ? &fz : nullptr);
    if (e != hipSuccess) return e;
    T* tmp = a;
    a = b;
    b = tmp;
  }
  return hipSuccess;
}

template hipError_t launch_vcycle<double>(fe_problem*, int, const double*, double*, CgState*, int, int);
template hipError_t launch_vcycle<float>(fe_problem*, int, const float*, float*, CgState*, int, int);
