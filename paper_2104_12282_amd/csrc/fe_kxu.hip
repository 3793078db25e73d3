// Matrix-free K(rho) * x for the structured brick mesh (gfx950, wave64).
//
// Layout of the work.  A workgroup of 16 x 16 threads owns a 15 x 15 block of
// node columns and marches up through kc node levels.  Thread (tx, ty) loads
// node column (I0 + tx, J0 + ty) and computes the brick whose lower-left
// corner is that node (one brick per thread per level).  Node values of the
// current level are exchanged through LDS; the lower level of a brick is the
// upper level of the brick below it, so it stays in registers, and so do the
// contributions of a brick to its upper four corners, which are added to the
// next brick's lower corners.  Contributions of the four bricks around a node
// column meet in LDS.  Every node's sum is formed by the one workgroup that
// owns it, in a fixed order: no atomics, bitwise reproducible.
//
// The brick operator.  With t = V u_e (V = per-axis sum/difference transform
// of the 8 corners, applied to each displacement component), Ke u_e =
// V S t where S has 45 non-zeros given by eight constants (isotropic cube);
// this is exact and costs about a fifth of the dense 24 x 24 product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "fe_internal.h"
#include "fe_reduce.h"

// No multiply-add is fused unless written as fma(): every kernel here then
// rounds the brick arithmetic alike, whatever the surrounding code (the
// fused Chebyshev launch relies on matching the single-step one bitwise).
#pragma clang fp contract(off)

namespace {

constexpr int TX = 16, TY = 16, OWN = 15;

#ifndef FE_KXU_MIN_WAVES
#define FE_KXU_MIN_WAVES 1  // no occupancy floor beyond what the registers give
#endif

// Occupancy floor per instance: the float32 last-sweep form (MODE 5) fits
// 128 VGPRs without spills when asked to, four waves per SIMD instead of
// three; every other instance keeps what its registers give.
template <typename T, int MODE>
constexpr int kxu_min_waves() {
  return std::is_same<T, float>::value && MODE == 5 ? 4 : FE_KXU_MIN_WAVES;
}

template <typename T>
struct WK {
  T A, B, G, C, D, F, H, J;
};

// Corner offsets of the brick in the fixed local order 000 100 110 010 001 101 111 011.
constexpr int kCornerX[8] = {0, 1, 1, 0, 0, 1, 1, 0};
constexpr int kCornerY[8] = {0, 0, 1, 1, 0, 0, 1, 1};
constexpr int kCornerZ[8] = {0, 0, 0, 0, 1, 1, 1, 1};

template <typename T>
__device__ inline void bf(T& a, T& b) {
  const T s = a + b, d = a - b;
  a = s;
  b = d;
}

// corners/modes in local order 000 100 110 010 001 101 111 011
template <typename T>
__device__ inline void walsh8(T (&v)[8]) {
  bf(v[0], v[1]); bf(v[3], v[2]); bf(v[4], v[5]); bf(v[7], v[6]);  // x
  bf(v[0], v[3]); bf(v[1], v[2]); bf(v[4], v[7]); bf(v[5], v[6]);  // y
  bf(v[0], v[4]); bf(v[1], v[5]); bf(v[2], v[6]); bf(v[3], v[7]);  // z
}

// s = S t for one brick (constants already scaled by the brick modulus).
// Mode numbers: 1=100 2=110 3=010 4=001 5=101 6=111 7=011.
template <typename T>
__device__ inline void apply_S(const WK<T>& k, const T (&t)[3][8], T (&s)[3][8]) {
  enum { X = 0, Y = 1, Z = 2 };
  s[X][0] = s[Y][0] = s[Z][0] = T(0);
  // linear modes: normal block
  const T n1 = t[X][1], n2 = t[Y][3], n3 = t[Z][4];
  s[X][1] = fma(k.A, n1, k.B * (n2 + n3));
  s[Y][3] = fma(k.A, n2, k.B * (n1 + n3));
  s[Z][4] = fma(k.A, n3, k.B * (n1 + n2));
  // linear modes: shear pairs
  T g = k.G * (t[Y][1] + t[X][3]);
  s[Y][1] = g;
  s[X][3] = g;
  g = k.G * (t[Z][1] + t[X][4]);
  s[Z][1] = g;
  s[X][4] = g;
  g = k.G * (t[Z][3] + t[Y][4]);
  s[Z][3] = g;
  s[Y][4] = g;
  // bilinear pairs
  s[X][2] = fma(k.C, t[X][2], k.D * t[Z][7]);
  s[Z][7] = fma(k.D, t[X][2], k.C * t[Z][7]);
  s[Y][2] = fma(k.C, t[Y][2], k.D * t[Z][5]);
  s[Z][5] = fma(k.D, t[Y][2], k.C * t[Z][5]);
  s[X][5] = fma(k.C, t[X][5], k.D * t[Y][7]);
  s[Y][7] = fma(k.D, t[X][5], k.C * t[Y][7]);
  // bilinear triple
  const T a = t[Z][2], b = t[Y][5], c = t[X][7];
  s[Z][2] = fma(k.F, a, k.H * (b + c));
  s[Y][5] = fma(k.F, b, k.H * (a + c));
  s[X][7] = fma(k.F, c, k.H * (a + b));
  // trilinear mode
  s[X][6] = k.J * t[X][6];
  s[Y][6] = k.J * t[Y][6];
  s[Z][6] = k.J * t[Z][6];
}

// Stores through a raw buffer resource.  The hardware drops a store whose
// byte offset lies outside [0, bytes), so a lane with nothing to store is
// given an offset past the end instead of a branch around its store: a
// divergent branch around stores makes the compiler count those stores as
// possibly missing at the join, and every later wait for an older load then
// also waits for loads issued after it (the prefetched levels).
constexpr uint32_t kStoreDrop = 0x80000000u;  // beyond any range below 2^31 bytes

__device__ inline __amdgpu_buffer_rsrc_t store_range(void* base, uint32_t bytes) {
  // word 3 of a gfx9 buffer descriptor: 32-bit data format, no swizzle
  return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, 0x00020000);
}

__device__ inline void store_at(__amdgpu_buffer_rsrc_t r, uint32_t off, double v) {
  typedef int i32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(i32x2, v), r, (int)off, 0, 0);
}
__device__ inline void store_at(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, (int)off, 0, 0);
}
// a node's three values: one 16-byte and one 8-byte store (double), one
// 12-byte store (float)
__device__ inline void store3(__amdgpu_buffer_rsrc_t r, uint32_t off, const double (&v)[3]) {
  typedef int i32x2 __attribute__((ext_vector_type(2)));
  typedef int i32x4 __attribute__((ext_vector_type(4)));
  const i32x2 a = __builtin_bit_cast(i32x2, v[0]), b = __builtin_bit_cast(i32x2, v[1]);
  const i32x4 ab = {a.x, a.y, b.x, b.y};
  __builtin_amdgcn_raw_buffer_store_b128(ab, r, (int)off, 0, 0);
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(i32x2, v[2]), r, (int)(off + 16), 0, 0);
}
__device__ inline void store3(__amdgpu_buffer_rsrc_t r, uint32_t off, const float (&v)[3]) {
  typedef int i32x3 __attribute__((ext_vector_type(3)));
  const i32x3 a = {__builtin_bit_cast(int, v[0]), __builtin_bit_cast(int, v[1]), __builtin_bit_cast(int, v[2])};
  __builtin_amdgcn_raw_buffer_store_b96(a, r, (int)off, 0, 0);
}

// Loads through raw buffer ranges: a load at or past the end of its range
// reads zero, which is the value of every node and brick off the mesh, so
// no lane selects a pad address or branches around its load.  Offsets are
// formed as (index in a level + index of the level) * unit, each part set to
// kOffIndex when the lane's node or the level is out of range; a range holds
// fewer than kOffIndex nodes or elements (bounded on the host), so any part
// past it lands past the range's end without wrapping (2 kOffIndex * 24
// bytes stays below 2^32).
constexpr uint32_t kOffIndex = 1u << 26;

__device__ inline __amdgpu_buffer_rsrc_t load_range(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ inline double load1(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
  typedef int i32x2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(double, (i32x2)__builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ inline float load1(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
  return __builtin_bit_cast(float, (int)__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ inline void load3(__amdgpu_buffer_rsrc_t r, uint32_t off, double (&v)[3]) {
  typedef int i32x2 __attribute__((ext_vector_type(2)));
  typedef int i32x4 __attribute__((ext_vector_type(4)));
  const i32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
  const i32x2 b = __builtin_amdgcn_raw_buffer_load_b64(r, (int)(off + 16), 0, 0);
  v[0] = __builtin_bit_cast(double, (i32x2){a[0], a[1]});
  v[1] = __builtin_bit_cast(double, (i32x2){a[2], a[3]});
  v[2] = __builtin_bit_cast(double, b);
}
__device__ inline void load3(__amdgpu_buffer_rsrc_t r, uint32_t off, float (&v)[3]) {
  typedef int i32x3 __attribute__((ext_vector_type(3)));
  const i32x3 a = __builtin_amdgcn_raw_buffer_load_b96(r, (int)off, 0, 0);
  // the elements go through scalars: __builtin_bit_cast of a vector element
  // reads the vector's first element on this toolchain
  const int a0 = a[0], a1 = a[1], a2 = a[2];
  v[0] = __builtin_bit_cast(float, a0);
  v[1] = __builtin_bit_cast(float, a1);
  v[2] = __builtin_bit_cast(float, a2);
}
__device__ inline uint8_t load_u8(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b8(r, (int)off, 0, 0);
}
// index part of a load offset: idx when in range, else kOffIndex
__device__ inline uint32_t off_part(bool in, int64_t idx) { return in ? (uint32_t)idx : kOffIndex; }
// level part: (k - lo) * stride for lo <= k < lo + n, else kOffIndex (one unsigned compare)
__device__ inline uint32_t lev_part(int k, int lo, int n, int64_t stride) {
  return (uint32_t)(k - lo) < (uint32_t)n ? (uint32_t)((int64_t)(k - lo) * stride) : kOffIndex;
}

// Epilogue operands of the modes below.
template <typename T>
struct Epi {
  const double* b64;  // MODE 2
  const T* bT;        // MODES 3, 4, 5
  const T* invd;      // MODES 3, 5, 6: inverse Jacobi diagonal per node
  T omega;            // MODES 3, 5: damping
  T* res;             // MODE 6: residual, updated in place
  T* acc;             // MODE 6: iterate, updated in place
  T c1, c2;           // MODE 6: direction recurrence
  int first;          // MODE 6: the iterate starts at zero
};

// Workgroup -> tile.  The grid is one-dimensional; consecutive workgroups
// are dispatched to the eight XCDs in turn, so workgroup b runs on XCD b % 8.
// Each XCD is given one contiguous run of tiles (x fastest, then y, then the
// z chunk): neighbouring tiles share their halo nodes through that XCD's L2.
struct TileMap {
  int gx, gy, nzc, kc, nblk;
};

__device__ inline void tile_of_block(const TileMap& tm, int& cx, int& cy, int& cz) {
  const int b = blockIdx.x, xcd = b & 7, m = b >> 3;
  const int q = tm.nblk >> 3, r = tm.nblk & 7;
  const int lid = xcd * q + min(xcd, r) + m;
  cx = lid % tm.gx;
  const int rest = lid / tm.gx;
  cy = rest % tm.gy;
  cz = rest / tm.gy;
}

// x and y butterflies of one face (corners 00 10 11 01 of a node level):
// the part of the brick transform that the brick below and the brick above
// a face have in common.
template <typename T>
__device__ inline void face4(T (&v)[4]) {
  bf(v[0], v[1]);
  bf(v[3], v[2]);
  bf(v[0], v[3]);
  bf(v[1], v[2]);
}

// One brick layer of a march up through node levels, for the brick whose
// lower-left corner is this thread's node column.  fl: the lower face,
// already x-y transformed (face4); on return the upper face, which is the
// next brick's lower face.  fu: the upper face's corner values 00 10 11 01
// (transformed here).  carry: the upper-corner contributions of the brick
// below (on return: this brick's, in the face domain).  lo: this brick's
// contributions to its lower corners 00 10 11 01 with the carry added, back
// in corner values.  Ee scales the constants (the brick's modulus).
template <typename T>
__device__ inline void brick_layer(T (&fl)[3][4], T (&fu)[3][4], T (&carry)[3][4], T Ee, const WK<T>& wk,
                                   T (&lo)[3][4]) {
  T t[3][8];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    face4(fu[c]);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      t[c][i] = fl[c][i] + fu[c][i];
      t[c][i + 4] = fl[c][i] - fu[c][i];
      fl[c][i] = fu[c][i];
    }
  }
  WK<T> k = wk;
  k.A *= Ee; k.B *= Ee; k.G *= Ee; k.C *= Ee; k.D *= Ee; k.F *= Ee; k.H *= Ee; k.J *= Ee;
  T w[3][8];
  apply_S(k, t, w);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      lo[c][i] = (w[c][i] + w[c][i + 4]) + carry[c][i];
      carry[c][i] = w[c][i] - w[c][i + 4];
    }
    face4(lo[c]);
  }
}

// Node sum of component c at a node whose own brick gave p0: the partials
// of the bricks at (x-1, y), (x-1, y-1) and (x, y-1), in this fixed order.
template <typename T>
__device__ inline T node_sum(T p0, const T (&syb)[9][TY][TX], int c, int ty, int tx, int tyl, int txl) {
  return p0 + syb[0 + c][ty][txl] + syb[3 + c][tyl][txl] + syb[6 + c][tyl][tx];
}

// Chebyshev step at one dof: residual r - (K d)_i and direction
// c1 d_i + c2 D^-1_i (new residual); both zero at a fixed dof.
template <typename T>
__device__ inline void cheb_dof(bool fx, T r, T Kd, T d, T invd, T c1, T c2, T& rn, T& dn) {
  rn = fx ? T(0) : r - Kd;
  dn = fx ? T(0) : fma(c1, d, (c2 * invd) * rn);
}

// Fused operand of a launch (see TileFuse): XIN 1 forms x = s D^-1 a, XIN 2
// the CG direction x = z + beta p; owners store the x they used to xout.
template <typename T>
struct XinK {
  const T* invd;  // XIN 1
  T s;            // XIN 1
  const T* pold;  // XIN 2
  T* xout;        // may be null
};
// Reduction folded into a launch: `what` 1 = r^T z partials (direction
// factor beta), 2 = r^T r partials (convergence test of the CG update).
struct FoldK {
  const double* part;
  int n;
  int what;
};

// Sum of part[0..n) in a fixed order, returned to every thread of the
// workgroup (each workgroup of a launch computes the same value).
__device__ inline double block_sum_all(const double* __restrict__ part, int n) {
  __shared__ double sh[TX * TY / 64];
  __shared__ double tot;
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += TX * TY) v += part[i];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < TX * TY / 64; ++w) t += sh[w];
    tot = t;
  }
  __syncthreads();
  return tot;
}

// MODE 0: y = Kx.  MODE 1: CG step, pq = x^T y, alpha = rz / pq.
// MODE 2: y = b - Kx (float64 only), ||y||^2 -> out[0].
// MODE 3: damped Jacobi sweep y = x + omega D^-1 (b - Kx).
// MODE 4: y = b - Kx.
// MODE 5: MODE 3 and rz = b^T y, beta = rz / rz_old into st (the last sweep of
//         a multigrid V-cycle that preconditions CG).
// MODE 6: one step of Jacobi-preconditioned Chebyshev iteration with
//         direction d = x: acc += d, res -= K d, y = c1 d + c2 D^-1 res.
// For modes 3, 4 and 6 a non-null st only guards: the launch is skipped once
// CG has stopped.  y must not alias x (other workgroups read x around their
// tiles).
//
// Pipeline of one level step (brick layer ek between node levels ek and
// ek + 1), with one barrier:
//   1. the upper level (loaded two steps ahead) goes to LDS buffer (ek+1)&1;
//   2. loads are issued for level ek + 3 and for the epilogue operands of
//      level ek + 1;
//   3. barrier;
//   4. the node sums of level ek - 1 (complete since the previous step) are
//      read from partial buffer (ek-1)&1 and written out;
//   5. the brick is computed: upper face from LDS, lower face (already in
//      the x-y transformed form) from registers, z butterflies, S, inverse z
//      butterflies; the upper half stays in registers as the carry to the
//      next brick, the lower half plus the carry from the brick below is
//      transformed back and goes to partial buffer ek&1.
// Double buffering of both LDS arrays makes the single barrier sufficient:
// a buffer is rewritten only after every thread has passed the barrier that
// follows its last read.
template <typename T, int MODE, int XIN>
__global__ void __launch_bounds__(TX* TY, (kxu_min_waves<T, MODE>())) kxu_tile_kernel(Grid g, TileMap tm, const T* __restrict__ x,
                                                         const T* __restrict__ E,
                                                         const uint8_t* __restrict__ nmask, WK<T> wk,
                                                         T* __restrict__ y, Epi<T> ep, CgState* st,
                                                         double* partials, double* out,
                                                         const T* __restrict__ zpad, XinK<T> xi, FoldK fo,
                                                         int64_t wsh) {
  if (wsh) {  // batched launch: this workgroup's problem
    const int64_t o = batch_offset(wsh);
    x = wshift(x, o);
    E = wshift(E, o);
    nmask = wshift(nmask, o);
    y = wshift(y, o);
    ep.b64 = wshift(ep.b64, o);
    ep.bT = wshift(ep.bT, o);
    ep.invd = wshift(ep.invd, o);
    ep.res = wshift(ep.res, o);
    ep.acc = wshift(ep.acc, o);
    st = wshift(st, o);
    partials = wshift(partials, o);
    out = wshift(out, o);
    zpad = wshift(zpad, o);
    xi.invd = wshift(xi.invd, o);
    xi.pold = wshift(xi.pold, o);
    xi.xout = wshift(xi.xout, o);
    fo.part = wshift(fo.part, o);
  }
  // the operand of the folded CG direction (set by the gate below)
  T beta = T(0);
  bool first_dir = false;
  __shared__ T su[2][3][TY + 1][TX + 1];  // node values of a level (17 x 17 ring)
  __shared__ T sy[2][9][TY][TX];          // lower-level partials of corners (1,0), (1,1), (0,1)

  int cx, cy, cz;
  tile_of_block(tm, cx, cy, cz);
  const int kc = tm.kc;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int I0 = cx * OWN - 1, J0 = cy * OWN - 1, K0 = cz * kc;
  const int ni = I0 + tx, nj = J0 + ty;
  const int64_t sx = g.nx + 1, sxy = (int64_t)(g.nx + 1) * (g.ny + 1);
  const bool owner = tx >= 1 && ty >= 1 && ni <= g.nx && nj <= g.ny;
  const bool ecol = ni >= 0 && ni < g.nx && nj >= 0 && nj < g.ny;
  const int kend = min(K0 + kc, g.nz + 1);  // owned levels: [K0, kend)
  // halo slot: threads 0..16 load column TX (rows 0..16), 17..32 row TY
  const int h = threadIdx.x;
  const bool hslot = h < TX + TY + 1;
  const int hx = h <= TY ? TX : h - (TY + 1), hy = h <= TY ? h : TY;
  const int hi = I0 + hx, hj = J0 + hy;

  // Loads go through raw buffer ranges (zero past the range: the nodes and
  // bricks off the mesh), so no instruction has to touch a load's registers
  // before the data is used and no lane branches around a load.  Node levels
  // loaded: [nlo, nhi]; brick layers: [elo, ehi].
  const int nlo = max(K0 - 1, 0), nhi = min(kend, g.nz), elo = max(K0 - 1, 0), ehi = min(kend - 1, g.nz - 1);
  const int64_t nlev = nhi - nlo + 1, nel = (int64_t)g.nx * g.ny;
  // XIN 3: the operand x (the preconditioned residual) is float32
  constexpr int64_t xsz = XIN == 3 ? 4 : (int64_t)sizeof(T);
  const int64_t vbytes = 3 * sxy * nlev * (int64_t)sizeof(T);
  const __amdgpu_buffer_rsrc_t rx =
      load_range(reinterpret_cast<const char*>(x) + 3 * sxy * nlo * xsz, 3 * sxy * nlev * xsz);
  const __amdgpu_buffer_rsrc_t rxd =
      load_range(XIN == 1 ? (const void*)(xi.invd + sxy * nlo) : (const void*)x, XIN == 1 ? vbytes / 3 : 0);
  const __amdgpu_buffer_rsrc_t rxp =
      load_range(XIN >= 2 ? (const void*)(xi.pold + 3 * sxy * nlo) : (const void*)x, XIN >= 2 ? vbytes : 0);
  const __amdgpu_buffer_rsrc_t re =
      load_range(E + nel * elo, ehi >= elo ? nel * (ehi - elo + 1) * (int64_t)sizeof(T) : 0);
  const uint32_t o_own = off_part(ni >= 0 && ni <= g.nx && nj >= 0 && nj <= g.ny, ni + sx * nj);
  const uint32_t o_halo = off_part(hslot && hi >= 0 && hi <= g.nx && hj >= 0 && hj <= g.ny, hi + sx * hj);
  const uint32_t o_el = off_part(ecol, ni + (int64_t)g.nx * nj);
  // the operand as loaded: float32 under XIN 3, widened when it goes to LDS
  using XT = typename std::conditional<XIN == 3, float, T>::type;
  struct LevelIn {
    XT own[3];
    XT halo[3];
    T Ee;  // modulus of the brick layer below this level
    T d_own, d_halo;       // XIN 1: inverse diagonal
    T p_own[3], p_halo[3];  // XIN 2: previous direction
  };
  auto node_in = [&](uint32_t o, XT (&v)[3], T& d, T (&pv)[3]) {
    load3(rx, o * (uint32_t)(3 * sizeof(XT)), v);
    if (XIN == 1) d = load1(rxd, o * (uint32_t)sizeof(T), T());
    if (XIN >= 2) load3(rxp, o * (uint32_t)(3 * sizeof(T)), pv);  // also on the first iteration (then unused)
  };
  auto load_level = [&](int k, LevelIn& L) {
    const uint32_t lk = lev_part(k, nlo, (int)nlev, sxy);  // k <= kend: nhi bounds it
    node_in(o_own + lk, L.own, L.d_own, L.p_own);
    node_in(o_halo + lk, L.halo, L.d_halo, L.p_halo);
    L.Ee = load1(re, (o_el + lev_part(k - 1, elo, ehi - elo + 1, nel)) * (uint32_t)sizeof(T), T());
  };
  // the operand value of a node from what was loaded for it
  auto operand = [&](const XT (&v)[3], T d, const T (&pv)[3], int c) -> T {
    const T x = (T)v[c];
    if (XIN == 1) return xi.s * d * x;
    if (XIN >= 2) return first_dir ? x : x + beta * pv[c];  // p_old is not set before the first
    return x;
  };
  // stores a level into LDS; the loaded registers die here (this thread's
  // own values are read back from LDS after the barrier), so the register
  // ring rotates in place and no copy waits for a load still in flight
  auto store_level = [&](int buf, const LevelIn& L) {
#pragma unroll
    for (int c = 0; c < 3; ++c) su[buf][c][ty][tx] = operand(L.own, L.d_own, L.p_own, c);
    if (hslot)
      for (int c = 0; c < 3; ++c) su[buf][c][hy][hx] = operand(L.halo, L.d_halo, L.p_halo, c);
  };
  // epilogue operands of this thread's node at one level (read only by owners)
  struct EpiIn {
    uint8_t m;
    T b[3];
    T d;
    T a[3];
    double b2[3];
  };
  // epilogue ranges: the owned levels [K0, kend)
  const int64_t elev = kend - K0;
  const __amdgpu_buffer_rsrc_t rm = load_range(nmask + sxy * K0, sxy * elev);
  const __amdgpu_buffer_rsrc_t rb2 =
      load_range(MODE == 2 ? (const void*)(ep.b64 + 3 * sxy * K0) : (const void*)x, MODE == 2 ? 24 * sxy * elev : 0);
  const bool has_b = MODE == 3 || MODE == 4 || MODE == 5, has_d = MODE == 3 || MODE == 5 || MODE == 6;
  const __amdgpu_buffer_rsrc_t rb = load_range(
      has_b ? (const void*)(ep.bT + 3 * sxy * K0) : MODE == 6 ? (const void*)(ep.res + 3 * sxy * K0) : (const void*)x,
      has_b || MODE == 6 ? 3 * sxy * elev * (int64_t)sizeof(T) : 0);
  const __amdgpu_buffer_rsrc_t ra = load_range(MODE == 6 ? (const void*)(ep.acc + 3 * sxy * K0) : (const void*)x,
                                               MODE == 6 ? 3 * sxy * elev * (int64_t)sizeof(T) : 0);
  const __amdgpu_buffer_rsrc_t rdi = load_range(has_d ? (const void*)(ep.invd + sxy * K0) : (const void*)x,
                                                has_d ? sxy * elev * (int64_t)sizeof(T) : 0);
  const uint32_t o_epi = off_part(owner, ni + sx * nj);
  auto load_epi = [&](int k, EpiIn& P) {
    const uint32_t o = o_epi + lev_part(k, K0, (int)elev, sxy);
    P.m = load_u8(rm, o);
    if (MODE == 2) load3(rb2, o * 24u, P.b2);
    if (has_b || MODE == 6) load3(rb, o * (uint32_t)(3 * sizeof(T)), P.b);
    if (MODE == 6) load3(ra, o * (uint32_t)(3 * sizeof(T)), P.a);  // unused on the first step (no branch)
    if (has_d) P.d = load1(rdi, o * (uint32_t)sizeof(T), T());
  };

  double dot = 0.0;
  // Stores of the owned levels [K0, kend) go through ranges that start at
  // level K0 (byte offsets below 2^31: the tile map bounds the chunk).
  const int64_t lev0 = 3 * sxy * K0;
  const uint32_t chunk_bytes = (uint32_t)(3 * sxy * (kend - K0) * (int64_t)sizeof(T));
  const __amdgpu_buffer_rsrc_t ry = store_range(y + lev0, chunk_bytes);
  const __amdgpu_buffer_rsrc_t rres = store_range(MODE == 6 ? ep.res + lev0 : y, MODE == 6 ? chunk_bytes : 0u);
  const __amdgpu_buffer_rsrc_t racc = store_range(MODE == 6 ? ep.acc + lev0 : y, MODE == 6 ? chunk_bytes : 0u);
  const __amdgpu_buffer_rsrc_t rxo =
      store_range(XIN && xi.xout ? xi.xout + lev0 : y, XIN && xi.xout ? chunk_bytes : 0u);
  // LDS reads of lanes that own no node stay inside the arrays
  const int txl = tx > 0 ? tx - 1 : 0, tyl = ty > 0 ? ty - 1 : 0;
  // node sums of level k: own corner p0 plus the partials of the three
  // neighbouring brick columns, then the mode's epilogue.  Every lane runs
  // it (no branch: see store_range); lanes without an owned node at level
  // k store at kStoreDrop and add nothing to the dot product.
  auto finish_level = [&](int k, const T (&p0)[3], const T (&own)[3], const EpiIn& P) {
    const bool mine = owner && k >= K0 && k < kend;
    const int buf = k & 1;
    const uint32_t at =
        mine ? (uint32_t)((ni + sx * nj + sxy * (k - K0)) * 3 * (int64_t)sizeof(T)) : kStoreDrop;
    T yv[3], rv[3], av[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T v2 = node_sum(p0[c], sy[buf], c, ty, tx, tyl, txl);
      const bool fx = (P.m >> c) & 1;
      if (fx) v2 = T(0);
      if (MODE == 2) {
        v2 = fx ? T(0) : (T)(P.b2[c] - (double)v2);
        dot += mine ? (double)v2 * (double)v2 : 0.0;
      } else if (MODE == 1) {
        dot += mine ? (double)own[c] * (double)v2 : 0.0;
      } else if (MODE == 3 || MODE == 5) {
        v2 = fx ? T(0) : own[c] + ep.omega * P.d * (P.b[c] - v2);
        if (MODE == 5) dot += mine ? (double)P.b[c] * (double)v2 : 0.0;
      } else if (MODE == 4) {
        v2 = fx ? T(0) : P.b[c] - v2;
      } else if (MODE == 6) {
        const T dv = own[c];
        cheb_dof(fx, P.b[c], v2, dv, P.d, ep.c1, ep.c2, rv[c], v2);
        av[c] = ep.first ? dv : P.a[c] + dv;
      }
      yv[c] = v2;
    }
    if (MODE == 6) {
      store3(rres, at, rv);
      store3(racc, at, av);
    }
    store3(ry, at, yv);
    if (XIN) store3(rxo, at, own);
  };

  T fl[3][4];      // lower face of the current brick, x-y transformed
  T carry[3][4];   // upper half of the brick below (z-transformed), to this level
  T own_lo[3];     // this thread's node on the lower level of the current brick
  T own_ll[3];     // ... and on the level below it (its sums finish one step late)
  T p0[3];         // own-corner sum of the level below
  // Register rings, two steps deep: R0..R2 hold node levels, Q0..Q2 epilogue
  // operands.  Step s (brick layer ek = K0 - 1 + s) uses level ek + 1 from
  // ring slot s % 3 and loads level ek + 3 into slot (s + 2) % 3 -- the slot
  // step s - 1 used -- and likewise the operands of level ek + 1, which
  // step s + 2 needs.  Loads thus have two steps to arrive.
  LevelIn R0, R1, R2;
  EpiIn Q0, Q1, Q2;
  {
    LevelIn L0;
    load_level(K0 - 1, L0);
    load_level(K0, R0);
    load_level(K0 + 1, R1);  // kend >= K0 + 1
    // The stop flag and the folded reductions are read only now, with the
    // first levels' loads already in flight (a read before them would put a
    // whole memory round trip in front of every launch); nothing has been
    // stored yet.  Folded reductions: every workgroup sums the same partials
    // in the same order, so all take the same decision; workgroup 0 records
    // it in st.
    if ((MODE == 1 || MODE == 5 || st) && st->done) return;
    if (fo.what == 1) {
      const double v = block_sum_all(fo.part, fo.n);
      const int it = st->iter;
      const bool bad = !(v > 0.0) || !finite_d(v);
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (bad) {
          st->status = FE_EBREAKDOWN;
          st->done = 1;
        } else {
          st->rz_new = v;
          st->beta = it == 0 ? 0.0 : v / st->rz;
        }
      }
      if (bad) return;
      first_dir = it == 0;
      beta = first_dir ? T(0) : (T)(v / st->rz);
    } else if (fo.what == 2) {
      const double v = block_sum_all(fo.part, fo.n);
      const int it = st->iter_next;
      int status = FE_OK;
      bool stop = false;
      if (!finite_d(v)) {
        stop = true;
        status = FE_EBREAKDOWN;
      } else if (v <= st->tol2) {
        stop = true;
      } else if (it >= st->max_iter) {
        stop = true;
        status = FE_ENOTCONV;
      }
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->iter = it;
        st->rr = v;
        if (stop) {
          st->status = status;
          st->done = 1;
        }
      }
      if (stop) return;
    }
    const int b0 = (K0 - 1) & 1;
    store_level(b0, L0);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      own_lo[c] = su[b0][c][ty][tx];
      fl[c][0] = own_lo[c];
      fl[c][1] = su[b0][c][ty][tx + 1];
      fl[c][2] = su[b0][c][ty + 1][tx + 1];
      fl[c][3] = su[b0][c][ty + 1][tx];
      face4(fl[c]);
      own_ll[c] = T(0);
      p0[c] = T(0);
      carry[c][0] = carry[c][1] = carry[c][2] = carry[c][3] = T(0);
    }
  }

  // fin: whether the step finishes level ek - 1 (the first two steps would
  // finish levels K0 - 2 and K0 - 1, which this workgroup does not own)
  auto step = [&](auto fin, int ek, const LevelIn& use, LevelIn& fill, const EpiIn& Pu, EpiIn& Pf) {
    const int bu = (ek + 1) & 1;
    store_level(bu, use);
    load_level(ek + 3, fill);
    load_epi(ek + 1, Pf);
    __syncthreads();
    T own_up[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) own_up[c] = su[bu][c][ty][tx];

    if constexpr (decltype(fin)::value) finish_level(ek - 1, p0, own_ll, Pu);

    T fu[3][4], lo[3][4];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      fu[c][0] = own_up[c];
      fu[c][1] = su[bu][c][ty][tx + 1];
      fu[c][2] = su[bu][c][ty + 1][tx + 1];
      fu[c][3] = su[bu][c][ty + 1][tx];
    }
    brick_layer(fl, fu, carry, use.Ee, wk, lo);
    const int bl = ek & 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      p0[c] = lo[c][0];
      sy[bl][0 + c][ty][tx] = lo[c][1];
      sy[bl][3 + c][ty][tx] = lo[c][2];
      sy[bl][6 + c][ty][tx] = lo[c][3];
      own_ll[c] = own_lo[c];
      own_lo[c] = own_up[c];
    }
  };

  // Step s (layer K0 - 1 + s) uses ring slot s % 3 and fills (s + 2) % 3;
  // the operands of level ek + 1 sit in slot (s + 2) % 3.  The first two
  // steps, which finish no owned level, are peeled off, so every step of
  // the loop stores.
  const std::false_type skip{};
  const std::true_type fin{};
  const int n = kend - K0 + 1;  // steps: layers K0 - 1 .. kend - 1 (n >= 2)
  step(skip, K0 - 1, R0, R2, Q0, Q2);
  step(skip, K0, R1, R0, Q1, Q0);
  int s = 2;
  for (; s + 3 <= n; s += 3) {
    step(fin, K0 - 1 + s, R2, R1, Q2, Q1);
    step(fin, K0 + s, R0, R2, Q0, Q2);
    step(fin, K0 + 1 + s, R1, R0, Q1, Q0);
  }
  if (s < n) step(fin, K0 - 1 + s, R2, R1, Q2, Q1);
  if (s + 1 < n) step(fin, K0 + s, R0, R2, Q0, Q2);
  __syncthreads();
  // level kend - 1 = K0 + n - 2: its operands went to slot n % 3
  const int last = n % 3;
  finish_level(kend - 1, p0, own_ll, last == 0 ? Q0 : last == 1 ? Q1 : Q2);

  if (MODE == 0 || MODE == 3 || MODE == 4 || MODE == 6) return;
  double vv[1] = {dot};
  block_partials<1>(vv, partials);
}

// ---------------------------------------------------------------------------
// Two steps of the coarsest-level Chebyshev iteration in one launch.
//
// On a small grid a launch costs mostly latency (loading what the previous
// launch wrote, a few march steps, the stores draining), so the coarse solve
// is bound by its number of launches.  A workgroup here runs two marches of
// 16 x 16 threads.  Group A marches step k (the tile kernel's march with the
// Chebyshev epilogue) over a 17 x 17 node ring and finishes the 15 x 15 node
// columns and the kc + 2 levels that step k + 1 needs around the 13 x 13
// columns and kc levels the workgroup owns; it hands r_{k+1} and d_{k+1} to
// group B through LDS, level by level.  Group B marches step k + 1 on those
// values behind it and writes the results.  The ring of step-k values is
// recomputed by the neighbouring workgroups as well (the price of the saved
// launch), and every node sum is formed in the tile kernel's order with the
// same per-dof update, so the result is bitwise that of two single-step
// launches.
//
// Unlike the tile kernel, a march step here finishes the level of its own
// brick layer, after a second barrier (bricks, then node sums), so a level
// reaches group B one step earlier.  Barriers are numbered from 0 for the
// whole workgroup: A's prologue passes barrier 0 and its step s barriers
// 2s + 1 and 2s + 2, finishing level l = K0 - 2 + s after the latter, i.e.
// after barrier 2(l - K0) + 6; B reads level l after barrier 2(l - K0) + 7
// (its prologue, level K0 - 1, after barrier 5; its step s, level K0 + s,
// after barrier 2s + 7), and A writes the same buffer again (level l + 2)
// after barrier 2(l - K0) + 10.  Both groups pass 2(kend - K0) + 9 barriers.
// The residual is read on the ring, so it cannot be updated in place
// (rin -> rout); the iterate acc is read and written at owned nodes only (in
// place).
template <typename T>
struct Cheb2 {
  T c1a, c2a;  // step k: d_{k+1} = c1a d_k + c2a D^-1 r_{k+1}
  T c1b, c2b;  // step k + 1
  int first;   // step k is the first (the iterate starts at zero)
  T dscale;    // 3D tiles: nonzero = d_k is not read but formed as dscale D^-1 r_k (the first direction)
  T c1c, c2c;  // step k + 2 (three steps per launch)
};

constexpr int OWN2 = 13;  // node columns per direction a fused workgroup finishes

template <typename T>
__global__ void __launch_bounds__(2 * TX * TY) cheb2_kernel(Grid g, TileMap tm, const T* __restrict__ dk,
                                                       const T* __restrict__ E,
                                                       const uint8_t* __restrict__ nmask, WK<T> wk,
                                                       const T* __restrict__ invd, const T* __restrict__ rin,
                                                       T* __restrict__ rout, T* __restrict__ acc,
                                                       T* __restrict__ y, Cheb2<T> cf, CgState* st,
                                                       const T* __restrict__ zpad, int64_t wsh) {
  if (wsh) {  // batched launch: this workgroup's problem
    const int64_t o = batch_offset(wsh);
    dk = wshift(dk, o);
    E = wshift(E, o);
    nmask = wshift(nmask, o);
    invd = wshift(invd, o);
    rin = wshift(rin, o);
    rout = wshift(rout, o);
    acc = wshift(acc, o);
    y = wshift(y, o);
    st = wshift(st, o);
    zpad = wshift(zpad, o);
  }
  __shared__ T suA[2][3][TY + 1][TX + 1];  // step-k direction by level (group A's ring)
  __shared__ T syA[9][TY][TX];
  __shared__ T suB[2][3][TY + 1][TX + 1];  // d_{k+1} by level, group B's frame
  __shared__ T srB[2][3][TY][TX];          // r_{k+1} by level, group B's frame
  __shared__ T syB[9][TY][TX];

  int cx, cy, cz;
  tile_of_block(tm, cx, cy, cz);
  const int K0 = cz * tm.kc, kend = min(K0 + tm.kc, g.nz + 1);  // owned levels: [K0, kend)
  const int64_t sx = g.nx + 1, sxy = (int64_t)(g.nx + 1) * (g.ny + 1);
  const int q = threadIdx.x % (TX * TY);
  const int tx = q % TX, ty = q / TX;
  const int nbar = 2 * (kend - K0) + 9;
  const int txl = tx > 0 ? tx - 1 : 0, tyl = ty > 0 ? ty - 1 : 0;
  const std::false_type skip{};
  const std::true_type fin{};
  // 256 threads are four whole waves: the group is uniform in a wave
  const int grp = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / (TX * TY)));

  if (grp == 0) {
    // ---- group A: step k on node columns I0 .. I0 + 16, levels ka0 - 1 .. kaend
    const int I0 = cx * OWN2 - 2, J0 = cy * OWN2 - 2;
    const int ni = I0 + tx, nj = J0 + ty;
    const int ka0 = K0 - 1, kaend = min(kend + 1, g.nz + 1);  // finished levels: [ka0, kaend)
    const bool owner = tx >= 1 && ty >= 1 && ni >= 0 && nj >= 0 && ni <= g.nx && nj <= g.ny;
    const bool ecol = ni >= 0 && ni < g.nx && nj >= 0 && nj < g.ny;
    const bool hslot = q < TX + TY + 1;
    const int hx = q <= TY ? TX : q - (TY + 1), hy = q <= TY ? q : TY;
    const int hi = I0 + hx, hj = J0 + hy;
    // load ranges: node levels [nlo, nhi], brick layers [elo, ehi]
    const int nlo = max(ka0 - 1, 0), nhi = min(kaend, g.nz);
    const int elo = max(ka0 - 1, 0), ehi = min(kaend - 1, g.nz - 1);
    const int64_t nel = (int64_t)g.nx * g.ny, nlev = nhi - nlo + 1;
    const __amdgpu_buffer_rsrc_t rx = load_range(dk + 3 * sxy * nlo, 3 * sxy * nlev * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t rr = load_range(rin + 3 * sxy * nlo, 3 * sxy * nlev * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t rd = load_range(invd + sxy * nlo, sxy * nlev * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t rm = load_range(nmask + sxy * nlo, sxy * nlev);
    const __amdgpu_buffer_rsrc_t re =
        load_range(E + nel * elo, ehi >= elo ? nel * (ehi - elo + 1) * (int64_t)sizeof(T) : 0);
    const uint32_t o_own = off_part(ni >= 0 && ni <= g.nx && nj >= 0 && nj <= g.ny, ni + sx * nj);
    const uint32_t o_halo = off_part(hslot && hi >= 0 && hi <= g.nx && hj >= 0 && hj <= g.ny, hi + sx * hj);
    const uint32_t o_epi = off_part(owner, ni + sx * nj);
    const uint32_t o_el = off_part(ecol, ni + (int64_t)g.nx * nj);
    struct LevelIn {
      T own[3];
      T halo[3];
      T Ee;  // modulus of the brick layer below this level
    };
    auto load_level = [&](int k, LevelIn& L) {
      const uint32_t lk = lev_part(k, nlo, (int)nlev, sxy);
      load3(rx, (o_own + lk) * (uint32_t)(3 * sizeof(T)), L.own);
      load3(rx, (o_halo + lk) * (uint32_t)(3 * sizeof(T)), L.halo);
      const int ek = k - 1;
      L.Ee = load1(re, (o_el + lev_part(ek, elo, ehi - elo + 1, nel)) * (uint32_t)sizeof(T), T());
    };
    auto store_level = [&](int buf, const LevelIn& L) {
#pragma unroll
      for (int c = 0; c < 3; ++c) suA[buf][c][ty][tx] = L.own[c];
      if (hslot)
        for (int c = 0; c < 3; ++c) suA[buf][c][hy][hx] = L.halo[c];
    };
    struct EpiIn {
      uint8_t m;
      T r[3];
      T d;
    };
    auto load_epi = [&](int k, EpiIn& P) {
      const int e0 = max(ka0, nlo);  // finished levels from here to kaend - 1
      const uint32_t o = o_epi + lev_part(k, e0, kaend - e0, sxy) + (uint32_t)((e0 - nlo) * sxy);
      P.m = load_u8(rm, o);
      load3(rr, o * (uint32_t)(3 * sizeof(T)), P.r);
      P.d = load1(rd, o * (uint32_t)sizeof(T), T());
    };
    // level k of step k: r_{k+1} and d_{k+1} (zero off the mesh) to group B
    auto finish = [&](int k, const T (&p0)[3], const T (&own)[3], const EpiIn& P) {
      const bool mine = owner && k >= 0 && k < kaend;
      const int buf = k & 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T v = node_sum(p0[c], syA, c, ty, tx, tyl, txl);
        const bool fx = (P.m >> c) & 1;
        if (fx) v = T(0);
        T rn, dn;
        cheb_dof(fx, P.r[c], v, own[c], P.d, cf.c1a, cf.c2a, rn, dn);
        if (tx >= 1 && ty >= 1) {
          suB[buf][c][ty - 1][tx - 1] = mine ? dn : T(0);
          srB[buf][c][ty - 1][tx - 1] = rn;
        }
      }
    };

    T fl[3][4], carry[3][4], own_lo[3], p0[3];
    LevelIn R0, R1, R2;
    EpiIn Q0, Q1, Q2;
    {
      LevelIn L0;
      load_level(ka0 - 1, L0);
      load_level(ka0, R0);
      load_level(ka0 + 1, R1);  // kaend >= ka0 + 2
      load_epi(ka0, Q1);        // finished by step 1
      if (st && st->done) return;  // group B leaves on the same flag
      const int b0 = (ka0 - 1) & 1;
      store_level(b0, L0);
      __syncthreads();  // barrier 0
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        own_lo[c] = suA[b0][c][ty][tx];
        fl[c][0] = own_lo[c];
        fl[c][1] = suA[b0][c][ty][tx + 1];
        fl[c][2] = suA[b0][c][ty + 1][tx + 1];
        fl[c][3] = suA[b0][c][ty + 1][tx];
        face4(fl[c]);
        carry[c][0] = carry[c][1] = carry[c][2] = carry[c][3] = T(0);
      }
    }
    // step s: brick layer ek = ka0 - 1 + s, then the node sums of level ek
    // (slot s % 3 of the rings is used, (s + 2) % 3 filled)
    auto step = [&](auto fn, int ek, const LevelIn& use, LevelIn& fill, const EpiIn& Pu, EpiIn& Pf) {
      const int bu = (ek + 1) & 1;
      store_level(bu, use);
      load_level(ek + 3, fill);
      load_epi(ek + 2, Pf);
      __syncthreads();
      T fu[3][4], lo[3][4];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        fu[c][0] = suA[bu][c][ty][tx];
        fu[c][1] = suA[bu][c][ty][tx + 1];
        fu[c][2] = suA[bu][c][ty + 1][tx + 1];
        fu[c][3] = suA[bu][c][ty + 1][tx];
      }
      T own_up[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) own_up[c] = fu[c][0];
      brick_layer(fl, fu, carry, use.Ee, wk, lo);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        p0[c] = lo[c][0];
        syA[0 + c][ty][tx] = lo[c][1];
        syA[3 + c][ty][tx] = lo[c][2];
        syA[6 + c][ty][tx] = lo[c][3];
      }
      __syncthreads();
      if constexpr (decltype(fn)::value) finish(ek, p0, own_lo, Pu);
#pragma unroll
      for (int c = 0; c < 3; ++c) own_lo[c] = own_up[c];
    };
    const int n = kaend - ka0 + 1;  // steps: layers ka0 - 1 .. kaend - 1 (n >= 3)
    step(skip, ka0 - 1, R0, R2, Q0, Q2);
    step(fin, ka0, R1, R0, Q1, Q0);
    int s = 2;
    for (; s + 3 <= n; s += 3) {
      step(fin, ka0 - 1 + s, R2, R1, Q2, Q1);
      step(fin, ka0 + s, R0, R2, Q0, Q2);
      step(fin, ka0 + 1 + s, R1, R0, Q1, Q0);
    }
    if (s < n) step(fin, ka0 - 1 + s, R2, R1, Q2, Q1);
    if (s + 1 < n) step(fin, ka0 + s, R0, R2, Q0, Q2);
    for (int b = 2 * n + 1; b < nbar; ++b) __syncthreads();  // group B is still marching
  } else {
    // ---- group B: step k + 1 on node columns I0 .. I0 + 15 (positions 0 .. 14
    // come from group A, 15 and 16 stay zero), owned 1 .. 13
    const int I0 = cx * OWN2 - 1, J0 = cy * OWN2 - 1;
    const int ni = I0 + tx, nj = J0 + ty;
    const bool owner = tx >= 1 && ty >= 1 && tx <= OWN2 && ty <= OWN2 && ni <= g.nx && nj <= g.ny;
    const bool ecol = ni >= 0 && ni < g.nx && nj >= 0 && nj < g.ny;
    for (int e = q; e < 2 * 3 * (TY + 1) * (TX + 1); e += TX * TY) {
      const int col = e % (TX + 1), row = (e / (TX + 1)) % (TY + 1);
      if (row > OWN2 + 1 || col > OWN2 + 1) (&suB[0][0][0][0])[e] = T(0);
    }
    // load ranges: owned node levels [K0, kend), brick layers [elo, ehi]
    const int elo = max(K0 - 1, 0), ehi = min(kend - 1, g.nz - 1);
    const int64_t nel = (int64_t)g.nx * g.ny, nlev = kend - K0;
    const __amdgpu_buffer_rsrc_t re =
        load_range(E + nel * elo, ehi >= elo ? nel * (ehi - elo + 1) * (int64_t)sizeof(T) : 0);
    const __amdgpu_buffer_rsrc_t rm = load_range(nmask + sxy * K0, sxy * nlev);
    const __amdgpu_buffer_rsrc_t rd = load_range(invd + sxy * K0, sxy * nlev * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t rac = load_range(acc + 3 * sxy * K0, 3 * sxy * nlev * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t rv = load_range(dk + 3 * sxy * K0, 3 * sxy * nlev * (int64_t)sizeof(T));
    const uint32_t o_el = off_part(ecol, ni + (int64_t)g.nx * nj);
    const uint32_t o_epi = off_part(owner, ni + sx * nj);
    auto load_E = [&](int ek) -> T {
      return load1(re, (o_el + lev_part(ek, elo, ehi - elo + 1, nel)) * (uint32_t)sizeof(T), T());
    };
    struct EpiIn {
      uint8_t m;
      T d;
      T a[3];  // iterate before step k
      T v[3];  // d_k
    };
    auto load_epi = [&](int k, EpiIn& P) {
      const uint32_t o = o_epi + lev_part(k, K0, kend - K0, sxy);
      P.m = load_u8(rm, o);
      P.d = load1(rd, o * (uint32_t)sizeof(T), T());
      load3(rac, o * (uint32_t)(3 * sizeof(T)), P.a);  // unused on the first step (no branch in the march)
      load3(rv, o * (uint32_t)(3 * sizeof(T)), P.v);
    };
    const int64_t lev0 = 3 * sxy * K0;
    const uint32_t chunk_bytes = (uint32_t)(3 * sxy * (kend - K0) * (int64_t)sizeof(T));
    const __amdgpu_buffer_rsrc_t rr = store_range(rout + lev0, chunk_bytes);
    const __amdgpu_buffer_rsrc_t ra = store_range(acc + lev0, chunk_bytes);
    const __amdgpu_buffer_rsrc_t ry = store_range(y + lev0, chunk_bytes);
    auto finish = [&](int k, const T (&p0)[3], const T (&own)[3], const T (&r1)[3], const EpiIn& P) {
      const bool mine = owner && k >= K0 && k < kend;
      const uint32_t at =
          mine ? (uint32_t)((ni + sx * nj + sxy * (k - K0)) * 3 * (int64_t)sizeof(T)) : kStoreDrop;
      T rn[3], an[3], dn[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T v = node_sum(p0[c], syB, c, ty, tx, tyl, txl);
        const bool fx = (P.m >> c) & 1;
        if (fx) v = T(0);
        cheb_dof(fx, r1[c], v, own[c], P.d, cf.c1b, cf.c2b, rn[c], dn[c]);
        an[c] = (cf.first ? P.v[c] : P.a[c] + P.v[c]) + own[c];
      }
      store3(rr, at, rn);
      store3(ra, at, an);
      store3(ry, at, dn);
    };
    // level k of d_{k+1} (zero off the mesh) and this node's r_{k+1}
    auto read_level = [&](int k, T (&fu)[3][4], T (&r1)[3]) {
      const bool in = k >= 0 && k <= g.nz;
      const int b = k & 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        fu[c][0] = in ? suB[b][c][ty][tx] : T(0);
        fu[c][1] = in ? suB[b][c][ty][tx + 1] : T(0);
        fu[c][2] = in ? suB[b][c][ty + 1][tx + 1] : T(0);
        fu[c][3] = in ? suB[b][c][ty + 1][tx] : T(0);
        r1[c] = srB[b][c][ty][tx];
      }
    };

    T fl[3][4], carry[3][4], own_lo[3], p0[3], r1_lo[3];
    T E0 = load_E(K0 - 1), E1 = load_E(K0), E2;  // layer K0 - 1 + s in slot s % 3
    EpiIn Q0, Q1, Q2;
    load_epi(K0, Q1);  // finished by step 1
    if (st && st->done) return;  // group A leaves on the same flag
    for (int b = 0; b < 5; ++b) __syncthreads();  // barriers 0 .. 4: group A's first levels
    __syncthreads();                                // barrier 5: level K0 - 1 of d_{k+1} is ready
    {
      T fu[3][4], r1[3];
      read_level(K0 - 1, fu, r1);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        own_lo[c] = fu[c][0];
#pragma unroll
        for (int i = 0; i < 4; ++i) fl[c][i] = fu[c][i];
        face4(fl[c]);
        r1_lo[c] = r1[c];
        carry[c][0] = carry[c][1] = carry[c][2] = carry[c][3] = T(0);
      }
    }
    __syncthreads();  // barrier 6
    // step s: brick layer ek = K0 - 1 + s, then the node sums of level ek
    auto step = [&](auto fn, int ek, T Ee, T& Efill, const EpiIn& Pu, EpiIn& Pf) {
      Efill = load_E(ek + 2);
      load_epi(ek + 2, Pf);
      __syncthreads();
      T fu[3][4], r1_up[3], own_up[3], lo[3][4];
      read_level(ek + 1, fu, r1_up);
#pragma unroll
      for (int c = 0; c < 3; ++c) own_up[c] = fu[c][0];
      brick_layer(fl, fu, carry, Ee, wk, lo);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        p0[c] = lo[c][0];
        syB[0 + c][ty][tx] = lo[c][1];
        syB[3 + c][ty][tx] = lo[c][2];
        syB[6 + c][ty][tx] = lo[c][3];
      }
      __syncthreads();
      if constexpr (decltype(fn)::value) finish(ek, p0, own_lo, r1_lo, Pu);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        own_lo[c] = own_up[c];
        r1_lo[c] = r1_up[c];
      }
    };
    const int n = kend - K0 + 1;  // steps: layers K0 - 1 .. kend - 1 (n >= 2)
    step(skip, K0 - 1, E0, E2, Q0, Q2);
    step(fin, K0, E1, E0, Q1, Q0);
    int s = 2;
    for (; s + 3 <= n; s += 3) {
      step(fin, K0 - 1 + s, E2, E1, Q2, Q1);
      step(fin, K0 + s, E0, E2, Q0, Q2);
      step(fin, K0 + 1 + s, E1, E0, Q1, Q0);
    }
    if (s < n) step(fin, K0 - 1 + s, E2, E1, Q2, Q1);
    if (s + 1 < n) step(fin, K0 + s, E0, E2, Q0, Q2);
  }
}

// ---------------------------------------------------------------------------
// Two coarsest-level Chebyshev steps in one launch on 3D tiles.
//
// The z-march above finishes a level per march step, so a workgroup's time is
// the length of its march; on the small coarsest grid (a few dozen levels in
// all) that chain, not arithmetic or bytes, sets the launch time.  Here a
// workgroup owns a 4 x 4 x OZ block of nodes (OZ = 4 or 8) and works on all
// of its levels at once.  It loads d_k, r_k, D^-1 and the masks of the
// 8 x 8 x (OZ + 4) nodes around the block (two-node halo; off the mesh: zero,
// every dof fixed) and the moduli of the 7 x 7 x (OZ + 3) bricks between them
// into LDS; then
//   step k:     every brick of the box computes its 24 products E_e Ke d_e
//               (one thread per brick, exact factorised operator) into LDS;
//               every node one node inside the halo sums the products of its
//               8 bricks (local corner order 0..7, a fixed order) and forms
//               r_{k+1}, d_{k+1};
//   step k + 1: the same on the 5 x 5 x (OZ + 1) bricks around the owned
//               block, whose corners all lie one node inside the halo;
// and the owned nodes store r_{k+2}, d_{k+2} and the iterate
// acc + d_k + d_{k+1}.  Four barriers per launch; no atomics, so the result is
// bitwise reproducible (its rounding differs from the march kernels', whose
// node sums run in another order).  Workgroup b takes tile (b % 8) * per +
// b / 8, so each XCD works on one contiguous run of tiles.
constexpr int C3_OWN = 4;  // owned nodes along x and y
constexpr int C3_IN = 8;   // input box nodes along x and y (two-node halo)

template <int OZ>
struct C3 {
  static constexpr int IN = C3_IN;                   // input box nodes along x and y
  static constexpr int IZ = OZ + 4;                  // input box nodes along z
  static constexpr int NIN = C3_IN * C3_IN * IZ;     // input box nodes
  static constexpr int B1X = C3_IN - 1, B1Z = IZ - 1;
  static constexpr int NB1 = B1X * B1X * B1Z;        // step-k bricks
  static constexpr int B2X = C3_OWN + 1, B2Z = OZ + 1;
  static constexpr int NB2 = B2X * B2X * B2Z;        // step-(k+1) bricks
  static constexpr int R1X = C3_OWN + 2, R1Z = OZ + 2;
  static constexpr int NR1 = R1X * R1X * R1Z;        // nodes of step k kept
  static constexpr int NOWN = C3_OWN * C3_OWN * OZ;  // owned nodes
  static constexpr int THREADS = (NB1 + 63) / 64 * 64;
};

// E_e Ke u_e of one brick from its corner values u (local corner order),
// in the same factorised form as brick_layer.
template <typename T>
__device__ inline void brick_full(T (&u)[3][8], T Ee, const WK<T>& wk, T (&yv)[3][8]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) walsh8(u[c]);
  WK<T> k = wk;
  k.A *= Ee; k.B *= Ee; k.G *= Ee; k.C *= Ee; k.D *= Ee; k.F *= Ee; k.H *= Ee; k.J *= Ee;
  T w[3][8];
  apply_S(k, u, w);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T lo[4], up[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      lo[i] = w[c][i] + w[c][i + 4];
      up[i] = w[c][i] - w[c][i + 4];
    }
    face4(lo);
    face4(up);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      yv[c][i] = lo[i];
      yv[c][i + 4] = up[i];
    }
  }
}

// Brick products of a box of BX x BX x BZ bricks whose lowest brick sits at
// local node (lo, lo, lo) of the input box (geometry G: G::IN nodes along x
// and y, moduli of its G::B1X x G::B1X x G::B1Z bricks): thread e computes
// brick e.
template <typename T, class G, int BX, int BZ>
__device__ inline void c3_bricks(const T (*sd)[G::NIN], const T* sE, int lo, const WK<T>& wk, T (*sbo)[G::NB1]) {
  const int e = threadIdx.x;
  if (e >= BX * BX * BZ) return;
  const int bi = lo + e % BX, bj = lo + (e / BX) % BX, bk = lo + e / (BX * BX);
  const int n0 = bi + G::IN * (bj + G::IN * bk);
  T u[3][8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int n = n0 + kCornerX[a] + G::IN * (kCornerY[a] + G::IN * kCornerZ[a]);
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c][a] = sd[c][n];
  }
  T yv[3][8];
  brick_full(u, sE[bi + G::B1X * (bj + G::B1X * bk)], wk, yv);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 8; ++a) sbo[c * 8 + a][e] = yv[c][a];
}

// (K d)_c at local node (li, lj, lk) from the brick products of a box of
// BX x BX x BZ bricks starting at local node lo: the 8 bricks holding the
// node, in local corner order.
template <typename T, class G, int BX>
__device__ inline T c3_node_sum(const T (*sbo)[G::NB1], int c, int li, int lj, int lk, int lo) {
  T v = T(0);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int e = (li - lo - kCornerX[a]) + BX * ((lj - lo - kCornerY[a]) + BX * (lk - lo - kCornerZ[a]));
    v = v + sbo[c * 8 + a][e];
  }
  return v;
}

template <typename T, int OZ>
__global__ void __launch_bounds__(C3<OZ>::THREADS) cheb3d_kernel(Grid g, int gx, int gy, int nblk, int per,
                                                                const T* __restrict__ dk,
                                                                const T* __restrict__ E,
                                                                const uint8_t* __restrict__ nmask, WK<T> wk,
                                                                const T* __restrict__ invd,
                                                                const T* __restrict__ rin, T* __restrict__ rout,
                                                                T* __restrict__ acc, T* __restrict__ y,
                                                                Cheb2<T> cf, CgState* st, int64_t wsh) {
  using Q = C3<OZ>;
  static_assert(Q::NIN <= 2 * Q::THREADS && Q::NR1 <= Q::THREADS && Q::NOWN <= Q::THREADS,
                "one or two passes cover every phase");
  static_assert(sizeof(T) * (10 * Q::NIN + 25 * Q::NB1) + Q::NIN <= 160 * 1024, "LDS of one workgroup");
  if (wsh) {  // batched launch: this workgroup's problem
    const int64_t o = batch_offset(wsh);
    dk = wshift(dk, o);
    E = wshift(E, o);
    nmask = wshift(nmask, o);
    invd = wshift(invd, o);
    rin = wshift(rin, o);
    rout = wshift(rout, o);
    acc = wshift(acc, o);
    y = wshift(y, o);
    st = wshift(st, o);
  }
  const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (tile >= nblk) return;
  __shared__ T sD0[3][Q::NIN], sD1[3][Q::NIN], sR[3][Q::NIN], sInv[Q::NIN], sE[Q::NB1];
  __shared__ T sBO[24][Q::NB1];
  __shared__ uint8_t sM[Q::NIN];
  const int tx = tile % gx, t1 = tile / gx, ty = t1 % gy, tz = t1 / gy;
  const int I0 = tx * C3_OWN - 2, J0 = ty * C3_OWN - 2, K0 = tz * OZ - 2;
  const int64_t sx = g.nx + 1, sxy = sx * (g.ny + 1);
  const int tid = threadIdx.x;
  // the iterate at the owned node this thread finishes (threads 0 .. NOWN - 1)
  int oi = 0, oj = 0, ok = 0;
  bool own_in = false;
  int64_t own_node = 0;
  T a0[3] = {T(0), T(0), T(0)};
  if (tid < Q::NOWN) {
    oi = 2 + tid % C3_OWN;
    oj = 2 + (tid / C3_OWN) % C3_OWN;
    ok = 2 + tid / (C3_OWN * C3_OWN);
    const int i = I0 + oi, j = J0 + oj, k = K0 + ok;
    own_in = i <= g.nx && j <= g.ny && k <= g.nz;  // owned nodes are never below the mesh
    own_node = i + sx * j + sxy * k;
    if (own_in && !cf.first) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a0[c] = acc[3 * own_node + c];
    }
  }
  // every load of the launch is issued before the first wait: node tid and
  // node tid + THREADS of the box, brick tid's modulus (one memory round
  // trip for the whole prologue)
  struct NodeIn {
    T d[3], r[3], iv;
    uint8_t m;
  };
  const bool form_d = cf.dscale != T(0);
  auto load_node = [&](int n, NodeIn& v) {
    const int i = I0 + n % C3_IN, j = J0 + (n / C3_IN) % C3_IN, k = K0 + n / (C3_IN * C3_IN);
    const bool in = n < Q::NIN && i >= 0 && i <= g.nx && j >= 0 && j <= g.ny && k >= 0 && k <= g.nz;
#pragma unroll
    for (int c = 0; c < 3; ++c) v.d[c] = v.r[c] = T(0);
    v.iv = T(0);
    v.m = 7;
    if (in) {
      const int64_t node = i + sx * j + sxy * k;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (!form_d) v.d[c] = dk[3 * node + c];
        v.r[c] = rin[3 * node + c];
      }
      v.iv = invd[node];
      v.m = nmask[node];
    }
  };
  // the formed first direction rounds as the separate first-direction launch does
  auto store_node = [&](int n, const NodeIn& v) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sD0[c][n] = form_d ? cf.dscale * v.iv * v.r[c] : v.d[c];
      sR[c][n] = v.r[c];
    }
    sInv[n] = v.iv;
    sM[n] = v.m;
  };
  NodeIn v0, v1;
  load_node(tid, v0);
  load_node(tid + Q::THREADS, v1);
  T Eb = T(0);
  {
    const int i = I0 + tid % Q::B1X, j = J0 + (tid / Q::B1X) % Q::B1X, k = K0 + tid / (Q::B1X * Q::B1X);
    if (tid < Q::NB1 && i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz)
      Eb = E[i + (int64_t)g.nx * (j + (int64_t)g.ny * k)];
  }
  // the CG stop flag is read while the loads are in flight
  if (st && st->done) return;
  if (tid < Q::NIN) store_node(tid, v0);
  if (tid + Q::THREADS < Q::NIN) store_node(tid + Q::THREADS, v1);
  if (tid < Q::NB1) sE[tid] = Eb;
  __syncthreads();
  // step k on the bricks of the box
  c3_bricks<T, Q, Q::B1X, Q::B1Z>(sD0, sE, 0, wk, sBO);
  __syncthreads();
  // r_{k+1}, d_{k+1} on the nodes one inside the halo
  if (tid < Q::NR1) {
    const int li = 1 + tid % Q::R1X, lj = 1 + (tid / Q::R1X) % Q::R1X, lk = 1 + tid / (Q::R1X * Q::R1X);
    const int n = li + C3_IN * (lj + C3_IN * lk);
    const uint8_t m = sM[n];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const bool fx = (m >> c) & 1;
      T v = c3_node_sum<T, Q, Q::B1X>(sBO, c, li, lj, lk, 0);
      if (fx) v = T(0);
      T rn, dn;
      cheb_dof(fx, sR[c][n], v, sD0[c][n], sInv[n], cf.c1a, cf.c2a, rn, dn);
      sR[c][n] = rn;
      sD1[c][n] = dn;
    }
  }
  __syncthreads();
  // step k + 1 on the bricks around the owned block
  c3_bricks<T, Q, Q::B2X, Q::B2Z>(sD1, sE, 1, wk, sBO);
  __syncthreads();
  if (tid < Q::NOWN && own_in) {
    const int n = oi + C3_IN * (oj + C3_IN * ok);
    const uint8_t m = sM[n];
    T rn[3], dn[3], an[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const bool fx = (m >> c) & 1;
      T v = c3_node_sum<T, Q, Q::B2X>(sBO, c, oi, oj, ok, 1);
      if (fx) v = T(0);
      cheb_dof(fx, sR[c][n], v, sD1[c][n], sInv[n], cf.c1b, cf.c2b, rn[c], dn[c]);
      an[c] = (cf.first ? sD0[c][n] : a0[c] + sD0[c][n]) + sD1[c][n];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      rout[3 * own_node + c] = rn[c];
      acc[3 * own_node + c] = an[c];
      y[3 * own_node + c] = dn[c];
    }
  }
}

// Three steps of the coarsest-level Chebyshev iteration in one launch, on
// OX x OY x OZ owned nodes with a three-node halo (an (OX + 6) x (OY + 6) x
// (OZ + 6) node box): the bricks of step k on all bricks of the box, the
// node updates one node inside, step k + 1 on the bricks one inside and the
// nodes two inside, step k + 2 on the bricks around the owned block and the
// owned nodes.  Each phase is the pair kernel's (same brick products, node
// sums in the same corner order, same per-dof update), so three steps here
// are bitwise two launches of that kernel's steps plus one, in any
// grouping, for any block shape.  float32 only (the brick products of a
// 4 x 4 x 4 block fill 70 KB of LDS; float64 ones would not fit with the
// box).
template <int OX, int OY, int OZ>
struct C3T {
  static constexpr int IX = OX + 6, IY = OY + 6, IZ = OZ + 6;  // box nodes per axis
  static constexpr int NIN = IX * IY * IZ;
  static constexpr int B1X = IX - 1, B1Y = IY - 1, B1Z = IZ - 1;
  static constexpr int NB1 = B1X * B1Y * B1Z;  // step-k bricks
  static constexpr int THREADS = (NB1 + 63) / 64 * 64;
  static constexpr int NOWN = OX * OY * OZ;
};

// Brick products of the BX x BY x BZ bricks from local node (lo, lo, lo) of
// a box of geometry G (moduli of its B1X x B1Y x B1Z bricks): thread e
// computes brick e.
template <typename T, class G, int BX, int BY, int BZ>
__device__ inline void box_bricks(const T (*sd)[G::NIN], const T* sE, int lo, const WK<T>& wk, T (*sbo)[G::NB1]) {
  const int e = threadIdx.x;
  if (e >= BX * BY * BZ) return;
  const int bi = lo + e % BX, bj = lo + (e / BX) % BY, bk = lo + e / (BX * BY);
  const int n0 = bi + G::IX * (bj + G::IY * bk);
  T u[3][8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int n = n0 + kCornerX[a] + G::IX * (kCornerY[a] + G::IY * kCornerZ[a]);
#pragma unroll
    for (int c = 0; c < 3; ++c) u[c][a] = sd[c][n];
  }
  T yv[3][8];
  brick_full(u, sE[bi + G::B1X * (bj + G::B1Y * bk)], wk, yv);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < 8; ++a) sbo[c * 8 + a][e] = yv[c][a];
}

// (K d)_c at local node (li, lj, lk) from the products of the BX x BY x ...
// bricks starting at local node lo: its 8 bricks in local corner order.
template <typename T, class G, int BX, int BY>
__device__ inline T box_node_sum(const T (*sbo)[G::NB1], int c, int li, int lj, int lk, int lo) {
  T v = T(0);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int e = (li - lo - kCornerX[a]) + BX * ((lj - lo - kCornerY[a]) + BY * (lk - lo - kCornerZ[a]));
    v = v + sbo[c * 8 + a][e];
  }
  return v;
}

template <int OX, int OY, int OZ>
__global__ void __launch_bounds__((C3T<OX, OY, OZ>::THREADS)) cheb3t_kernel(
    Grid g, int gx, int gy, int nblk, int per, const float* __restrict__ dk, const float* __restrict__ E,
    const uint8_t* __restrict__ nmask, WK<float> wk, const float* __restrict__ invd, const float* __restrict__ rin,
    float* __restrict__ rout, float* __restrict__ acc, float* __restrict__ y, Cheb2<float> cf, CgState* st,
    int64_t wsh) {
  using Q = C3T<OX, OY, OZ>;
  using T = float;
  static_assert(Q::NIN <= 2 * Q::THREADS, "two passes cover the box");
  static_assert((Q::IX - 2) * (Q::IY - 2) * (Q::IZ - 2) <= Q::THREADS, "one pass covers the first node phase");
  static_assert(sizeof(T) * (10 * Q::NIN + 25 * Q::NB1) + Q::NIN <= 160 * 1024, "LDS of one workgroup");
  if (wsh) {  // batched launch: this workgroup's problem
    const int64_t o = batch_offset(wsh);
    dk = wshift(dk, o);
    E = wshift(E, o);
    nmask = wshift(nmask, o);
    invd = wshift(invd, o);
    rin = wshift(rin, o);
    rout = wshift(rout, o);
    acc = wshift(acc, o);
    y = wshift(y, o);
    st = wshift(st, o);
  }
  const int tile = (int)(blockIdx.x % 8) * per + (int)(blockIdx.x / 8);
  if (tile >= nblk) return;
  // sD0 holds d_k, then d_{k+2}; sD1 d_{k+1}; sR the running residual
  __shared__ T sD0[3][Q::NIN], sD1[3][Q::NIN], sR[3][Q::NIN], sInv[Q::NIN], sE[Q::NB1];
  __shared__ T sBO[24][Q::NB1];
  __shared__ uint8_t sM[Q::NIN];
  const int tx = tile % gx, t1 = tile / gx, ty = t1 % gy, tz = t1 / gy;
  const int I0 = tx * OX - 3, J0 = ty * OY - 3, K0 = tz * OZ - 3;
  const int64_t sx = g.nx + 1, sxy = sx * (g.ny + 1);
  const int tid = threadIdx.x;
  int oi = 0, oj = 0, ok = 0;
  bool own_in = false;
  int64_t own_node = 0;
  T a0[3] = {T(0), T(0), T(0)};
  if (tid < Q::NOWN) {
    oi = 3 + tid % OX;
    oj = 3 + (tid / OX) % OY;
    ok = 3 + tid / (OX * OY);
    const int i = I0 + oi, j = J0 + oj, k = K0 + ok;
    own_in = i <= g.nx && j <= g.ny && k <= g.nz;  // owned nodes are never below the mesh
    own_node = i + sx * j + sxy * k;
    if (own_in && !cf.first) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a0[c] = acc[3 * own_node + c];
    }
  }
  // every load is issued before the first wait (one memory round trip)
  struct NodeIn {
    T d[3], r[3], iv;
    uint8_t m;
  };
  const bool form_d = cf.dscale != T(0);
  auto load_node = [&](int n, NodeIn& v) {
    const int i = I0 + n % Q::IX, j = J0 + (n / Q::IX) % Q::IY, k = K0 + n / (Q::IX * Q::IY);
    const bool in = n < Q::NIN && i >= 0 && i <= g.nx && j >= 0 && j <= g.ny && k >= 0 && k <= g.nz;
#pragma unroll
    for (int c = 0; c < 3; ++c) v.d[c] = v.r[c] = T(0);
    v.iv = T(0);
    v.m = 7;
    if (in) {
      const int64_t node = i + sx * j + sxy * k;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (!form_d) v.d[c] = dk[3 * node + c];
        v.r[c] = rin[3 * node + c];
      }
      v.iv = invd[node];
      v.m = nmask[node];
    }
  };
  // the formed first direction rounds as the separate first-direction launch does
  auto store_node = [&](int n, const NodeIn& v) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      sD0[c][n] = form_d ? cf.dscale * v.iv * v.r[c] : v.d[c];
      sR[c][n] = v.r[c];
    }
    sInv[n] = v.iv;
    sM[n] = v.m;
  };
  NodeIn v0, v1;
  load_node(tid, v0);
  load_node(tid + Q::THREADS, v1);
  T Eb = T(0);
  {
    const int i = I0 + tid % Q::B1X, j = J0 + (tid / Q::B1X) % Q::B1Y, k = K0 + tid / (Q::B1X * Q::B1Y);
    if (tid < Q::NB1 && i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz)
      Eb = E[i + (int64_t)g.nx * (j + (int64_t)g.ny * k)];
  }
  // the CG stop flag is read while the loads are in flight
  if (st && st->done) return;
  if (tid < Q::NIN) store_node(tid, v0);
  if (tid + Q::THREADS < Q::NIN) store_node(tid + Q::THREADS, v1);
  if (tid < Q::NB1) sE[tid] = Eb;
  __syncthreads();
  // d_k at the owned node, before its buffer takes d_{k+2}
  T d0own[3] = {T(0), T(0), T(0)};
  if (tid < Q::NOWN) {
    const int n = oi + Q::IX * (oj + Q::IY * ok);
#pragma unroll
    for (int c = 0; c < 3; ++c) d0own[c] = sD0[c][n];
  }
  // one step on the NX x NY x NZ nodes from local node lo + 1: residual and
  // direction from the bricks of the box one larger from lo (in sBO), d from
  // din to dout
  auto node_step = [&](auto nx_c, auto ny_c, auto nz_c, int lo, const T (*din)[Q::NIN], T (*dout)[Q::NIN], T c1,
                       T c2) {
    constexpr int NX = decltype(nx_c)::value, NY = decltype(ny_c)::value, NZ = decltype(nz_c)::value;
    if (tid < NX * NY * NZ) {
      const int li = lo + 1 + tid % NX, lj = lo + 1 + (tid / NX) % NY, lk = lo + 1 + tid / (NX * NY);
      const int n = li + Q::IX * (lj + Q::IY * lk);
      const uint8_t m = sM[n];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const bool fx = (m >> c) & 1;
        T v = box_node_sum<T, Q, NX + 1, NY + 1>(sBO, c, li, lj, lk, lo);
        if (fx) v = T(0);
        T rn, dn;
        cheb_dof(fx, sR[c][n], v, din[c][n], sInv[n], c1, c2, rn, dn);
        sR[c][n] = rn;
        dout[c][n] = dn;
      }
    }
  };
  // step k: bricks of the box, nodes one inside
  box_bricks<T, Q, Q::B1X, Q::B1Y, Q::B1Z>(sD0, sE, 0, wk, sBO);
  __syncthreads();
  node_step(std::integral_constant<int, OX + 4>{}, std::integral_constant<int, OY + 4>{},
            std::integral_constant<int, OZ + 4>{}, 0, sD0, sD1, cf.c1a, cf.c2a);
  __syncthreads();
  // step k + 1: bricks one inside, nodes two inside (d_{k+2} into sD0)
  box_bricks<T, Q, OX + 3, OY + 3, OZ + 3>(sD1, sE, 1, wk, sBO);
  __syncthreads();
  node_step(std::integral_constant<int, OX + 2>{}, std::integral_constant<int, OY + 2>{},
            std::integral_constant<int, OZ + 2>{}, 1, sD1, sD0, cf.c1b, cf.c2b);
  __syncthreads();
  // step k + 2: bricks around the owned block, the owned nodes
  box_bricks<T, Q, OX + 1, OY + 1, OZ + 1>(sD0, sE, 2, wk, sBO);
  __syncthreads();
  if (tid < Q::NOWN && own_in) {
    const int n = oi + Q::IX * (oj + Q::IY * ok);
    const uint8_t m = sM[n];
    T rn[3], dn[3], an[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const bool fx = (m >> c) & 1;
      T v = box_node_sum<T, Q, OX + 1, OY + 1>(sBO, c, oi, oj, ok, 2);
      if (fx) v = T(0);
      cheb_dof(fx, sR[c][n], v, sD0[c][n], sInv[n], cf.c1c, cf.c2c, rn[c], dn[c]);
      an[c] = ((cf.first ? d0own[c] : a0[c] + d0own[c]) + sD1[c][n]) + sD0[c][n];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      rout[3 * own_node + c] = rn[c];
      acc[3 * own_node + c] = an[c];
      y[3 * own_node + c] = dn[c];
    }
  }
}

// ---------------------------------------------------------------------------
// The same operator with the brick contraction Ke u_e on bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16, float32 accumulation), float32 vectors.
//
// A wave holds 4 x 16 brick columns of the tile.  For each of its four rows t
// (an N-tile of 16 bricks) the product is D (32 x 16) = Ke_pad (32 x 32) *
// U_t (32 x 16), with the dof index of Ke_pad and U_t ordered 4 * corner +
// component (slot 3 of each corner is zero padding).  In the operand layout
// lane group g (lanes 16g .. 16g+15) supplies k = 8g .. 8g+7, i.e. corners
// 2g and 2g+1 of its brick, read straight from the two LDS level buffers; in
// the result layout the same lane receives rows 4g .. 4g+3 of each 16-row
// M-tile, i.e. the three components of corner g (lower level, M-tile 0) and
// corner 4 + g (upper level, M-tile 1) of its brick -- exactly what the
// z-carry and the node sums need.
//
// Rigid motion is removed before rounding.  Ke annihilates the six rigid
// modes, so subtracting any translation plus infinitesimal rotation w x p
// from all eight corners leaves the exact product unchanged.  The kernel
// subtracts corner 0 and the rotation estimated from the three edges at
// corner 0 (every lane of a brick reads the same six values, so the whole
// brick sees one rigid field).  Rounding then acts on the deformation of the
// brick alone, and the bf16 error of Ke along the rigid modes -- which the
// rotations of a bending structure would otherwise amplify far beyond the
// strain energy -- never enters.
//
// SPLIT: both operands as a pair of bf16 numbers (hi + lo, about 16
// significant bits each); the product keeps hi*hi + lo*hi + hi*lo (three
// matrix-core passes), i.e. the split-bf16 product of Henry, Tang and
// Heinecke (2019) with one cross term fewer than their six-term form.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int MODE, bool SPLIT>
__global__ void __launch_bounds__(TX* TY) kxu_mfma_kernel(Grid g, TileMap tm, const float* __restrict__ x,
                                                         const float* __restrict__ E,
                                                         const uint8_t* __restrict__ nmask,
                                                         const float* __restrict__ ke, float kscale,
                                                         float* __restrict__ y, Epi<float> ep, CgState* st,
                                                         double* partials) {
  if ((MODE == 1 || MODE == 5 || st) && st->done) return;
  __shared__ float su[2][3][TY + 1][TX + 1];  // two node levels
  __shared__ float sy[4][3][TY][TX];          // level partials per corner
  __shared__ float sE[TY][TX];

  int cx, cy, cz;
  tile_of_block(tm, cx, cy, cz);
  const int kc = tm.kc;
  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane >> 4, ln = lane & 15;
  const int I0 = cx * OWN - 1, J0 = cy * OWN - 1, K0 = cz * kc;
  const int ni = I0 + tx, nj = J0 + ty;
  const int64_t sx = g.nx + 1, sxy = (int64_t)(g.nx + 1) * (g.ny + 1);
  const bool owner = tx >= 1 && ty >= 1 && ni <= g.nx && nj <= g.ny;
  const bool ecol = ni >= 0 && ni < g.nx && nj >= 0 && nj < g.ny;
  const int kend = min(K0 + kc, g.nz + 1);

  // Ke_pad rows 16 mt + ln, columns 8 grp .. 8 grp + 7 (bf16), in registers
  bf16x8 a[2], alo[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int m = 16 * mt + ln, cm = m >> 2, am = m & 3;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = 8 * grp + i, ck = k >> 2, ak = k & 3;
      const float v = (am < 3 && ak < 3) ? ke[(3 * cm + am) * 24 + 3 * ck + ak] * kscale : 0.0f;
      a[mt][i] = (__bf16)v;
      alo[mt][i] = (__bf16)(v - (float)a[mt][i]);
    }
  }

  auto node_ok = [&](int i, int j, int k) {
    return i >= 0 && i <= g.nx && j >= 0 && j <= g.ny && k >= 0 && k <= g.nz;
  };
  struct LevelRegs {
    float own[3];
    float ext[3][3];
  };
  const bool ex0 = tx == TX - 1, ex1 = ty == TY - 1, ex2 = ex0 && ex1;
  auto fetch = [&](int i, int j, int k, float (&v)[3]) {
    if (node_ok(i, j, k)) {
      const int64_t n = i + sx * j + sxy * k;
      v[0] = x[3 * n];
      v[1] = x[3 * n + 1];
      v[2] = x[3 * n + 2];
    } else {
      v[0] = v[1] = v[2] = 0.0f;
    }
  };
  auto load_regs = [&](int k, LevelRegs& L) {
    fetch(ni, nj, k, L.own);
    if (ex0) fetch(I0 + TX, nj, k, L.ext[0]);
    if (ex1) fetch(ni, J0 + TY, k, L.ext[1]);
    if (ex2) fetch(I0 + TX, J0 + TY, k, L.ext[2]);
  };
  auto store_lds = [&](int buf, const LevelRegs& L) {
#pragma unroll
    for (int c = 0; c < 3; ++c) su[buf][c][ty][tx] = L.own[c];
    if (ex0)
      for (int c = 0; c < 3; ++c) su[buf][c][ty][TX] = L.ext[0][c];
    if (ex1)
      for (int c = 0; c < 3; ++c) su[buf][c][TY][tx] = L.ext[1][c];
    if (ex2)
      for (int c = 0; c < 3; ++c) su[buf][c][TY][TX] = L.ext[2][c];
  };
  auto modulus = [&](int ek) -> float {
    return (ecol && ek >= 0 && ek < g.nz) ? E[ni + (int64_t)g.nx * (nj + (int64_t)g.ny * ek)] : 0.0f;
  };

  // lane group grp supplies corners 2 grp and 2 grp + 1: (0,0),(1,0) for
  // grp 0 and 2, (1,1),(0,1) for grp 1 and 3, on the upper level for grp >= 2
  const int oxA = grp & 1, oyA = grp & 1, oxB = 1 - (grp & 1), oyB = grp & 1, upper = grp >= 2;

  float carry[4][3];  // upper-corner outputs of the brick below, per row t
  float own_prev[3];
  LevelRegs nxt;
  float Enxt;
  {
    LevelRegs L0;
    load_regs(K0 - 1, L0);
    load_regs(K0, nxt);
    Enxt = modulus(K0 - 1);
    store_lds((K0 - 1) & 1, L0);
#pragma unroll
    for (int c = 0; c < 3; ++c) own_prev[c] = L0.own[c];
#pragma unroll
    for (int t = 0; t < 4; ++t) carry[t][0] = carry[t][1] = carry[t][2] = 0.0f;
  }

  double dot = 0.0;
  for (int s = 0; s <= kc; ++s) {
    const int ek = K0 - 1 + s;
    if (ek >= g.nz + 1) break;  // uniform
    const LevelRegs cur = nxt;
    const int blo = ek & 1, bhi = (ek + 1) & 1;
    store_lds(bhi, cur);
    sE[ty][tx] = Enxt;
    if (s < kc) {
      load_regs(ek + 2, nxt);
      Enxt = modulus(ek + 1);
    }
    __syncthreads();

#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = 4 * wave + t;  // brick row of this N-tile inside the tile
      const int b = upper ? bhi : blo;
      // rigid field of the brick: corner 0 and the edge-estimated rotation w
      float ref[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) ref[c] = su[blo][c][r][ln];
      const float wz = 0.5f * ((su[blo][1][r][ln + 1] - ref[1]) - (su[blo][0][r + 1][ln] - ref[0]));
      const float wy = 0.5f * ((su[bhi][0][r][ln] - ref[0]) - (su[blo][2][r][ln + 1] - ref[2]));
      const float wx = 0.5f * ((su[blo][2][r + 1][ln] - ref[2]) - (su[bhi][1][r][ln] - ref[1]));
      const float pz = upper ? 1.0f : 0.0f;
      float dA[3], dB[3];  // w x p at the two corners
      dA[0] = wy * pz - wz * oyA;
      dA[1] = wz * oxA - wx * pz;
      dA[2] = wx * oyA - wy * oxA;
      dB[0] = wy * pz - wz * oyB;
      dB[1] = wz * oxB - wx * pz;
      dB[2] = wx * oyB - wy * oxB;
      bf16x8 bv, bl;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float vA = su[b][c][r + oyA][ln + oxA] - ref[c] - dA[c];
        const float vB = su[b][c][r + oyB][ln + oxB] - ref[c] - dB[c];
        bv[c] = (__bf16)vA;
        bv[4 + c] = (__bf16)vB;
        if (SPLIT) {
          bl[c] = (__bf16)(vA - (float)bv[c]);
          bl[4 + c] = (__bf16)(vB - (float)bv[4 + c]);
        }
      }
      bv[3] = bv[7] = (__bf16)0.0f;
      const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
      f32x4 dlo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bv, zero, 0, 0, 0);
      f32x4 dhi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], bv, zero, 0, 0, 0);
      if (SPLIT) {
        bl[3] = bl[7] = (__bf16)0.0f;
        dlo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[0], bv, dlo, 0, 0, 0);
        dhi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[1], bv, dhi, 0, 0, 0);
        dlo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bl, dlo, 0, 0, 0);
        dhi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], bl, dhi, 0, 0, 0);
      }
      const float Ee = sE[r][ln];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        sy[grp][c][r][ln] = carry[t][c] + Ee * dlo[c];
        carry[t][c] = Ee * dhi[c];
      }
    }
    __syncthreads();
    if (s >= 1 && owner && ek >= K0 && ek < kend) {
      const int64_t n = ni + sx * nj + sxy * ek;
      const uint8_t m = nmask[n];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        float v2 = sy[0][c][ty][tx] + sy[1][c][ty][tx - 1] + sy[2][c][ty - 1][tx - 1] + sy[3][c][ty - 1][tx];
        const bool fx = (m >> c) & 1;
        if (fx) v2 = 0.0f;
        if (MODE == 1) {
          dot += (double)own_prev[c] * (double)v2;
        } else if (MODE == 3 || MODE == 5) {
          const float bvv = ep.bT[3 * n + c];
          v2 = fx ? 0.0f : own_prev[c] + ep.omega * ep.invd[n] * (bvv - v2);
          if (MODE == 5) dot += (double)bvv * (double)v2;
        } else if (MODE == 4) {
          v2 = fx ? 0.0f : ep.bT[3 * n + c] - v2;
        }
        y[3 * n + c] = v2;
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) own_prev[c] = cur.own[c];
  }
  if (MODE == 0 || MODE == 3 || MODE == 4) return;
  double vv[1] = {dot};
  block_partials<1>(vv, partials);
}

template <typename T>
WK<T> scaled_wk(const WalshK& w, double h) {
  WK<T> k;
  k.A = (T)(w.A * h); k.B = (T)(w.B * h); k.G = (T)(w.G * h); k.C = (T)(w.C * h);
  k.D = (T)(w.D * h); k.F = (T)(w.F * h); k.H = (T)(w.H * h); k.J = (T)(w.J * h);
  return k;
}

}  // namespace

#ifndef FE_KXU_KCMAX
#define FE_KXU_KCMAX 16  // most node levels one workgroup marches through
#endif

// Resident workgroups per compute unit of a kernel on the current device
// (cached per device and kernel).
// Compute units of the current device (cached per device).
static int device_cus() {
  static std::mutex mu;
  static std::map<int, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it != cache.end()) return it->second;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  (void)hipGetLastError();
  cache[dev] = cus;
  return cus;
}

static int kxu_slots(const void* kernel, int threads = TX * TY) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({dev, kernel});
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 1;
  (void)hipGetLastError();
  const int slots = per_cu * cus;
  cache[{dev, kernel}] = slots;
  return slots;
}

// Tiles of 15 x 15 node columns, split in z into chunks of kc levels so that
// the workgroups fill whole rounds of the resident slots (no lone tail
// round) with at most FE_KXU_KCMAX levels each.
static TileMap kxu_tile_map(const Grid& g, int slots, int own = OWN) {
  TileMap tm;
  tm.gx = (g.nx + 1 + own - 1) / own;
  tm.gy = (g.ny + 1 + own - 1) / own;
  const int64_t cols = (int64_t)tm.gx * tm.gy, L = g.nz + 1;
  const int64_t rounds = std::max<int64_t>(1, (cols * L + (int64_t)slots * FE_KXU_KCMAX - 1) /
                                                  ((int64_t)slots * FE_KXU_KCMAX));
  int64_t nzc = std::max<int64_t>(1, std::min<int64_t>(L, rounds * slots / cols));
  // the stores address a chunk's levels with 31-bit byte offsets, the loads
  // index fewer than kOffIndex nodes (kc + 2 levels)
  const int64_t sxy = (int64_t)(g.nx + 1) * (g.ny + 1);
  const int64_t kc_fit =
      std::max<int64_t>(1, std::min<int64_t>(((int64_t)1 << 31) / (24 * sxy), (int64_t)kOffIndex / sxy - 4));
  tm.kc = (int)std::min<int64_t>((L + nzc - 1) / nzc, kc_fit);
  tm.nzc = (int)((L + tm.kc - 1) / tm.kc);
  tm.nblk = (int)(cols * tm.nzc);
  return tm;
}

// Upper bound of the workgroup count of any tile map of g (partials sizing).
int64_t kxu_tile_blocks(const Grid& g) {
  return (int64_t)((g.nx + 1 + OWN - 1) / OWN) * ((g.ny + 1 + OWN - 1) / OWN) * (g.nz + 1);
}

template <typename T, int MODE, int XIN>
static int launch_tile(hipStream_t stream, const Grid& g, const T* x, const T* E, const uint8_t* nm,
                       const WK<T>& wk, T* y, const Epi<T>& ep, CgState* st, double* partials, double* out,
                       const T* zpad, const XinK<T>& xi, const FoldK& fo, int bcount, int64_t bstride) {
  const void* k = reinterpret_cast<const void*>(&kxu_tile_kernel<T, MODE, XIN>);
  const TileMap tm = kxu_tile_map(g, kxu_slots(k));
  if (3 * (int64_t)(g.nx + 1) * (g.ny + 1) * tm.kc * (int64_t)sizeof(T) >= ((int64_t)1 << 31) ||
      (int64_t)(g.nx + 1) * (g.ny + 1) * (tm.kc + 4) >= (int64_t)kOffIndex)
    return -1;
  hipLaunchKernelGGL((kxu_tile_kernel<T, MODE, XIN>), dim3(tm.nblk, bcount), dim3(TX * TY), 0, stream, g, tm, x,
                     E, nm, wk, y, ep, st, partials, out, zpad, xi, fo, bcount > 1 ? bstride : (int64_t)0);
  return tm.nblk;
}

template <int MODE, bool SPLIT>
static int launch_mfma_mode(hipStream_t stream, const Grid& g, const float* x, const float* E,
                            const uint8_t* nm, const float* ke, float ks, float* y, const Epi<float>& ef,
                            CgState* st, double* partials) {
  const void* k = reinterpret_cast<const void*>(&kxu_mfma_kernel<MODE, SPLIT>);
  const TileMap tm = kxu_tile_map(g, kxu_slots(k));
  hipLaunchKernelGGL((kxu_mfma_kernel<MODE, SPLIT>), dim3(tm.nblk), dim3(TX * TY), 0, stream, g, tm, x, E, nm,
                     ke, ks, y, ef, st, partials);
  return tm.nblk;
}

template <bool SPLIT>
static int launch_mfma(int mode, hipStream_t stream, const Grid& g, const float* x, const float* E,
                       const uint8_t* nm, const float* ke, float ks, float* y, const Epi<float>& ef, CgState* st,
                       double* partials) {
  switch (mode) {
    case 1: return launch_mfma_mode<1, SPLIT>(stream, g, x, E, nm, ke, ks, y, ef, st, partials);
    case 3: return launch_mfma_mode<3, SPLIT>(stream, g, x, E, nm, ke, ks, y, ef, st, partials);
    case 4: return launch_mfma_mode<4, SPLIT>(stream, g, x, E, nm, ke, ks, y, ef, st, partials);
    case 5: return launch_mfma_mode<5, SPLIT>(stream, g, x, E, nm, ke, ks, y, ef, st, partials);
    default: return launch_mfma_mode<0, SPLIT>(stream, g, x, E, nm, ke, ks, y, ef, st, partials);
  }
}

// Workgroups of the level-`lev` launch of the last smoothing sweep with
// r^T z (mode 5, plain operand): the count of r^T z partials it leaves.
template <typename T>
int kxu_rz_partials(const fe_problem* p, int lev) {
  const void* k = reinterpret_cast<const void*>(&kxu_tile_kernel<T, 5, 0>);
  return kxu_tile_map(p->L[lev].g, kxu_slots(k)).nblk;
}
template int kxu_rz_partials<double>(const fe_problem*, int);
template int kxu_rz_partials<float>(const fe_problem*, int);

// Launch form of a pair of coarse Chebyshev steps on level lev (see fe_set_coarse_fusion).
static int cheb2_form(const fe_problem* p, int lev, bool tall) {
  const Grid g = p->L[lev].g;
  const int gx = (g.nx + C3_OWN) / C3_OWN, gy = (g.ny + C3_OWN) / C3_OWN;
  const int64_t n4 = (int64_t)gx * gy * ((g.nz + 4) / 4), n8 = (int64_t)gx * gy * ((g.nz + 8) / 8);
  // automatic form: 3D tiles while every workgroup of the launch (all batch
  // slots) gets a compute unit of its own, the shorter blocks first; beyond
  // that workgroups share units and the z-marching tiles are faster
  // (measured on the 56 x 28 x 14 coarsest grid of 224 x 112 x 56 with
  // 4 x 4 x 4 blocks: 480 workgroups)
  // (4 x 4 x 8 blocks only in float32: in float64 their LDS exceeds a workgroup's 160 KB)
  // (three steps per launch on 4 x 4 x 4 blocks, float32 only, wherever
  // 4 x 4 x 4 pairs would fit: one launch instead of 1.5)
  int form = p->cheb_per_launch;
  if (form == 0) {
    const int64_t cus = device_cus();
    form = n4 * p->bcount <= cus ? (FE_CHEB_TRIPLES ? 5 : 3) : (tall && n8 * p->bcount <= cus) ? 4 : 2;
  }
  return form == 5 && !tall ? 3 : form;
}

template <typename T>
bool cheb2_forms_first_direction(const fe_problem* p, int lev) {
  return cheb2_form(p, lev, sizeof(T) == 4) >= 3;
}

template <typename T>
bool cheb_triples(const fe_problem* p, int lev) {
  return sizeof(T) == 4 && cheb2_form(p, lev, true) == 5;
}

template <typename T>
hipError_t launch_cheb3(fe_problem* p, int lev, const T* dk, T* y, const T* E, const T* invd, const T* rin,
                        T* rout, T* acc, const double (&c)[6], int first, CgState* st, double dscale) {
  if constexpr (!std::is_same<T, float>::value) {
    return hipErrorInvalidValue;
  } else {
    if (!cheb_triples<T>(p, lev)) return hipErrorInvalidValue;
    const Grid g = p->L[lev].g;
    Cheb2<T> cf;
    cf.c1a = (T)c[0];
    cf.c2a = (T)c[1];
    cf.c1b = (T)c[2];
    cf.c2b = (T)c[3];
    cf.c1c = (T)c[4];
    cf.c2c = (T)c[5];
    cf.first = first;
    cf.dscale = (T)dscale;
    // block shape: the smallest of 2 x 2 x 4, 2 x 4 x 4 and 4 x 4 x 4 nodes
    // whose launch (all batch slots) still has at most one workgroup per
    // compute unit -- more units at work, each with a smaller first brick
    // phase, for a larger share of recomputed halo (28 x 14 x 7 coarsest
    // grid: 6.8 / 7.3 / 7.7 us per launch; 2 x 2 x 2 blocks, two workgroups
    // per unit: 10.3 us)
    const int64_t cus = device_cus();
    auto blocks = [&](int ox, int oy, int oz) {
      return (int64_t)((g.nx + ox) / ox) * ((g.ny + oy) / oy) * ((g.nz + oz) / oz);
    };
    int shape = FE_CHEB3_SHAPE;
    if (shape == 0) shape = blocks(2, 2, 4) * p->bcount <= cus ? 3 : blocks(2, 4, 4) * p->bcount <= cus ? 2 : 1;
    const int ox = shape == 1 ? 4 : 2, oy = shape == 3 ? 2 : 4, oz = 4;
    const int gx = (g.nx + ox) / ox, gy = (g.ny + oy) / oy;
    const int64_t nblk = blocks(ox, oy, oz), per = (nblk + 7) / 8;
    if (8 * per > ((int64_t)1 << 31) - 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(8 * per), p->bcount);
    const WK<T> wk = scaled_wk<T>(p->wk, p->L[lev].h);
    const int64_t wsh = p->bcount > 1 ? p->bstride : (int64_t)0;
    if (shape == 3)
      hipLaunchKernelGGL((cheb3t_kernel<2, 2, 4>), grid, dim3(C3T<2, 2, 4>::THREADS), 0, p->stream, g, gx, gy,
                         (int)nblk, (int)per, dk, E, p->L[lev].nmask, wk, invd, rin, rout, acc, y, cf, st, wsh);
    else if (shape == 2)
      hipLaunchKernelGGL((cheb3t_kernel<2, 4, 4>), grid, dim3(C3T<2, 4, 4>::THREADS), 0, p->stream, g, gx, gy,
                         (int)nblk, (int)per, dk, E, p->L[lev].nmask, wk, invd, rin, rout, acc, y, cf, st, wsh);
    else
      hipLaunchKernelGGL((cheb3t_kernel<4, 4, 4>), grid, dim3(C3T<4, 4, 4>::THREADS), 0, p->stream, g, gx, gy,
                         (int)nblk, (int)per, dk, E, p->L[lev].nmask, wk, invd, rin, rout, acc, y, cf, st, wsh);
    return hipGetLastError();
  }
}

template <typename T>
hipError_t launch_cheb2(fe_problem* p, int lev, const T* dk, T* y, const T* E, const T* invd, const T* rin,
                        T* rout, T* acc, const double (&c)[4], int first, CgState* st, double dscale) {
  const Grid g = p->L[lev].g;
  Cheb2<T> cf;
  cf.c1a = (T)c[0];
  cf.c2a = (T)c[1];
  cf.c1b = (T)c[2];
  cf.c2b = (T)c[3];
  cf.first = first;
  cf.dscale = (T)dscale;
  // 3D tiles of 4 x 4 x 4 or 4 x 4 x 8 owned nodes
  const int gx = (g.nx + C3_OWN) / C3_OWN, gy = (g.ny + C3_OWN) / C3_OWN;
  const int64_t n4 = (int64_t)gx * gy * ((g.nz + 4) / 4), n8 = (int64_t)gx * gy * ((g.nz + 8) / 8);
  constexpr bool tall = sizeof(T) == 4;
  const int form = cheb2_form(p, lev, tall);
  if (dscale != 0.0 && form < 3) return hipErrorInvalidValue;  // only the 3D tiles form the first direction
  if (form >= 3) {
    const bool oz4 = form == 3 || form == 5 || !tall;
    const int64_t nblk = oz4 ? n4 : n8, per = (nblk + 7) / 8;
    if (8 * per > ((int64_t)1 << 31) - 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(8 * per), p->bcount);
    const WK<T> wk = scaled_wk<T>(p->wk, p->L[lev].h);
    const int64_t wsh = p->bcount > 1 ? p->bstride : (int64_t)0;
    if (oz4)
      hipLaunchKernelGGL((cheb3d_kernel<T, 4>), grid, dim3(C3<4>::THREADS), 0, p->stream, g, gx, gy, (int)nblk,
                         (int)per, dk, E, p->L[lev].nmask, wk, invd, rin, rout, acc, y, cf, st, wsh);
    else if constexpr (tall)
      hipLaunchKernelGGL((cheb3d_kernel<T, 8>), grid, dim3(C3<8>::THREADS), 0, p->stream, g, gx, gy, (int)nblk,
                         (int)per, dk, E, p->L[lev].nmask, wk, invd, rin, rout, acc, y, cf, st, wsh);
    return hipGetLastError();
  }
  const void* k = reinterpret_cast<const void*>(&cheb2_kernel<T>);
  const TileMap tm = kxu_tile_map(g, kxu_slots(k, 2 * TX * TY), OWN2);
  if (3 * (int64_t)(g.nx + 1) * (g.ny + 1) * tm.kc * (int64_t)sizeof(T) >= ((int64_t)1 << 31) ||
      (int64_t)(g.nx + 1) * (g.ny + 1) * (tm.kc + 4) >= (int64_t)kOffIndex)
    return hipErrorInvalidValue;  // the stores' 31-bit offsets, the load ranges' index bound
  hipLaunchKernelGGL(cheb2_kernel<T>, dim3(tm.nblk, p->bcount), dim3(2 * TX * TY), 0, p->stream, g, tm, dk, E,
                     p->L[lev].nmask, scaled_wk<T>(p->wk, p->L[lev].h), invd, rin, rout, acc, y, cf, st,
                     reinterpret_cast<const T*>(p->zpad), p->bcount > 1 ? p->bstride : (int64_t)0);
  return hipGetLastError();
}
template hipError_t launch_cheb2<double>(fe_problem*, int, const double*, double*, const double*, const double*,
                                         const double*, double*, double*, const double (&)[4], int, CgState*,
                                         double);
template hipError_t launch_cheb2<float>(fe_problem*, int, const float*, float*, const float*, const float*,
                                        const float*, float*, float*, const double (&)[4], int, CgState*, double);
template bool cheb2_forms_first_direction<double>(const fe_problem*, int);
template bool cheb2_forms_first_direction<float>(const fe_problem*, int);
template bool cheb_triples<double>(const fe_problem*, int);
template bool cheb_triples<float>(const fe_problem*, int);
template hipError_t launch_cheb3<double>(fe_problem*, int, const double*, double*, const double*, const double*,
                                         const double*, double*, double*, const double (&)[6], int, CgState*,
                                         double);
template hipError_t launch_cheb3<float>(fe_problem*, int, const float*, float*, const float*, const float*,
                                        const float*, float*, float*, const double (&)[6], int, CgState*, double);

template <typename T>
hipError_t launch_kxu_tile(fe_problem* p, int lev, const T* x, const T* E, T* y, CgState* st, int mode,
                           const double* b64, double* out, const T* bT, const T* invd, double omega,
                           const ChebStep<T>* cs, const TileFuse<T>* fz) {
  const Grid g = p->L[lev].g;
  const WK<T> wk = scaled_wk<T>(p->wk, p->L[lev].h);
  Epi<T> ep;
  ep.b64 = b64;
  ep.bT = bT;
  ep.invd = invd;
  ep.omega = (T)omega;
  ep.res = cs ? cs->res : nullptr;
  ep.acc = cs ? cs->acc : nullptr;
  ep.c1 = cs ? (T)cs->c1 : T(0);
  ep.c2 = cs ? (T)cs->c2 : T(0);
  ep.first = cs ? cs->first : 0;
  const uint8_t* nm = p->L[lev].nmask;
  // algorithmic bytes: read x and E, write y, plus b (modes 2-5) and the
  // Jacobi diagonal (modes 3, 5, 6) and the fused operand's extra arrays;
  // each array touched once
  int slot = -1;
  if (lev == 0 && p->kst.on && (p->kst.mode < 0 || p->kst.mode == mode)) {
    const double vb = sizeof(T);
    double bytes = vb * (2.0 * (double)g.ndof + (double)g.nelem);
    if (mode == 2) bytes += 8.0 * (double)g.ndof;
    if (mode >= 3) bytes += vb * (double)g.ndof;
    if (mode == 3 || mode == 5 || mode == 6) bytes += vb * (double)g.nnode;
    if (mode == 6) bytes += vb * 3.0 * (double)g.ndof;  // res in/out, acc in/out (res read counted above)
    if (fz && fz->xin == 1) bytes += vb * (double)g.nnode;  // inverse diagonal of the fused first sweep
    if (fz && fz->xin >= 2) bytes += vb * (double)g.ndof;   // previous direction
    if (fz && fz->xin == 3) bytes -= (vb - 4.0) * (double)g.ndof;  // the operand read in float32
    if (fz && fz->xin && fz->xout) bytes += vb * (double)g.ndof;  // the operand, stored
    slot = kstats_begin(p, bytes);
  }
  int nb = 0;
  double* pt = (fz && fz->part) ? fz->part : p->partials;
  const bool fused = fz && (fz->xin != 0 || fz->fold);  // the matrix-core kernel has no fused operand
  if (p->bcount > 1 && (p->mfma_l0 || (lev == 0 && p->kst.on))) return hipErrorInvalidValue;  // not batched
  if (std::is_same<T, float>::value && lev == 0 && p->mfma_l0 && mode != 2 && mode != 6 && !fused) {
    Epi<float> ef;
    ef.b64 = b64;
    ef.bT = reinterpret_cast<const float*>(bT);
    ef.invd = reinterpret_cast<const float*>(invd);
    ef.omega = (float)omega;
    ef.res = nullptr;
    ef.acc = nullptr;
    ef.c1 = ef.c2 = 0.0f;
    ef.first = 0;
    const float* xf = reinterpret_cast<const float*>(x);
    const float* Ef = reinterpret_cast<const float*>(E);
    float* yf = reinterpret_cast<float*>(y);
    const float ks = (float)p->L[lev].h;
    nb = p->mfma_l0 == 2 ? launch_mfma<true>(mode, p->stream, g, xf, Ef, nm, p->ke32, ks, yf, ef, st, pt)
                         : launch_mfma<false>(mode, p->stream, g, xf, Ef, nm, p->ke32, ks, yf, ef, st, pt);
  } else {
    const T* zp = reinterpret_cast<const T*>(p->zpad);
    XinK<T> xi;
    xi.invd = fz ? fz->invd : nullptr;
    xi.s = fz ? (T)fz->s : T(0);
    xi.pold = fz ? fz->pold : nullptr;
    xi.xout = fz ? fz->xout : nullptr;
    FoldK fo;
    fo.part = fz ? fz->fold : nullptr;
    fo.n = fz ? fz->nfold : 0;
    fo.what = (fz && fz->fold) ? (fz->fold_rr ? 2 : 1) : 0;
    const int xin = fz ? fz->xin : 0;
#define FE_TILE(M, X) \
  launch_tile<T, M, X>(p->stream, g, x, E, nm, wk, y, ep, st, pt, out, zp, xi, fo, p->bcount, p->bstride)
    switch (mode * 4 + xin) {
      case 1 * 4: nb = FE_TILE(1, 0); break;
      case 1 * 4 + 2: nb = FE_TILE(1, 2); break;
      case 1 * 4 + 3:
        if (!std::is_same<T, double>::value) return hipErrorInvalidValue;
        nb = FE_TILE(1, 3);
        break;
      case 2 * 4: nb = FE_TILE(2, 0); break;
      case 3 * 4: nb = FE_TILE(3, 0); break;
      case 3 * 4 + 1: nb = FE_TILE(3, 1); break;
      case 4 * 4: nb = FE_TILE(4, 0); break;
      case 4 * 4 + 1: nb = FE_TILE(4, 1); break;
      case 5 * 4: nb = FE_TILE(5, 0); break;
      case 6 * 4: nb = FE_TILE(6, 0); break;
      case 0: nb = FE_TILE(0, 0); break;
      default: return hipErrorInvalidValue;
    }
#undef FE_TILE
    if (nb < 0) {  // a chunk too large for the stores' 31-bit offsets (about 89M nodes per level)
      kstats_end(p, slot);
      return hipErrorInvalidValue;
    }
  }
  hipError_t e = hipGetLastError();
  kstats_end(p, slot);
  if (e != hipSuccess) return e;
  if (fz && fz->nblocks) *fz->nblocks = nb;
  if (fz && fz->no_finalize) return hipSuccess;
  if (mode == 1) return launch_cg_finalize(p, FIN_ALPHA, nb, 0, st, nullptr);
  if (mode == 2) return launch_cg_finalize(p, FIN_SCALAR, nb, 0, nullptr, out);
  if (mode == 5) return launch_cg_finalize(p, FIN_RZ, nb, 1, st, nullptr);
  return hipSuccess;
}

template hipError_t launch_kxu_tile<double>(fe_problem*, int, const double*, const double*, double*,
                                            CgState*, int, const double*, double*, const double*,
                                            const double*, double, const ChebStep<double>*,
                                            const TileFuse<double>*);
template hipError_t launch_kxu_tile<float>(fe_problem*, int, const float*, const float*, float*, CgState*,
                                           int, const double*, double*, const float*, const float*, double,
                                           const ChebStep<float>*, const TileFuse<float>*);
