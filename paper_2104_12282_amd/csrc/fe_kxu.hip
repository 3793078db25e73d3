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

#include <type_traits>

#include "fe_internal.h"
#include "fe_reduce.h"

namespace {

constexpr int TX = 16, TY = 16, OWN = 15;

template <typename T>
struct WK {
  T A, B, G, C, D, F, H, J;
};

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
  s[X][1] = k.A * n1 + k.B * (n2 + n3);
  s[Y][3] = k.A * n2 + k.B * (n1 + n3);
  s[Z][4] = k.A * n3 + k.B * (n1 + n2);
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
  s[X][2] = k.C * t[X][2] + k.D * t[Z][7];
  s[Z][7] = k.D * t[X][2] + k.C * t[Z][7];
  s[Y][2] = k.C * t[Y][2] + k.D * t[Z][5];
  s[Z][5] = k.D * t[Y][2] + k.C * t[Z][5];
  s[X][5] = k.C * t[X][5] + k.D * t[Y][7];
  s[Y][7] = k.D * t[X][5] + k.C * t[Y][7];
  // bilinear triple
  const T a = t[Z][2], b = t[Y][5], c = t[X][7];
  s[Z][2] = k.F * a + k.H * (b + c);
  s[Y][5] = k.F * b + k.H * (a + c);
  s[X][7] = k.F * c + k.H * (a + b);
  // trilinear mode
  s[X][6] = k.J * t[X][6];
  s[Y][6] = k.J * t[Y][6];
  s[Z][6] = k.J * t[Z][6];
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
template <typename T, int MODE>
__global__ void __launch_bounds__(TX* TY) kxu_tile_kernel(Grid g, int kc, const T* __restrict__ x,
                                                         const T* __restrict__ E,
                                                         const uint8_t* __restrict__ nmask, WK<T> wk,
                                                         T* __restrict__ y, Epi<T> ep, CgState* st,
                                                         double* partials, double* out) {
  if ((MODE == 1 || MODE == 5 || st) && st->done) return;
  __shared__ T su[3][TY + 1][TX + 1];  // node values of the current upper level
  __shared__ T sy[9][TY][TX];          // level partials of corners (1,0), (1,1), (0,1)

  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int I0 = blockIdx.x * OWN - 1, J0 = blockIdx.y * OWN - 1, K0 = blockIdx.z * kc;
  const int ni = I0 + tx, nj = J0 + ty;
  const int64_t sx = g.nx + 1, sxy = (int64_t)(g.nx + 1) * (g.ny + 1);
  const bool owner = tx >= 1 && ty >= 1 && ni <= g.nx && nj <= g.ny;
  const bool ecol = ni >= 0 && ni < g.nx && nj >= 0 && nj < g.ny;
  const int kend = min(K0 + kc, g.nz + 1);  // owned levels: [K0, kend)

  auto node_ok = [&](int i, int j, int k) {
    return i >= 0 && i <= g.nx && j >= 0 && j <= g.ny && k >= 0 && k <= g.nz;
  };
  // Node values of one level held in registers: this thread's column and, for
  // threads on the high edges of the tile, the extra column/row/corner that
  // closes the 17 x 17 ring of the tile.
  struct LevelRegs {
    T own[3];
    T ext[3][3];
  };
  const bool ex0 = tx == TX - 1, ex1 = ty == TY - 1, ex2 = ex0 && ex1;
  auto fetch = [&](int i, int j, int k, T (&v)[3]) {
    if (node_ok(i, j, k)) {
      const int64_t n = i + sx * j + sxy * k;
      v[0] = x[3 * n];
      v[1] = x[3 * n + 1];
      v[2] = x[3 * n + 2];
    } else {
      v[0] = v[1] = v[2] = T(0);
    }
  };
  auto load_regs = [&](int k, LevelRegs& L) {
    fetch(ni, nj, k, L.own);
    if (ex0) fetch(I0 + TX, nj, k, L.ext[0]);
    if (ex1) fetch(ni, J0 + TY, k, L.ext[1]);
    if (ex2) fetch(I0 + TX, J0 + TY, k, L.ext[2]);
  };
  auto store_lds = [&](const LevelRegs& L) {
#pragma unroll
    for (int c = 0; c < 3; ++c) su[c][ty][tx] = L.own[c];
    if (ex0)
      for (int c = 0; c < 3; ++c) su[c][ty][TX] = L.ext[0][c];
    if (ex1)
      for (int c = 0; c < 3; ++c) su[c][TY][tx] = L.ext[1][c];
    if (ex2)
      for (int c = 0; c < 3; ++c) su[c][TY][TX] = L.ext[2][c];
  };
  auto modulus = [&](int ek) -> T {
    return (ecol && ek >= 0 && ek < g.nz) ? E[ni + (int64_t)g.nx * (nj + (int64_t)g.ny * ek)] : T(0);
  };

  T lo[4][3];      // corners (0,0) (1,0) (1,1) (0,1) of the brick's lower level
  T carry[4][3];   // contributions of the brick below to those corners
  T own_prev[3];   // this thread's node at the lower level
  LevelRegs nxt;
  T Enxt;
  {
    LevelRegs L0;
    load_regs(K0 - 1, L0);
    load_regs(K0, nxt);  // in flight during the prologue
    Enxt = modulus(K0 - 1);
    store_lds(L0);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      own_prev[c] = L0.own[c];
      lo[0][c] = su[c][ty][tx];
      lo[1][c] = su[c][ty][tx + 1];
      lo[2][c] = su[c][ty + 1][tx + 1];
      lo[3][c] = su[c][ty + 1][tx];
      carry[0][c] = carry[1][c] = carry[2][c] = carry[3][c] = T(0);
    }
    __syncthreads();
  }

  double dot = 0.0;
  for (int s = 0; s <= kc; ++s) {
    const int ek = K0 - 1 + s;  // brick layer between node levels ek and ek + 1
    if (ek >= g.nz + 1) break;  // uniform over the workgroup
    const LevelRegs cur = nxt;
    const T Ee = Enxt;
    store_lds(cur);
    if (s < kc) {  // prefetch the next level while this one is computed
      load_regs(ek + 2, nxt);
      Enxt = modulus(ek + 1);
    }
    __syncthreads();

    T v[3][8];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[c][0] = lo[0][c];
      v[c][1] = lo[1][c];
      v[c][2] = lo[2][c];
      v[c][3] = lo[3][c];
      v[c][4] = cur.own[c];
      v[c][5] = su[c][ty][tx + 1];
      v[c][6] = su[c][ty + 1][tx + 1];
      v[c][7] = su[c][ty + 1][tx];
      lo[0][c] = v[c][4];
      lo[1][c] = v[c][5];
      lo[2][c] = v[c][6];
      lo[3][c] = v[c][7];
    }
    walsh8(v[0]);
    walsh8(v[1]);
    walsh8(v[2]);
    WK<T> k = wk;
    k.A *= Ee; k.B *= Ee; k.G *= Ee; k.C *= Ee; k.D *= Ee; k.F *= Ee; k.H *= Ee; k.J *= Ee;
    T w[3][8];
    apply_S(k, v, w);
    walsh8(w[0]);
    walsh8(w[1]);
    walsh8(w[2]);
    // level-ek sums of this brick column's four corners
    T p0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      p0[c] = carry[0][c] + w[c][0];
      sy[0 + c][ty][tx] = carry[1][c] + w[c][1];
      sy[3 + c][ty][tx] = carry[2][c] + w[c][2];
      sy[6 + c][ty][tx] = carry[3][c] + w[c][3];
      carry[0][c] = w[c][4];
      carry[1][c] = w[c][5];
      carry[2][c] = w[c][6];
      carry[3][c] = w[c][7];
    }
    __syncthreads();
    if (s >= 1 && owner && ek >= K0 && ek < kend) {
      const int64_t n = ni + sx * nj + sxy * ek;
      const uint8_t m = nmask[n];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T v2 = p0[c] + sy[0 + c][ty][tx - 1] + sy[3 + c][ty - 1][tx - 1] + sy[6 + c][ty - 1][tx];
        const bool fx = (m >> c) & 1;
        if (fx) v2 = T(0);
        if (MODE == 2) {
          v2 = fx ? T(0) : (T)(ep.b64[3 * n + c] - (double)v2);
          dot += (double)v2 * (double)v2;
        } else if (MODE == 1) {
          dot += (double)own_prev[c] * (double)v2;
        } else if (MODE == 3 || MODE == 5) {
          const T bv = ep.bT[3 * n + c];
          v2 = fx ? T(0) : own_prev[c] + ep.omega * ep.invd[n] * (bv - v2);
          if (MODE == 5) dot += (double)bv * (double)v2;
        } else if (MODE == 4) {
          v2 = fx ? T(0) : ep.bT[3 * n + c] - v2;
        } else if (MODE == 6) {
          const T dv = own_prev[c];
          const T rn = fx ? T(0) : ep.res[3 * n + c] - v2;
          ep.res[3 * n + c] = rn;
          ep.acc[3 * n + c] = ep.first ? dv : ep.acc[3 * n + c] + dv;
          v2 = fx ? T(0) : ep.c1 * dv + ep.c2 * ep.invd[n] * rn;
        }
        y[3 * n + c] = v2;
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) own_prev[c] = cur.own[c];
  }
  if (MODE == 0 || MODE == 3 || MODE == 4 || MODE == 6) return;
  double vv[1] = {dot};
  block_partials<1>(vv, partials);
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
// z-carry and the node sums need.  Before rounding to bf16 the corner values
// are taken relative to corner 0 of the brick: Ke annihilates translations,
// so the product is unchanged in exact arithmetic while the rounding acts on
// the deformation only.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int MODE>
__global__ void __launch_bounds__(TX* TY) kxu_mfma_kernel(Grid g, int kc, const float* __restrict__ x,
                                                         const float* __restrict__ E,
                                                         const uint8_t* __restrict__ nmask,
                                                         const float* __restrict__ ke, float kscale,
                                                         float* __restrict__ y, Epi<float> ep, CgState* st,
                                                         double* partials) {
  if ((MODE == 1 || MODE == 5 || st) && st->done) return;
  __shared__ float su[2][3][TY + 1][TX + 1];  // two node levels
  __shared__ float sy[4][3][TY][TX];          // level partials per corner
  __shared__ float sE[TY][TX];

  const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int grp = lane >> 4, ln = lane & 15;
  const int I0 = blockIdx.x * OWN - 1, J0 = blockIdx.y * OWN - 1, K0 = blockIdx.z * kc;
  const int ni = I0 + tx, nj = J0 + ty;
  const int64_t sx = g.nx + 1, sxy = (int64_t)(g.nx + 1) * (g.ny + 1);
  const bool owner = tx >= 1 && ty >= 1 && ni <= g.nx && nj <= g.ny;
  const bool ecol = ni >= 0 && ni < g.nx && nj >= 0 && nj < g.ny;
  const int kend = min(K0 + kc, g.nz + 1);

  // Ke_pad rows 16 mt + ln, columns 8 grp .. 8 grp + 7 (bf16), in registers
  bf16x8 a[2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    const int m = 16 * mt + ln, cm = m >> 2, am = m & 3;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = 8 * grp + i, ck = k >> 2, ak = k & 3;
      const float v = (am < 3 && ak < 3) ? ke[(3 * cm + am) * 24 + 3 * ck + ak] * kscale : 0.0f;
      a[mt][i] = (__bf16)v;
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
      bf16x8 bv;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float ref = su[blo][c][r][ln];  // corner 0 of the brick
        bv[c] = (__bf16)(su[b][c][r + oyA][ln + oxA] - ref);
        bv[4 + c] = (__bf16)(su[b][c][r + oyB][ln + oxB] - ref);
      }
      bv[3] = (__bf16)0.0f;
      bv[7] = (__bf16)0.0f;
      const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
      const f32x4 dlo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], bv, zero, 0, 0, 0);
      const f32x4 dhi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], bv, zero, 0, 0, 0);
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

#ifndef FE_KXU_KC
#define FE_KXU_KC 8  // most node levels one workgroup marches through
#endif
#ifndef FE_KXU_TARGET_BLOCKS
#define FE_KXU_TARGET_BLOCKS 1024  // aim: four workgroups per compute unit
#endif

// Levels per workgroup: long marches amortise the tile halo, but small grids
// need short ones to give every compute unit work.
static int kxu_levels_per_block(const Grid& g) {
  const int64_t cols = (int64_t)((g.nx + 1 + OWN - 1) / OWN) * ((g.ny + 1 + OWN - 1) / OWN);
  int64_t kc = ((int64_t)(g.nz + 1) * cols + FE_KXU_TARGET_BLOCKS - 1) / FE_KXU_TARGET_BLOCKS;
  if (kc < 1) kc = 1;
  if (kc > FE_KXU_KC) kc = FE_KXU_KC;
  return (int)kc;
}

static dim3 kxu_grid(const Grid& g, int kc) {
  return dim3((unsigned)((g.nx + 1 + OWN - 1) / OWN), (unsigned)((g.ny + 1 + OWN - 1) / OWN),
              (unsigned)((g.nz + 1 + kc - 1) / kc));
}

int64_t kxu_tile_blocks(const Grid& g) {
  const dim3 d = kxu_grid(g, kxu_levels_per_block(g));
  return (int64_t)d.x * d.y * d.z;
}

template <typename T>
hipError_t launch_kxu_tile(fe_problem* p, int lev, const T* x, const T* E, T* y, CgState* st, int mode,
                           const double* b64, double* out, const T* bT, const T* invd, double omega,
                           const ChebStep<T>* cs) {
  const Grid g = p->L[lev].g;
  const int kc = kxu_levels_per_block(g);
  const dim3 grid = kxu_grid(g, kc);
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
  // Jacobi diagonal (modes 3, 5); each array touched once
  int slot = -1;
  if (lev == 0 && p->kst.on) {
    const double vb = sizeof(T);
    double bytes = vb * (2.0 * (double)g.ndof + (double)g.nelem);
    if (mode == 2) bytes += 8.0 * (double)g.ndof;
    if (mode >= 3) bytes += vb * (double)g.ndof;
    if (mode == 3 || mode == 5 || mode == 6) bytes += vb * (double)g.nnode;
    if (mode == 6) bytes += vb * 3.0 * (double)g.ndof;  // res in/out, acc in/out (res read counted above)
    slot = kstats_begin(p, bytes);
  }
  if (std::is_same<T, float>::value && lev == 0 && p->mfma_l0 && mode != 2 && mode != 6) {
    const float* xf = reinterpret_cast<const float*>(x);
    const float* Ef = reinterpret_cast<const float*>(E);
    float* yf = reinterpret_cast<float*>(y);
    Epi<float> ef;
    ef.b64 = b64;
    ef.bT = reinterpret_cast<const float*>(bT);
    ef.invd = reinterpret_cast<const float*>(invd);
    ef.omega = (float)omega;
    ef.res = nullptr;
    ef.acc = nullptr;
    ef.c1 = ef.c2 = 0.0f;
    ef.first = 0;
    const float ks = (float)p->L[lev].h;
    switch (mode) {
      case 1:
        hipLaunchKernelGGL(kxu_mfma_kernel<1>, grid, dim3(TX * TY), 0, p->stream, g, kc, xf, Ef, nm, p->ke32,
                           ks, yf, ef, st, p->partials);
        break;
      case 3:
        hipLaunchKernelGGL(kxu_mfma_kernel<3>, grid, dim3(TX * TY), 0, p->stream, g, kc, xf, Ef, nm, p->ke32,
                           ks, yf, ef, st, p->partials);
        break;
      case 4:
        hipLaunchKernelGGL(kxu_mfma_kernel<4>, grid, dim3(TX * TY), 0, p->stream, g, kc, xf, Ef, nm, p->ke32,
                           ks, yf, ef, st, p->partials);
        break;
      case 5:
        hipLaunchKernelGGL(kxu_mfma_kernel<5>, grid, dim3(TX * TY), 0, p->stream, g, kc, xf, Ef, nm, p->ke32,
                           ks, yf, ef, st, p->partials);
        break;
      default:
        hipLaunchKernelGGL(kxu_mfma_kernel<0>, grid, dim3(TX * TY), 0, p->stream, g, kc, xf, Ef, nm, p->ke32,
                           ks, yf, ef, st, p->partials);
    }
  } else switch (mode) {
    case 1:
      hipLaunchKernelGGL((kxu_tile_kernel<T, 1>), grid, dim3(TX * TY), 0, p->stream, g, kc, x, E, nm, wk,
                         y, ep, st, p->partials, out);
      break;
    case 2:
      hipLaunchKernelGGL((kxu_tile_kernel<T, 2>), grid, dim3(TX * TY), 0, p->stream, g, kc, x, E, nm, wk,
                         y, ep, st, p->partials, out);
      break;
    case 3:
      hipLaunchKernelGGL((kxu_tile_kernel<T, 3>), grid, dim3(TX * TY), 0, p->stream, g, kc, x, E, nm, wk,
                         y, ep, st, p->partials, out);
      break;
    case 4:
      hipLaunchKernelGGL((kxu_tile_kernel<T, 4>), grid, dim3(TX * TY), 0, p->stream, g, kc, x, E, nm, wk,
                         y, ep, st, p->partials, out);
      break;
    case 5:
      hipLaunchKernelGGL((kxu_tile_kernel<T, 5>), grid, dim3(TX * TY), 0, p->stream, g, kc, x, E, nm, wk,
                         y, ep, st, p->partials, out);
      break;
    case 6:
      hipLaunchKernelGGL((kxu_tile_kernel<T, 6>), grid, dim3(TX * TY), 0, p->stream, g, kc, x, E, nm, wk,
                         y, ep, st, p->partials, out);
      break;
    default:
      hipLaunchKernelGGL((kxu_tile_kernel<T, 0>), grid, dim3(TX * TY), 0, p->stream, g, kc, x, E, nm, wk,
                         y, ep, st, p->partials, out);
  }
  hipError_t e = hipGetLastError();
  kstats_end(p, slot);
  if (e != hipSuccess) return e;
  const int nb = (int)((int64_t)grid.x * grid.y * grid.z);
  if (mode == 1) return launch_cg_finalize(p, FIN_ALPHA, nb, 0, st, nullptr);
  if (mode == 2) return launch_cg_finalize(p, FIN_SCALAR, nb, 0, nullptr, out);
  if (mode == 5) return launch_cg_finalize(p, FIN_RZ, nb, 1, st, nullptr);
  return hipSuccess;
}

template hipError_t launch_kxu_tile<double>(fe_problem*, int, const double*, const double*, double*,
                                            CgState*, int, const double*, double*, const double*,
                                            const double*, double, const ChebStep<double>*);
template hipError_t launch_kxu_tile<float>(fe_problem*, int, const float*, const float*, float*, CgState*,
                                           int, const double*, double*, const float*, const float*, double,
                                           const ChebStep<float>*);
