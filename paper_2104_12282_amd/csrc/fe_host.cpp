// Host-side setup arithmetic: the hex8 element stiffness by Gauss quadrature
// and its constants in the per-axis sum/difference (Walsh) basis.
#include <cmath>
#include <cstring>
#include <string>

#include "fe_internal.h"

static thread_local std::string g_last_error;

void fe_set_error(const std::string& msg) { g_last_error = msg; }

extern "C" const char* fe_last_error(void) { return g_last_error.c_str(); }

// Corner offsets of the brick in the fixed local order.
static const int kCorner[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                                  {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};

// Ke = integral over the cube [0,h]^3 of B^T D B (isotropic D with Lame
// constants from E and nu, Voigt order xx yy zz yz xz xy, engineering
// shear).  2x2x2 Gauss points integrate the degree-2-per-axis integrand
// exactly.
int host_hex8_ke(double nu, double E, double h, double* Ke) {
  const double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
  const double mu = E / (2.0 * (1.0 + nu));
  double D[6][6] = {};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) D[a][b] = lam;
  for (int a = 0; a < 3; ++a) D[a][a] = lam + 2.0 * mu;
  for (int a = 3; a < 6; ++a) D[a][a] = mu;

  const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  std::memset(Ke, 0, sizeof(double) * 576);
  for (int qx = 0; qx < 2; ++qx)
    for (int qy = 0; qy < 2; ++qy)
      for (int qz = 0; qz < 2; ++qz) {
        const double t[3] = {gp[qx], gp[qy], gp[qz]};
        double B[6][24] = {};
        for (int a = 0; a < 8; ++a) {
          double g[3];
          for (int d = 0; d < 3; ++d) {
            double v = (kCorner[a][d] ? 1.0 : -1.0) / h;
            for (int d2 = 0; d2 < 3; ++d2)
              if (d2 != d) v *= kCorner[a][d2] ? t[d2] : 1.0 - t[d2];
            g[d] = v;
          }
          const int cx = 3 * a, cy = 3 * a + 1, cz = 3 * a + 2;
          B[0][cx] = g[0];
          B[1][cy] = g[1];
          B[2][cz] = g[2];
          B[3][cy] = g[2];
          B[3][cz] = g[1];
          B[4][cx] = g[2];
          B[4][cz] = g[0];
          B[5][cx] = g[1];
          B[5][cy] = g[0];
        }
        const double w = 0.125 * h * h * h;  // product of the three 1/2 weights times volume
        double DB[6][24];
        for (int r = 0; r < 6; ++r)
          for (int c = 0; c < 24; ++c) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += D[r][k] * B[k][c];
            DB[r][c] = s;
          }
        for (int r = 0; r < 24; ++r)
          for (int c = 0; c < 24; ++c) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += B[k][r] * DB[k][c];
            Ke[r * 24 + c] += w * s;
          }
      }
  return 0;
}

// S = V^T Ke V / 64 with V[s][m] = prod_d (-1)^(s_d m_d) (per component).
// Extracts the eight constants of WalshK and reports the largest deviation of
// S from the structure they describe (relative to max |S|).
int host_walsh_constants(const double* Ke, WalshK* wk, double* max_dev) {
  double V[8][8];
  for (int s = 0; s < 8; ++s)
    for (int m = 0; m < 8; ++m) {
      int sg = 0;
      for (int d = 0; d < 3; ++d) sg += kCorner[s][d] * kCorner[m][d];
      V[s][m] = (sg & 1) ? -1.0 : 1.0;
    }
  static double S[24][24];
  for (int m1 = 0; m1 < 8; ++m1)
    for (int c1 = 0; c1 < 3; ++c1)
      for (int m2 = 0; m2 < 8; ++m2)
        for (int c2 = 0; c2 < 3; ++c2) {
          double acc = 0.0;
          for (int s1 = 0; s1 < 8; ++s1)
            for (int s2 = 0; s2 < 8; ++s2)
              acc += V[s1][m1] * Ke[(3 * s1 + c1) * 24 + 3 * s2 + c2] * V[s2][m2];
          S[3 * m1 + c1][3 * m2 + c2] = acc / 64.0;
        }
  // mode numbers in the local order: 000=0 100=1 110=2 010=3 001=4 101=5 111=6 011=7
  auto at = [&](int m1, int c1, int m2, int c2) { return S[3 * m1 + c1][3 * m2 + c2]; };
  enum { X = 0, Y = 1, Z = 2 };
  const int m100 = 1, m110 = 2, m010 = 3, m001 = 4, m101 = 5, m111 = 6, m011 = 7;
  wk->A = at(m100, X, m100, X);
  wk->B = at(m100, X, m010, Y);
  wk->G = at(m100, Y, m100, Y);
  wk->C = at(m110, X, m110, X);
  wk->D = at(m110, X, m011, Z);
  wk->F = at(m110, Z, m110, Z);
  wk->H = at(m110, Z, m101, Y);
  wk->J = at(m111, X, m111, X);

  // Rebuild the structured S and compare.
  double R[24][24] = {};
  auto set = [&](int m1, int c1, int m2, int c2, double v) { R[3 * m1 + c1][3 * m2 + c2] = v; };
  const int lin[3] = {m100, m010, m001};  // linear mode along axis d
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) set(lin[a], a, lin[b], b, a == b ? wk->A : wk->B);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      if (a != b) {  // shear pair (lin[a], comp b) <-> (lin[b], comp a)
        set(lin[a], b, lin[a], b, wk->G);
        set(lin[a], b, lin[b], a, wk->G);
      }
  // bilinear modes: mode missing axis d is bil[d] (110 misses z, 101 misses y, 011 misses x)
  const int bil[3] = {m011, m101, m110};
  for (int d = 0; d < 3; ++d) {
    // component d of the mode that misses axis d couples to the triple
    for (int e = 0; e < 3; ++e) set(bil[d], d, bil[e], e, d == e ? wk->F : wk->H);
    // component c != d of mode bil[d] pairs with component d of mode bil[c]
    for (int c = 0; c < 3; ++c)
      if (c != d) {
        set(bil[d], c, bil[d], c, wk->C);
        set(bil[d], c, bil[c], d, wk->D);
      }
  }
  for (int c = 0; c < 3; ++c) set(m111, c, m111, c, wk->J);
  double smax = 0.0, dev = 0.0;
  for (int i = 0; i < 24; ++i)
    for (int j = 0; j < 24; ++j) {
      smax = std::fmax(smax, std::fabs(S[i][j]));
      dev = std::fmax(dev, std::fabs(S[i][j] - R[i][j]));
    }
  *max_dev = dev / smax;
  return 0;
}
