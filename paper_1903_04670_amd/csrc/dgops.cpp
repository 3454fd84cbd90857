// Host-side operators: nodal DG matrices on Gauss-Lobatto-Legendre points and
// the normal matrix of the conservation constraints.
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace dgfs {

// Legendre P_n and P_n' at x by the three-term recurrence.
static void legendre(int n, double x, double &p, double &dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  // P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1), away from the endpoints
  dp = (std::fabs(x * x - 1.0) > 1e-14) ? n * (x * p1 - p0) / (x * x - 1.0) : 0.5 * n * (n + 1) * std::pow(x, n - 1);
}

// Gauss-Jordan inverse with partial pivoting; returns false if singular.
bool invert(std::vector<double> &A, int n) {
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    for (int k = 0; k < n; ++k) {
      std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(I[c * n + k], I[piv * n + k]);
    }
    double d = A[c * n + c];
    for (int k = 0; k < n; ++k) { A[c * n + k] /= d; I[c * n + k] /= d; }
    for (int r = 0; r < n; ++r)
      if (r != c) {
        double f = A[r * n + c];
        if (f == 0.0) continue;
        for (int k = 0; k < n; ++k) { A[r * n + k] -= f * A[c * n + k]; I[r * n + k] -= f * I[c * n + k]; }
      }
  }
  A = I;
  return true;
}

// GLL nodes: -1, 1 and the roots of P_P' (Newton from Chebyshev-Lobatto guesses);
// V_ij = sqrt((2j+1)/2) P_j(r_i), Minv = V V^T, Dr = Vr V^{-1}.
bool dg_setup(int P, std::vector<double> &r, std::vector<double> &Dr, std::vector<double> &Minv) {
  const int n = P + 1;
  r.assign(n, 0.0);
  r[0] = -1.0;
  r[P] = 1.0;
  for (int i = 1; i < P; ++i) {
    double x = -std::cos(M_PI * i / P);
    for (int it = 0; it < 100; ++it) {
      // f = P_P'(x); f' = P_P''(x) = (2x P_P' - P(P+1) P_P)/(1 - x^2)
      double p, dp;
      legendre(P, x, p, dp);
      double d2p = (2.0 * x * dp - P * (P + 1.0) * p) / (1.0 - x * x);
      double dx = dp / d2p;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    r[i] = x;
  }
  std::vector<double> V(n * n), Vr(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double p, dp;
      legendre(j, r[i], p, dp);
      double s = std::sqrt((2.0 * j + 1.0) / 2.0);
      V[i * n + j] = s * p;
      Vr[i * n + j] = s * dp;
    }
  Minv.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) Minv[i * n + j] += V[i * n + k] * V[j * n + k];
  std::vector<double> Vi = V;
  if (!invert(Vi, n)) return false;
  Dr.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) Dr[i * n + j] += Vr[i * n + k] * Vi[k * n + j];
  return true;
}

// (C C^T)^{-1} for the constraint rows [mass_p (p in species), momentum x,y,z,
// energy], each a grid sum with weight h^3 (see the projection kernel).
bool projection_ginv(const dgfs_plan_s *pl, const std::vector<int> &species, std::vector<double> &G) {
  const int N = pl->N, k = (int)species.size() + 4, nsp = (int)species.size();
  const double h = 2.0 * pl->L / N, w = h * h * h;
  double s0 = 0, s2 = 0, s4 = 0, sx2 = 0;  // sums over the grid of 1, |c|^2, |c|^4, c_x^2
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      for (int l = 0; l < N; ++l) {
        double cx = -pl->L + (i + 0.5) * h, cy = -pl->L + (j + 0.5) * h, cz = -pl->L + (l + 0.5) * h;
        double c2 = cx * cx + cy * cy + cz * cz;
        s0 += 1.0;
        s2 += c2;
        s4 += c2 * c2;
        sx2 += cx * cx;
      }
  G.assign(k * k, 0.0);
  double mm2 = 0.0, mm4 = 0.0;
  for (int a = 0; a < nsp; ++a) {
    double m = pl->mass[species[a]];
    G[a * k + a] = w * w * s0;
    G[a * k + nsp + 3] = G[(nsp + 3) * k + a] = w * w * 0.5 * m * s2;
    mm2 += m * m;
    mm4 += 0.25 * m * m;
  }
  for (int d = 0; d < 3; ++d) G[(nsp + d) * k + nsp + d] = w * w * mm2 * sx2;
  G[(nsp + 3) * k + nsp + 3] = w * w * mm4 * s4;
  return invert(G, k);
}

}  // namespace dgfs
