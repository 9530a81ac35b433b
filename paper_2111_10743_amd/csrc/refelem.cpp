// Reference element on T0 (Section 4, discretization by order-k patches).
//
// Nodes: the paper samples charts at Vioreanu-Rokhlin nodes; their tables are
// not available, so the library uses the symmetric Blyth-Pozrikidis
// construction driven by the k+1 Gauss-Legendre points g_0 < ... < g_k of
// [0, 1]: for i + j + l = k the point has barycentric coordinates
// (1 + 2 g_a - g_b - g_c) / 3 over the cyclic triples of (i, j, l).  Every
// node is interior and the interpolatory weights are positive for k <= 7.
//
// Basis: psi_ij = (1 - v)^i P_i((2u - 1 + v)/(1 - v)) P_j^{(2i+1,0)}(2v - 1),
// i + j <= k, with the first factor evaluated by the Legendre recurrence
// multiplied through by powers of (1 - v) (no division, valid on all of T0).
#include "refelem.hpp"
#include "common.hpp"

#include <cmath>

namespace lb {

void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = t;
      for (int m = 2; m <= n; ++m) {
        double p2 = ((2.0 * m - 1.0) * t * p1 - (m - 1.0) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = t; p0 = 1.0; }
      dp = n * (t * p1 - p0) / (t * t - 1.0);
      double dt = p1 / dp;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    // recompute derivative at the converged root
    double p0 = 1.0, p1 = t;
    for (int m = 2; m <= n; ++m) {
      double p2 = ((2.0 * m - 1.0) * t * p1 - (m - 1.0) * p0) / m;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = t; p0 = 1.0; }
    dp = n * (t * p1 - p0) / (t * t - 1.0);
    // ascending order on [0, 1]
    x[n - 1 - i] = 0.5 * (t + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp);  // = (2/((1-t^2)P'^2)) / 2
  }
}

double jacobi(int n, double a, double b, double x) {
  if (n < 0) return 0.0;
  double p0 = 1.0;
  if (n == 0) return p0;
  double p1 = 0.5 * ((a - b) + (a + b + 2.0) * x);
  for (int m = 1; m < n; ++m) {
    double c = 2.0 * m + a + b;
    double a1 = 2.0 * (m + 1) * (m + a + b + 1.0) * c;
    double a2 = (c + 1.0) * (a * a - b * b);
    double a3 = c * (c + 1.0) * (c + 2.0);
    double a4 = 2.0 * (m + a) * (m + b) * (c + 2.0);
    double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

std::vector<double> ref_nodes(int k) {
  if (k < 1 || k > 7) fail(LB_EINVAL, "order %d out of range 1..7", k);
  std::vector<double> g, gw;
  gauss_legendre01(k + 1, g, gw);
  std::vector<double> uv;
  for (int i = 0; i <= k; ++i)
    for (int j = 0; j <= k - i; ++j) {
      int l = k - i - j;
      uv.push_back((1.0 + 2.0 * g[i] - g[j] - g[l]) / 3.0);
      uv.push_back((1.0 + 2.0 * g[j] - g[i] - g[l]) / 3.0);
    }
  return uv;
}

void RefElem::basis(double u, double v, double* K, double* Ku, double* Kv) const {
  const double a = 2.0 * u - 1.0 + v, b = 1.0 - v, eta = 2.0 * v - 1.0;
  double Q[16], Qu[16], Qv[16];
  Q[0] = 1.0; Qu[0] = 0.0; Qv[0] = 0.0;
  if (k >= 1) { Q[1] = a; Qu[1] = 2.0; Qv[1] = 1.0; }
  for (int i = 1; i < k; ++i) {
    Q[i + 1] = ((2 * i + 1) * a * Q[i] - i * b * b * Q[i - 1]) / (i + 1);
    if (Ku) {
      Qu[i + 1] = ((2 * i + 1) * (2.0 * Q[i] + a * Qu[i]) - i * b * b * Qu[i - 1]) / (i + 1);
      Qv[i + 1] = ((2 * i + 1) * (Q[i] + a * Qv[i]) - i * (-2.0 * b * Q[i - 1] + b * b * Qv[i - 1])) / (i + 1);
    }
  }
  const int K1 = k + 1;
  for (int i = 0; i <= k; ++i) {
    // P_j^{(2i+1,0)}(eta) and P_j^{(2i+2,1)}(eta), j = 0..k-i, by the precomputed recurrences
    const int jm = k - i;
    double P[16], D[16];
    P[0] = 1.0;
    D[0] = 1.0;
    for (int j = 0; j < jm; ++j) {
      const int r = i * K1 + j;
      P[j + 1] = (ja[r] + jb[r] * eta) * P[j] - (j > 0 ? jc[r] * P[j - 1] : 0.0);
      D[j + 1] = (dja[r] + djb[r] * eta) * D[j] - (j > 0 ? djc[r] * D[j - 1] : 0.0);
    }
    for (int j = 0; j <= jm; ++j) {
      const int n = i + j;
      const int c = n * (n + 1) / 2 + i;
      K[c] = Q[i] * P[j];
      if (Ku) {
        // d/deta P_j^{(a,0)} = (j + a + 1)/2 P_{j-1}^{(a+1,1)}
        const double dP = j > 0 ? 0.5 * (j + 2 * i + 2) * D[j - 1] : 0.0;
        Ku[c] = Qu[i] * P[j];
        Kv[c] = Qv[i] * P[j] + 2.0 * Q[i] * dP;
      }
    }
  }
}

void RefElem::lagrange(double u, double v, double* L) const {
  double K[64];
  basis(u, v, K);
  for (int bb = 0; bb < n_p; ++bb) {
    double s = 0.0;
    for (int c = 0; c < n_p; ++c) s += K[c] * Vinv[c * n_p + bb];
    L[bb] = s;
  }
}

RefElem::RefElem(int k_, int q_) : k(k_), q(q_) {
  n_p = order_npts(k);
  // Jacobi three-term recurrence coefficients (a, b) -> P_{j+1}
  auto coef = [](int m, double al, double be, double& A, double& B, double& C) {
    if (m == 0) {
      A = 0.5 * (al - be);
      B = 0.5 * (al + be + 2.0);
      C = 0.0;
      return;
    }
    double c = 2.0 * m + al + be;
    double a1 = 2.0 * (m + 1) * (m + al + be + 1.0) * c;
    A = (c + 1.0) * (al * al - be * be) / a1;
    B = c * (c + 1.0) * (c + 2.0) / a1;
    C = 2.0 * (m + al) * (m + be) * (c + 2.0) / a1;
  };
  const int K1 = k + 1;
  ja.assign(K1 * K1, 0.0); jb = ja; jc = ja; dja = ja; djb = ja; djc = ja;
  for (int i = 0; i <= k; ++i)
    for (int m = 0; m <= k; ++m) {
      coef(m, 2.0 * i + 1.0, 0.0, ja[i * K1 + m], jb[i * K1 + m], jc[i * K1 + m]);
      coef(m, 2.0 * i + 2.0, 1.0, dja[i * K1 + m], djb[i * K1 + m], djc[i * K1 + m]);
    }
  uv = ref_nodes(k);
  // Vandermonde V[a][c] = psi_c(node a); Vinv its inverse
  std::vector<double> V(n_p * n_p), Ku(n_p * n_p), Kv(n_p * n_p);
  for (int a = 0; a < n_p; ++a) basis(uv[2 * a], uv[2 * a + 1], &V[a * n_p], &Ku[a * n_p], &Kv[a * n_p]);
  Vinv = V;
  invert(Vinv, n_p);
  Du.assign(n_p * n_p, 0.0);
  Dv.assign(n_p * n_p, 0.0);
  for (int a = 0; a < n_p; ++a)
    for (int bb = 0; bb < n_p; ++bb) {
      double su = 0.0, sv = 0.0;
      for (int c = 0; c < n_p; ++c) {
        su += Ku[a * n_p + c] * Vinv[c * n_p + bb];
        sv += Kv[a * n_p + c] * Vinv[c * n_p + bb];
      }
      Du[a * n_p + bb] = su;
      Dv[a * n_p + bb] = sv;
    }
  // weights: w_b = sum_c Vinv[c][b] * integral(psi_c); psi_00 = 1 and the
  // others are orthogonal to it, so the integral vector is (1/2, 0, ...).
  w_ref.assign(n_p, 0.0);
  for (int bb = 0; bb < n_p; ++bb) w_ref[bb] = 0.5 * Vinv[0 * n_p + bb];
  // conical rule u = a (1 - b), v = b
  std::vector<double> g, gw;
  gauss_legendre01(q, g, gw);
  n_o = q * q;
  over_uv.resize(2 * n_o);
  over_w.resize(n_o);
  for (int jb = 0; jb < q; ++jb)
    for (int ia = 0; ia < q; ++ia) {
      int m = jb * q + ia;
      over_uv[2 * m] = g[ia] * (1.0 - g[jb]);
      over_uv[2 * m + 1] = g[jb];
      over_w[m] = gw[ia] * gw[jb] * (1.0 - g[jb]);
    }
  P.resize(n_o * n_p);
  for (int m = 0; m < n_o; ++m) lagrange(over_uv[2 * m], over_uv[2 * m + 1], &P[m * n_p]);
}

void invert(std::vector<double>& A, int n) {
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(A[r * n + col]) > std::fabs(A[piv * n + col])) piv = r;
    if (std::fabs(A[piv * n + col]) < 1e-300) fail(LB_EINVAL, "singular matrix");
    if (piv != col)
      for (int c = 0; c < n; ++c) {
        std::swap(A[piv * n + c], A[col * n + c]);
        std::swap(I[piv * n + c], I[col * n + c]);
      }
    double d = 1.0 / A[col * n + col];
    for (int c = 0; c < n; ++c) { A[col * n + c] *= d; I[col * n + c] *= d; }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double f = A[r * n + col];
      if (f == 0.0) continue;
      for (int c = 0; c < n; ++c) { A[r * n + c] -= f * A[col * n + c]; I[r * n + c] -= f * I[col * n + c]; }
    }
  }
  A = I;
}

}  // namespace lb
