// Reference element on T0 = {u, v >= 0, u + v <= 1}: order-k nodes,
// orthogonal (Dubiner/Koornwinder) basis, interpolation, weights,
// differentiation matrices and the oversampled conical rule (Section 4).
#pragma once
#include <vector>

namespace lb {

// Gauss-Legendre nodes and weights on [0, 1] (Newton on P_n).
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w);

// Jacobi polynomial P_n^{(a,b)}(x) by its three-term recurrence.
double jacobi(int n, double a, double b, double x);

struct RefElem {
  int k = 0, n_p = 0, q = 0, n_o = 0;
  std::vector<double> uv;        // [n_p][2]
  std::vector<double> Vinv;      // [n_p][n_p], modal coefficients = Vinv * nodal values
  std::vector<double> w_ref;     // [n_p]
  std::vector<double> Du, Dv;    // [n_p][n_p] nodal differentiation
  std::vector<double> over_uv;   // [n_o][2]
  std::vector<double> over_w;    // [n_o]
  std::vector<double> P;         // [n_o][n_p] interpolation to the oversampled points
  // Jacobi recurrence P_{j+1} = (ja + jb x) P_j - jc P_{j-1} for alpha = 2i+1,
  // beta = 0 (and the derivative family alpha = 2i+2, beta = 1): [k+1][k+1]
  std::vector<double> ja, jb, jc, dja, djb, djc;

  RefElem(int k, int q);
  // Basis values psi_c(u, v) (and derivatives when Ku/Kv are non-null).
  void basis(double u, double v, double* K, double* Ku = nullptr, double* Kv = nullptr) const;
  // Lagrange values L_b(u, v) of the node set.
  void lagrange(double u, double v, double* L) const;
};

// Order-k node set (Blyth-Pozrikidis construction on Gauss-Legendre points).
std::vector<double> ref_nodes(int k);
inline int order_npts(int k) { return (k + 1) * (k + 2) / 2; }

}  // namespace lb
