// Host-side discretization of one surface: geometry at the nodes, the
// oversampled far rule, patch centres/radii, near lists and the locally
// corrected quadrature (Section 4).
#pragma once
#include <cstdint>
#include <vector>

#include "nker.hpp"
#include "refelem.hpp"

namespace lb {

struct QuadOpts {
  int self_n = 20;       // self rule: Gauss points along each ray
  int self_nt = 12;      // self rule: Gauss points per panel of the sinh edge variable
  double self_panel = 2.0;
  int near_q = 8;        // conical rule per adaptive leaf: near_q x near_q
  double near_adm = 2.0; // leaf accepted when dist >= near_adm * diam
  int max_depth = 16;
};

// An oversampled far rule on every patch (Section 4: the q x q conical
// Gauss points of the reference element mapped by the interpolated chart):
// positions, unit normals and weights, patch-major.
struct OverRule {
  const RefElem* re = nullptr;  // the reference element holding P and the rule
  int n_o = 0;
  int64_t No = 0;
  std::vector<double> s, nu, wo;  // [No][3], [No][3], [No]
};

struct Surface {
  const RefElem* re = nullptr;
  int NP = 0, n_p = 0, n_o = 0;
  int64_t N = 0, No = 0;
  // node samples (patch-major), as given
  std::vector<double> X, Xu, Xv;          // [N][3]
  // node geometry
  std::vector<double> nrm, w, J, H;       // [N][3], [N], [N], [N]
  std::vector<double> dXu, dXv;           // derivative of the interpolated X at nodes [N][3]
  // modal coefficients of X, Xu, Xv per patch: [NP][n_p][3]
  std::vector<double> cX, cXu, cXv;
  // modal coefficients of the derivatives of the interpolated X (the
  // polynomials dXu, dXv of degree k - 1): [NP][n_p][3]
  std::vector<double> cDu, cDv;
  // oversampled far rule (the primary one: FP64 path, patch radii)
  std::vector<double> s, nu, wo;          // [No][3], [No][3], [No]
  // the FP32 path's own far rule (build_over)
  OverRule o32;
  // patches
  std::vector<double> cen, R;             // [NP][3], [NP]
  double eta = 2.0;
  // surface of each patch (several independent surfaces; empty = one)
  std::vector<int> surf_of_patch;
  // near lists (block CSR rows = targets; only patches of the target's surface)
  std::vector<int64_t> near_ptr;          // [N+1]
  std::vector<int32_t> near_patch;        // [nnz_blocks]

  void build(const RefElem& re, int NP, const double* X, const double* Xu, const double* Xv,
             double eta);
  void build_near_lists();
  // Chart at param (u, v) of patch p: position, interpolated X_u, X_v and the
  // basis values K (modal), n_p of them.
  void chart(int p, double u, double v, double* K, double* x, double* xu, double* xv) const;
  // A second far rule (for instance a coarser one for the FP32 path) from
  // the same chart samples; the primary rule above sets the patch radii.
  void build_over(const RefElem& reo, OverRule& out) const;
  // Derivatives of the interpolated X (not the interpolated X_u, X_v) at
  // param (u, v) of patch p; K is basis scratch of n_p values.
  void dchart(int p, double u, double v, double* K, double* du, double* dv) const;
};

// Accurate near integrals A (eq. nys-lcq2) for every (target, near patch)
// block: vals [nnz_blocks][n_p][NKER], kernels S, Gx, Gy, Gz, S', S''+D', D.
// With self_only, A must already hold nnz_blocks * n_p * NKER values and only
// the blocks of each target's own patch are written.
void near_integrals(const Surface& S, const QuadOpts& qo, std::vector<double>& A, bool self_only = false);

// Leaf rule of the adaptive near quadrature: the q x q conical Gauss rule on
// T0 (points ru [q*q][2], weights rw [q*q]).
void near_leaf_rule(int q, std::vector<double>& ru, std::vector<double>& rw);

// Far-rule contributions B of the near patches.  When fp32_mask is set, the
// oversampled sources whose float32 squared distance to the target is below
// the float32 mask radius squared of the source (the FP32 near-field kernel
// skips exactly these pairs) are left out.
// `over` (nullable): the far rule to use instead of the surface's primary one
// (rm2_f32 and sx32 then index its points).
void far_rule_blocks(const Surface& S, const std::vector<float>& rm2_f32,
                     const std::vector<float>& tx32, const std::vector<float>& sx32,
                     bool fp32_mask, std::vector<double>& B, const OverRule* over = nullptr);

}  // namespace lb
