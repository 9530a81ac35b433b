// Geometry and near lists of one surface (Section 2 and Section 4).
//
// * w_i = |X_u x X_v|_i w_ref,i and n_i = X_u x X_v / |.| at the nodes.
// * Mean curvature from second derivatives obtained by spectral
//   differentiation of the stored X_u, X_v (Section 4, paragraph on normals
//   at oversampled nodes): X_uu = D_u X_u, X_vv = D_v X_v,
//   X_uv = (D_v X_u + D_u X_v)/2, H = -(E N2 - 2F M2 + G L2) / (2(EG - F^2)),
//   the sign giving H = +1 on the unit sphere with the outward normal.
// * Oversampled rule: positions from the interpolated chart, normals and
//   weights from the interpolated X_u, X_v.
// * Near(x_i) = { l : |x_i - c_l| < eta R_l } plus the patch of x_i, with
//   c_l the weighted node centroid and R_l the largest distance from c_l to
//   the patch's nodes, oversampled points and mapped T0 vertices.
#include "surface.hpp"
#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <unordered_map>

namespace lb {

static inline void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

void Surface::chart(int p, double u, double v, double* K, double* x, double* xu, double* xv) const {
  re->basis(u, v, K);
  const double* a = &cX[(size_t)p * n_p * 3];
  const double* b = &cXu[(size_t)p * n_p * 3];
  const double* c = &cXv[(size_t)p * n_p * 3];
  double x0 = 0, x1 = 0, x2 = 0, u0 = 0, u1 = 0, u2 = 0, v0 = 0, v1 = 0, v2 = 0;
  for (int m = 0; m < n_p; ++m) {
    double k = K[m];
    x0 += k * a[3 * m]; x1 += k * a[3 * m + 1]; x2 += k * a[3 * m + 2];
    u0 += k * b[3 * m]; u1 += k * b[3 * m + 1]; u2 += k * b[3 * m + 2];
    v0 += k * c[3 * m]; v1 += k * c[3 * m + 1]; v2 += k * c[3 * m + 2];
  }
  x[0] = x0; x[1] = x1; x[2] = x2;
  xu[0] = u0; xu[1] = u1; xu[2] = u2;
  xv[0] = v0; xv[1] = v1; xv[2] = v2;
}

void Surface::dchart(int p, double u, double v, double* K, double* du, double* dv) const {
  re->basis(u, v, K);
  const double* a = &cDu[(size_t)p * n_p * 3];
  const double* b = &cDv[(size_t)p * n_p * 3];
  double u0 = 0, u1 = 0, u2 = 0, v0 = 0, v1 = 0, v2 = 0;
  for (int m = 0; m < n_p; ++m) {
    const double k = K[m];
    u0 += k * a[3 * m]; u1 += k * a[3 * m + 1]; u2 += k * a[3 * m + 2];
    v0 += k * b[3 * m]; v1 += k * b[3 * m + 1]; v2 += k * b[3 * m + 2];
  }
  du[0] = u0; du[1] = u1; du[2] = u2;
  dv[0] = v0; dv[1] = v1; dv[2] = v2;
}

void Surface::build_over(const RefElem& reo, OverRule& out) const {
  out.re = &reo;
  out.n_o = reo.n_o;
  out.No = (int64_t)NP * reo.n_o;
  out.s.assign(3 * out.No, 0.0);
  out.nu.assign(3 * out.No, 0.0);
  out.wo.assign(out.No, 0.0);
  int bad = -1;
#pragma omp parallel for schedule(static)
  for (int p = 0; p < NP; ++p) {
    const int64_t o = (int64_t)p * n_p, oo = (int64_t)p * reo.n_o;
    for (int m = 0; m < reo.n_o; ++m) {
      double xs[3] = {0, 0, 0}, su[3] = {0, 0, 0}, sv[3] = {0, 0, 0};
      for (int b = 0; b < n_p; ++b) {
        const double pw = reo.P[m * n_p + b];
        for (int d = 0; d < 3; ++d) {
          xs[d] += pw * X[3 * (o + b) + d];
          su[d] += pw * Xu[3 * (o + b) + d];
          sv[d] += pw * Xv[3 * (o + b) + d];
        }
      }
      double c[3];
      cross3(su, sv, c);
      double j = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
      if (!(j > 0.0)) {
#pragma omp critical
        bad = p;
        j = 1.0;
      }
      for (int d = 0; d < 3; ++d) {
        out.s[3 * (oo + m) + d] = xs[d];
        out.nu[3 * (oo + m) + d] = c[d] / j;
      }
      out.wo[oo + m] = j * reo.over_w[m];
    }
  }
  if (bad >= 0) fail(LB_EGEOM, "degenerate patch %d (zero Jacobian)", bad);
}

void Surface::build(const RefElem& re_, int NP_, const double* X_, const double* Xu_,
                    const double* Xv_, double eta_) {
  re = &re_;
  NP = NP_;
  n_p = re->n_p;
  n_o = re->n_o;
  N = (int64_t)NP * n_p;
  No = (int64_t)NP * n_o;
  eta = eta_;
  X.assign(X_, X_ + 3 * N);
  Xu.assign(Xu_, Xu_ + 3 * N);
  Xv.assign(Xv_, Xv_ + 3 * N);
  for (int64_t i = 0; i < 3 * N; ++i)
    if (!std::isfinite(X[i]) || !std::isfinite(Xu[i]) || !std::isfinite(Xv[i]))
      fail(LB_EINVAL, "non-finite chart sample at node %lld", (long long)(i / 3));
  nrm.resize(3 * N); w.resize(N); J.resize(N); H.resize(N);
  dXu.resize(3 * N); dXv.resize(3 * N);
  cX.resize(3 * N); cXu.resize(3 * N); cXv.resize(3 * N);
  cDu.resize(3 * N); cDv.resize(3 * N);
  s.resize(3 * No); nu.resize(3 * No); wo.resize(No);
  cen.resize(3 * NP); R.resize(NP);
  const std::vector<double>& Du = re->Du;
  const std::vector<double>& Dv = re->Dv;
  int bad = -1;
#pragma omp parallel for schedule(static)
  for (int p = 0; p < NP; ++p) {
    const int64_t o = (int64_t)p * n_p;
    for (int a = 0; a < n_p; ++a) {
      const double* xu = &Xu[3 * (o + a)];
      const double* xv = &Xv[3 * (o + a)];
      double c[3];
      cross3(xu, xv, c);
      double j = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
      if (!(j > 0.0)) {
#pragma omp critical
        bad = p;
        j = 1.0;
      }
      J[o + a] = j;
      for (int d = 0; d < 3; ++d) nrm[3 * (o + a) + d] = c[d] / j;
      w[o + a] = j * re->w_ref[a];
      // spectral derivatives
      double Xuu[3] = {0, 0, 0}, Xvv[3] = {0, 0, 0}, Xuv[3] = {0, 0, 0}, dU[3] = {0, 0, 0}, dV[3] = {0, 0, 0};
      for (int b = 0; b < n_p; ++b) {
        double du = Du[a * n_p + b], dv = Dv[a * n_p + b];
        for (int d = 0; d < 3; ++d) {
          Xuu[d] += du * Xu[3 * (o + b) + d];
          Xvv[d] += dv * Xv[3 * (o + b) + d];
          Xuv[d] += 0.5 * (dv * Xu[3 * (o + b) + d] + du * Xv[3 * (o + b) + d]);
          dU[d] += du * X[3 * (o + b) + d];
          dV[d] += dv * X[3 * (o + b) + d];
        }
      }
      const double* n = &nrm[3 * (o + a)];
      double E = xu[0] * xu[0] + xu[1] * xu[1] + xu[2] * xu[2];
      double F = xu[0] * xv[0] + xu[1] * xv[1] + xu[2] * xv[2];
      double G = xv[0] * xv[0] + xv[1] * xv[1] + xv[2] * xv[2];
      double L2 = Xuu[0] * n[0] + Xuu[1] * n[1] + Xuu[2] * n[2];
      double M2 = Xuv[0] * n[0] + Xuv[1] * n[1] + Xuv[2] * n[2];
      double N2 = Xvv[0] * n[0] + Xvv[1] * n[1] + Xvv[2] * n[2];
      H[o + a] = -(E * N2 - 2.0 * F * M2 + G * L2) / (2.0 * (E * G - F * F));
      for (int d = 0; d < 3; ++d) { dXu[3 * (o + a) + d] = dU[d]; dXv[3 * (o + a) + d] = dV[d]; }
    }
    // modal coefficients: c[m] = sum_b Vinv[m][b] X[b]
    for (int m = 0; m < n_p; ++m)
      for (int d = 0; d < 3; ++d) {
        double sx = 0, su = 0, sv = 0, sdu = 0, sdv = 0;
        for (int b = 0; b < n_p; ++b) {
          double vi = re->Vinv[m * n_p + b];
          sx += vi * X[3 * (o + b) + d];
          su += vi * Xu[3 * (o + b) + d];
          sv += vi * Xv[3 * (o + b) + d];
          sdu += vi * dXu[3 * (o + b) + d];
          sdv += vi * dXv[3 * (o + b) + d];
        }
        cX[3 * (o + m) + d] = sx;
        cXu[3 * (o + m) + d] = su;
        cXv[3 * (o + m) + d] = sv;
        cDu[3 * (o + m) + d] = sdu;
        cDv[3 * (o + m) + d] = sdv;
      }
    // oversampled points
    const int64_t oo = (int64_t)p * n_o;
    for (int m = 0; m < n_o; ++m) {
      double xs[3] = {0, 0, 0}, su[3] = {0, 0, 0}, sv[3] = {0, 0, 0};
      for (int b = 0; b < n_p; ++b) {
        double pw = re->P[m * n_p + b];
        for (int d = 0; d < 3; ++d) {
          xs[d] += pw * X[3 * (o + b) + d];
          su[d] += pw * Xu[3 * (o + b) + d];
          sv[d] += pw * Xv[3 * (o + b) + d];
        }
      }
      double c[3];
      cross3(su, sv, c);
      double j = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
      if (!(j > 0.0)) {
#pragma omp critical
        bad = p;
        j = 1.0;
      }
      for (int d = 0; d < 3; ++d) {
        s[3 * (oo + m) + d] = xs[d];
        nu[3 * (oo + m) + d] = c[d] / j;
      }
      wo[oo + m] = j * re->over_w[m];
    }
    // centre and radius
    double ws = 0, cc[3] = {0, 0, 0};
    for (int a = 0; a < n_p; ++a) {
      ws += w[o + a];
      for (int d = 0; d < 3; ++d) cc[d] += w[o + a] * X[3 * (o + a) + d];
    }
    for (int d = 0; d < 3; ++d) cen[3 * p + d] = cc[d] / ws;
    double r = 0;
    auto upd = [&](const double* y) {
      double dx = y[0] - cen[3 * p], dy = y[1] - cen[3 * p + 1], dz = y[2] - cen[3 * p + 2];
      r = std::max(r, std::sqrt(dx * dx + dy * dy + dz * dz));
    };
    for (int a = 0; a < n_p; ++a) upd(&X[3 * (o + a)]);
    for (int m = 0; m < n_o; ++m) upd(&s[3 * (oo + m)]);
    const double vtx[3][2] = {{0, 0}, {1, 0}, {0, 1}};
    for (int t = 0; t < 3; ++t) {
      double K[64], y[3], yu[3], yv[3];
      chart(p, vtx[t][0], vtx[t][1], K, y, yu, yv);
      upd(y);
    }
    R[p] = r;
  }
  if (bad >= 0) fail(LB_EGEOM, "degenerate patch %d (zero Jacobian)", bad);
}

void Surface::build_near_lists() {
  double Rmax = 0;
  for (int p = 0; p < NP; ++p) Rmax = std::max(Rmax, R[p]);
  const double cell = eta * Rmax;
  double lo[3] = {1e300, 1e300, 1e300};
  for (int p = 0; p < NP; ++p)
    for (int d = 0; d < 3; ++d) lo[d] = std::min(lo[d], cen[3 * p + d]);
  auto key = [&](int64_t ix, int64_t iy, int64_t iz) { return (ix * 2097152 + iy) * 2097152 + iz; };
  auto coord = [&](const double* x, int d) { return (int64_t)std::floor((x[d] - lo[d]) / cell); };
  std::unordered_map<int64_t, std::vector<int>> grid;
  for (int p = 0; p < NP; ++p) {
    const double* c = &cen[3 * p];
    grid[key(coord(c, 0), coord(c, 1), coord(c, 2))].push_back(p);
  }
  std::vector<std::vector<int32_t>> rows(N);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < N; ++i) {
    const double* x = &X[3 * i];
    int64_t cx = coord(x, 0), cy = coord(x, 1), cz = coord(x, 2);
    std::vector<int32_t>& row = rows[i];
    const int self = (int)(i / n_p);
    for (int64_t a = cx - 1; a <= cx + 1; ++a)
      for (int64_t b = cy - 1; b <= cy + 1; ++b)
        for (int64_t c = cz - 1; c <= cz + 1; ++c) {
          auto it = grid.find(key(a, b, c));
          if (it == grid.end()) continue;
          for (int p : it->second) {
            if (!surf_of_patch.empty() && surf_of_patch[p] != surf_of_patch[self]) continue;
            const double* cc = &cen[3 * p];
            double dx = x[0] - cc[0], dy = x[1] - cc[1], dz = x[2] - cc[2];
            if (p == self || std::sqrt(dx * dx + dy * dy + dz * dz) < eta * R[p]) row.push_back(p);
          }
        }
    std::sort(row.begin(), row.end());
    row.erase(std::unique(row.begin(), row.end()), row.end());
  }
  near_ptr.assign(N + 1, 0);
  for (int64_t i = 0; i < N; ++i) near_ptr[i + 1] = near_ptr[i] + (int64_t)rows[i].size();
  near_patch.resize(near_ptr[N]);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i)
    std::copy(rows[i].begin(), rows[i].end(), near_patch.begin() + near_ptr[i]);
}

}  // namespace lb
