// Locally corrected quadrature (Section 4, eqs. nys-lcq and nys-lcq2).
//
// For target x_i and near patch l the stored correction is C = A - B with
//   A_k = int_T0 K(x_i, X_l(u,v)) L_k(u,v) J_l(u,v) du dv   (accurate rule)
//   B_k = sum_m K(x_i, s_lm) w^over_lm P_mk                  (far rule)
// The paper's generalized Gaussian and adaptive rules belong to a third-party
// package; the rules used here are:
//  * self patch: T0 is split at the target node into three triangles, each
//    parametrized by the Duffy map (s in [0,1] along the ray from the node,
//    and a coordinate along the opposite edge).  The edge coordinate is the
//    arclength x = h sinh(t) from the closest point, both measured in the
//    metric of the chart at the node (h = distance to the edge), which removes
//    the 1/(h^2 + x^2) behaviour of nodes near an edge; t is split into
//    panels of length <= self_panel with self_nt Gauss points each.
//    The gradient kernel is a Cauchy principal value whose exclusion set is a
//    ball in R^3: the 1/s part f_{-1}/s of the integrand is subtracted and its
//    integral from the ball radius to 1 is added analytically; the ln(eps)
//    parts cancel over the full angle, leaving f_{-1} ln|B| with B the tangent
//    of the interpolated chart along the ray (Guiggiani-Gigante subtraction).
//    The double layer D takes the same subtraction as S' with the opposite
//    sign (its 1/s part is non-zero only through the chart's interpolation
//    error).
//    The displacement from the node to a point s e of a ray is formed without
//    cancellation: the interpolated chart is a polynomial of degree k, so
//    X(u0 + s e) - X(u0) = s int_0^1 X'(u0 + t s e) e dt exactly with
//    ceil(k/2) Gauss points in t (X' the derivative of the interpolant, of
//    degree k - 1); subtracting two nearly equal positions instead would put
//    a rounding error of order |X| eps / |x - y| into the 1/r^2 kernels.
//  * other near patches: recursive 4-way subdivision of T0 with a conical
//    Gauss rule per leaf, leaf accepted when its distance to the target is at
//    least near_adm times its diameter.
// Integrals accumulate modal moments int K psi_c, turned into Lagrange-basis
// values with V^{-T} at the end.
#include "surface.hpp"
#include "common.hpp"

#include <cmath>
#include <cstring>

namespace lb {

static const double INV4PI = 0.25 / M_PI;

// S, Gx, Gy, Gz, S', S''+D', D at target x (normal n) from source y (normal
// nu); D = grad_y G . nu, the double layer (Section 3).
static inline void kernel7_d(const double* d, const double* n, const double* nu, double* k) {
  const double d0 = d[0], d1 = d[1], d2 = d[2];
  double r2 = d0 * d0 + d1 * d1 + d2 * d2;
  double ir = 1.0 / std::sqrt(r2);
  double ir3 = ir / r2;
  double ir5 = ir3 / r2;
  k[0] = ir * INV4PI;
  k[1] = -d0 * ir3 * INV4PI;
  k[2] = -d1 * ir3 * INV4PI;
  k[3] = -d2 * ir3 * INV4PI;
  k[4] = n[0] * k[1] + n[1] * k[2] + n[2] * k[3];
  double m0 = n[0] - nu[0], m1 = n[1] - nu[1], m2 = n[2] - nu[2];
  double nd = n[0] * d0 + n[1] * d1 + n[2] * d2;
  double md = m0 * d0 + m1 * d1 + m2 * d2;
  double nm = n[0] * m0 + n[1] * m1 + n[2] * m2;
  k[5] = (3.0 * nd * md * ir5 - nm * ir3) * INV4PI;
  k[6] = (nu[0] * d0 + nu[1] * d1 + nu[2] * d2) * ir3 * INV4PI;
}

static inline void kernel7(const double* x, const double* n, const double* y, const double* nu, double* k) {
  const double d[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
  kernel7_d(d, n, nu, k);
}

// Accumulate weight * kernel(x, chart(p, u, v)) * psi_c(u, v) into mom[c][NKER];
// dsp (nullable) is the displacement x - chart(p, u, v) when the caller has
// formed it without cancellation (self rule).
static inline void accum_point(const Surface& S, int p, double u, double v, double wgt,
                               const double* x, const double* n, double* mom, double* kv_out,
                               const double* dsp = nullptr) {
  double K[64], y[3], yu[3], yv[3], c[3];
  S.chart(p, u, v, K, y, yu, yv);
  const double dxy[3] = {x[0] - y[0], x[1] - y[1], x[2] - y[2]};
  c[0] = yu[1] * yv[2] - yu[2] * yv[1];
  c[1] = yu[2] * yv[0] - yu[0] * yv[2];
  c[2] = yu[0] * yv[1] - yu[1] * yv[0];
  double J = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  double nu[3] = {c[0] / J, c[1] / J, c[2] / J};
  double kv[NKER];
  kernel7_d(dsp ? dsp : dxy, n, nu, kv);
  double f = wgt * J;
  for (int t = 0; t < NKER; ++t) kv[t] *= f;
  for (int m = 0; m < S.n_p; ++m)
    for (int t = 0; t < NKER; ++t) mom[NKER * m + t] += K[m] * kv[t];
  if (kv_out)
    for (int t = 0; t < NKER; ++t) kv_out[t] = kv[t];
}

// moments -> Lagrange values: out[b][t] = sum_c Vinv[c][b] mom[c][t]
static void moments_to_nodal(const Surface& S, const double* mom, double* out) {
  const int n_p = S.n_p;
  for (int b = 0; b < n_p; ++b)
    for (int t = 0; t < NKER; ++t) {
      double acc = 0;
      for (int c = 0; c < n_p; ++c) acc += S.re->Vinv[c * n_p + b] * mom[NKER * c + t];
      out[NKER * b + t] = acc;
    }
}

static void self_integral(const Surface& S, int64_t i, const QuadOpts& qo,
                          const std::vector<double>& g, const std::vector<double>& gw,
                          const std::vector<double>& tg, const std::vector<double>& tw,
                          double* out) {
  const int n_p = S.n_p;
  const int p = (int)(i / n_p), a = (int)(i % n_p);
  const double u0 = S.re->uv[2 * a], v0 = S.re->uv[2 * a + 1];
  const double* x = &S.X[3 * i];
  const double* n = &S.nrm[3 * i];
  const double* bu = &S.dXu[3 * i];
  const double* bv = &S.dXv[3 * i];
  const double Ji = S.J[i];
  const int ns = qo.self_n, nt = (int)tg.size();
  // Gauss rule in the ray variable of the displacement integral (exact for
  // the degree k - 1 of the chart's derivative)
  std::vector<double> mg, mw;
  gauss_legendre01((S.re->k + 1) / 2, mg, mw);
  const int nm = (int)mg.size();
  double mom[NKER * 64];
  std::memset(mom, 0, sizeof(double) * NKER * n_p);
  double pv[4] = {0, 0, 0, 0};
  double sub = 0;
  for (int js = 0; js < ns; ++js) sub += gw[js] / g[js];
  // metric of the interpolated chart at the node: the edge coordinate is the
  // metric arclength from the closest point, graded with sinh
  const double G11 = bu[0] * bu[0] + bu[1] * bu[1] + bu[2] * bu[2];
  const double G12 = bu[0] * bv[0] + bu[1] * bv[1] + bu[2] * bv[2];
  const double G22 = bv[0] * bv[0] + bv[1] * bv[1] + bv[2] * bv[2];
  auto gdot = [&](double a1, double a2, double b1, double b2) { return a1 * (G11 * b1 + G12 * b2) + a2 * (G12 * b1 + G22 * b2); };
  const double vx[3] = {0.0, 1.0, 0.0}, vy[3] = {0.0, 0.0, 1.0};
  for (int e = 0; e < 3; ++e) {
    const double ax = vx[e], ay = vy[e], bx = vx[(e + 1) % 3], by = vy[(e + 1) % 3];
    const double ex = bx - ax, ey = by - ay;
    const double eG = std::sqrt(gdot(ex, ey, ex, ey));
    const double tstar = -gdot(ax - u0, ay - v0, ex, ey) / (eG * eG);
    const double fx = ax + tstar * ex, fy = ay + tstar * ey;
    const double h = std::sqrt(gdot(fx - u0, fy - v0, fx - u0, fy - v0));
    const double c0 = std::fabs((ax - u0) * ey - (ay - v0) * ex);
    const double ta = std::asinh((0.0 - tstar) * eG / h);
    const double tb = std::asinh((1.0 - tstar) * eG / h);
    const int npan = std::max(1, (int)std::ceil((tb - ta) / qo.self_panel));
    const double dl = (tb - ta) / npan;
    for (int ip = 0; ip < npan; ++ip)
      for (int jt = 0; jt < nt; ++jt) {
        const double t = ta + dl * (ip + tg[jt]);
        const double wt = dl * tw[jt];
        const double sh = std::sinh(t), ch = std::cosh(t);
        const double du = fx + (h * sh / eG) * ex - u0, dv = fy + (h * sh / eG) * ey - v0;
        const double jac = c0 * h * ch / eG;
        for (int js = 0; js < ns; ++js) {
          const double sv = g[js];
          // x - X(u0 + s e) = -s sum_j mw_j X'(u0 + mg_j s e) e without cancellation
          double dsp[3] = {0, 0, 0}, K[64], pu[3], pv3[3];
          for (int jm = 0; jm < nm; ++jm) {
            S.dchart(p, u0 + mg[jm] * sv * du, v0 + mg[jm] * sv * dv, K, pu, pv3);
            for (int c = 0; c < 3; ++c) dsp[c] += mw[jm] * (pu[c] * du + pv3[c] * dv);
          }
          for (int c = 0; c < 3; ++c) dsp[c] *= -sv;
          accum_point(S, p, u0 + sv * du, v0 + sv * dv, wt * gw[js] * jac * sv, x, n, mom, nullptr, dsp);
        }
        // principal-value term of the gradient kernels at column a
        double B[3] = {du * bu[0] + dv * bv[0], du * bu[1] + dv * bv[1], du * bu[2] + dv * bv[2]};
        double Bn = std::sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
        double f = Ji * jac * INV4PI / (Bn * Bn * Bn);
        double lg = std::log(Bn) - sub;
        double fm[3] = {B[0] * f, B[1] * f, B[2] * f};
        pv[0] += wt * fm[0] * lg;
        pv[1] += wt * fm[1] * lg;
        pv[2] += wt * fm[2] * lg;
        pv[3] += wt * (fm[0] * n[0] + fm[1] * n[1] + fm[2] * n[2]) * lg;
      }
  }
  moments_to_nodal(S, mom, out);
  for (int t = 0; t < 4; ++t) out[NKER * a + 1 + t] += pv[t];
  // D has the 1/s^2 part of S' with the opposite sign (nu . d = -n . d to
  // first order along the ray): the same principal value
  out[NKER * a + 6] -= pv[3];
}

static void near_integral(const Surface& S, int64_t i, int p, const QuadOpts& qo,
                          const std::vector<double>& ru, const std::vector<double>& rw,
                          double* out) {
  const int n_p = S.n_p;
  const double* x = &S.X[3 * i];
  const double* n = &S.nrm[3 * i];
  double mom[NKER * 64];
  std::memset(mom, 0, sizeof(double) * NKER * n_p);
  struct Tri { double v[6]; int depth; };
  Tri stack[4 * 20 + 8];
  int top = 0;
  stack[top++] = Tri{{0, 0, 1, 0, 0, 1}, 0};
  const int nq = (int)rw.size();
  while (top > 0) {
    Tri T = stack[--top];
    double Xv[3][3], Xc[3], K[64], yu[3], yv[3];
    for (int c = 0; c < 3; ++c) S.chart(p, T.v[2 * c], T.v[2 * c + 1], K, Xv[c], yu, yv);
    S.chart(p, (T.v[0] + T.v[2] + T.v[4]) / 3.0, (T.v[1] + T.v[3] + T.v[5]) / 3.0, K, Xc, yu, yv);
    auto dist = [](const double* a, const double* b) {
      return std::sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) + (a[2] - b[2]) * (a[2] - b[2]));
    };
    double diam = std::max(dist(Xv[0], Xv[1]), std::max(dist(Xv[1], Xv[2]), dist(Xv[2], Xv[0])));
    double dd = dist(x, Xc);
    if (dd >= qo.near_adm * diam || T.depth >= qo.max_depth) {
      const double e1u = T.v[2] - T.v[0], e1v = T.v[3] - T.v[1];
      const double e2u = T.v[4] - T.v[0], e2v = T.v[5] - T.v[1];
      const double area2 = std::fabs(e1u * e2v - e1v * e2u);
      for (int m = 0; m < nq; ++m) {
        double u = T.v[0] + ru[2 * m] * e1u + ru[2 * m + 1] * e2u;
        double v = T.v[1] + ru[2 * m] * e1v + ru[2 * m + 1] * e2v;
        accum_point(S, p, u, v, area2 * rw[m], x, n, mom, nullptr);
      }
    } else {
      const double* q = T.v;
      double m01[2] = {0.5 * (q[0] + q[2]), 0.5 * (q[1] + q[3])};
      double m12[2] = {0.5 * (q[2] + q[4]), 0.5 * (q[3] + q[5])};
      double m20[2] = {0.5 * (q[4] + q[0]), 0.5 * (q[5] + q[1])};
      int d = T.depth + 1;
      stack[top++] = Tri{{q[0], q[1], m01[0], m01[1], m20[0], m20[1]}, d};
      stack[top++] = Tri{{m01[0], m01[1], q[2], q[3], m12[0], m12[1]}, d};
      stack[top++] = Tri{{m20[0], m20[1], m12[0], m12[1], q[4], q[5]}, d};
      stack[top++] = Tri{{m12[0], m12[1], m20[0], m20[1], m01[0], m01[1]}, d};
    }
  }
  moments_to_nodal(S, mom, out);
}

void near_leaf_rule(int q, std::vector<double>& ru, std::vector<double>& rw) {
  std::vector<double> a, aw;
  gauss_legendre01(q, a, aw);
  ru.assign(2 * q * q, 0.0);
  rw.assign(q * q, 0.0);
  for (int jb = 0; jb < q; ++jb)
    for (int ia = 0; ia < q; ++ia) {
      int m = jb * q + ia;
      ru[2 * m] = a[ia] * (1.0 - a[jb]);
      ru[2 * m + 1] = a[jb];
      rw[m] = aw[ia] * aw[jb] * (1.0 - a[jb]);
    }
}

void near_integrals(const Surface& S, const QuadOpts& qo, std::vector<double>& A, bool self_only) {
  const int n_p = S.n_p;
  const int64_t nb = S.near_ptr[S.N];
  if (!self_only) A.assign((size_t)nb * n_p * NKER, 0.0);
  std::vector<double> g, gw, tg, tw;
  gauss_legendre01(qo.self_n, g, gw);
  gauss_legendre01(qo.self_nt, tg, tw);
  std::vector<double> ru, rw;
  near_leaf_rule(qo.near_q, ru, rw);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < S.N; ++i) {
    const int self = (int)(i / n_p);
    for (int64_t b = S.near_ptr[i]; b < S.near_ptr[i + 1]; ++b) {
      double* out = &A[(size_t)b * n_p * NKER];
      int p = S.near_patch[b];
      if (p == self)
        self_integral(S, i, qo, g, gw, tg, tw, out);
      else if (!self_only)
        near_integral(S, i, p, qo, ru, rw, out);
    }
  }
}

void far_rule_blocks(const Surface& S, const std::vector<float>& rm2_f32,
                     const std::vector<float>& tx32, const std::vector<float>& sx32,
                     bool fp32_mask, std::vector<double>& B, const OverRule* over) {
  const int n_p = S.n_p, n_o = over ? over->n_o : S.n_o;
  const int64_t nb = S.near_ptr[S.N];
  B.assign((size_t)nb * n_p * NKER, 0.0);
  const std::vector<double>& P = over ? over->re->P : S.re->P;
  const std::vector<double>& Ss = over ? over->s : S.s;
  const std::vector<double>& Snu = over ? over->nu : S.nu;
  const std::vector<double>& Swo = over ? over->wo : S.wo;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < S.N; ++i) {
    const double* x = &S.X[3 * i];
    const double* n = &S.nrm[3 * i];
    for (int64_t b = S.near_ptr[i]; b < S.near_ptr[i + 1]; ++b) {
      double* out = &B[(size_t)b * n_p * NKER];
      const int64_t p = S.near_patch[b];
      for (int m = 0; m < n_o; ++m) {
        const int64_t sm = p * n_o + m;
        if (fp32_mask) {
          // the float32 near-field kernel's own test, in its own arithmetic
          float dx = tx32[3 * i] - sx32[3 * sm];
          float dy = tx32[3 * i + 1] - sx32[3 * sm + 1];
          float dz = tx32[3 * i + 2] - sx32[3 * sm + 2];
          float r2 = std::fmaf(dz, dz, std::fmaf(dy, dy, dx * dx));
          if (r2 < rm2_f32[sm]) continue;
        }
        double kv[NKER];
        kernel7(x, n, &Ss[3 * sm], &Snu[3 * sm], kv);
        const double wm = Swo[sm];
        for (int t = 0; t < NKER; ++t) kv[t] *= wm;
        const double* Pm = &P[(size_t)m * n_p];
        for (int k = 0; k < n_p; ++k)
          for (int t = 0; t < NKER; ++t) out[NKER * k + t] += Pm[k] * kv[t];
      }
    }
  }
}

}  // namespace lb
