// Correction integrals of the locally corrected rule on the device
// (Section 4, eqs. nys-lcq and nys-lcq2): for a target x_i and a near patch
// l, C = A - B with A the accurate integral of the kernel times the Lagrange
// basis of l and B the oversampled far rule restricted to l.
//
// The rules are the host's (quadrature.cpp):
//  * self patch: the reference triangle split at the target node into three
//    Duffy triangles; along each edge the sinh-graded arclength variable in
//    the metric of the chart at the node, panels of self_panel, nt x ns
//    Gauss points; the principal value of the gradient kernels by
//    subtracting the 1/s part and adding f_{-1} ln|B| (Guiggiani-Gigante);
//    the displacement from the node to a point of a ray as the integral of
//    the chart's derivative along the ray (no cancellation of nearly equal
//    positions).
//  * other near patches: recursive 4-way subdivision of the reference
//    triangle, a triangle accepted as a leaf when its distance to the target
//    is at least `adm` times its diameter (or at depth max_depth), and the
//    conical Gauss rule (ru, rw) on every leaf.
//  * far rule: the oversampled points of the patch with weights and the
//    interpolation matrix P; the FP32 variant leaves out the points that the
//    float32 near-field kernel skips (its own float test against the mask
//    radius of the point).
// The accurate integrals accumulate modal moments int K psi_c J and are
// turned into Lagrange-basis values with V^{-T} at the end.
//
// One wavefront per (target, patch) pair (per target for the self rule).
// The quadrature points are taken 64 at a time, one per lane: the lane
// evaluates the modal basis, the chart and the NKER kernels and stages the
// basis values and weighted kernel values in LDS; lane l then owns the
// moments (c, t) = (o / NKER, o % NKER) for o = l, l + 64, l + 128, l + 192
// (NKER n_p <= 256 up to order 7).  The
// subdivision stack of the near rule is wave-uniform and lives in LDS.  The
// order is a template parameter so that a point's n_p basis values stay in
// registers.
#include "kernels.hpp"

#include <hip/hip_runtime.h>

namespace lb {

namespace {

constexpr int NQ_STACK = 72;  // >= 3 max_depth + 1 entries
constexpr double NQ_INV4PI = 0.07957747154594767;

template <int KO>
struct QuadLds {
  static constexpr int NPP = (KO + 1) * (KO + 2) / 2;
  static constexpr int NJ = (KO + 1) * (KO + 1);
  double sc[3][NPP * 3];  // modal coefficients of X, X_u, X_v of the patch
  double sj[3][NJ];       // Jacobi recurrence tables of the modal basis
  double sK[64][NPP + 1]; // basis values of the staged points
  double sKV[64][NKER];   // weighted kernel values of the staged points
  double sM[NKER * NPP];
};

// modal basis psi_c(u, v), c = n (n + 1) / 2 + i (total degree n, index i):
// Legendre-type polynomial of the collapsed coordinate times the Jacobi
// polynomial P_j^{(2i+1,0)} of eta from the recurrence tables ja, jb, jc
template <int KO>
__device__ inline void nq_basis(const double* ja, const double* jb, const double* jc, double u, double v,
                                double* K) {
  const double a = 2.0 * u - 1.0 + v, b = 1.0 - v, eta = 2.0 * v - 1.0;
  double Q[KO + 1];
  Q[0] = 1.0;
  if (KO >= 1) Q[1] = a;
#pragma unroll
  for (int i = 1; i < KO; ++i) Q[i + 1] = ((2 * i + 1) * a * Q[i] - i * b * b * Q[i - 1]) / (i + 1);
#pragma unroll
  for (int i = 0; i <= KO; ++i) {
    double P[KO + 1];
    P[0] = 1.0;
#pragma unroll
    for (int j = 0; j < KO - i; ++j) {
      const int r = i * (KO + 1) + j;
      P[j + 1] = (ja[r] + jb[r] * eta) * P[j] - (j > 0 ? jc[r] * P[j - 1] : 0.0);
    }
#pragma unroll
    for (int j = 0; j <= KO - i; ++j) K[(i + j) * (i + j + 1) / 2 + i] = Q[i] * P[j];
  }
}

template <int KO>
__device__ inline void load_patch(QuadLds<KO>& L, const double* cX, const double* cXu, const double* cXv,
                                  const double* ja, const double* jb, const double* jc, int64_t p, int lane) {
  constexpr int NPP = QuadLds<KO>::NPP;
  for (int e = lane; e < 3 * NPP; e += 64) {
    L.sc[0][e] = cX[p * NPP * 3 + e];
    L.sc[1][e] = cXu[p * NPP * 3 + e];
    L.sc[2][e] = cXv[p * NPP * 3 + e];
  }
  for (int e = lane; e < QuadLds<KO>::NJ; e += 64) {
    L.sj[0][e] = ja[e];
    L.sj[1][e] = jb[e];
    L.sj[2][e] = jc[e];
  }
}

// position of the chart at (u, v)
template <int KO>
__device__ inline void chart_pos(const QuadLds<KO>& L, double u, double v, double* y) {
  double K[QuadLds<KO>::NPP];
  nq_basis<KO>(L.sj[0], L.sj[1], L.sj[2], u, v, K);
  y[0] = y[1] = y[2] = 0.0;
#pragma unroll
  for (int m = 0; m < QuadLds<KO>::NPP; ++m) {
    y[0] += K[m] * L.sc[0][3 * m];
    y[1] += K[m] * L.sc[0][3 * m + 1];
    y[2] += K[m] * L.sc[0][3 * m + 2];
  }
}

// One batch of 64 quadrature points (lane l: point (u, v) with weight wgt
// when `active`): acc[j] += sum_points wgt J psi_c kernel_t for the lane's
// moments (c, t).  Every lane of the wavefront calls it (two barriers).
// dsp (nullable): the displacement x - X(u, v) of the lane's point when the
// caller formed it without cancellation (self rule).
template <int KO>
__device__ inline void quad_batch(QuadLds<KO>& L, int lane, bool active, double u, double v, double wgt,
                                  double x0, double x1, double x2, double n0, double n1, double n2,
                                  double* acc, const double* dsp = nullptr) {
  constexpr int NPP = QuadLds<KO>::NPP;
  double K[NPP];
  double kv[NKER] = {0, 0, 0, 0, 0, 0, 0};
  if (active) {
    nq_basis<KO>(L.sj[0], L.sj[1], L.sj[2], u, v, K);
    double y[3] = {0, 0, 0}, yu[3] = {0, 0, 0}, yv[3] = {0, 0, 0};
#pragma unroll
    for (int m = 0; m < NPP; ++m) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        y[c] += K[m] * L.sc[0][3 * m + c];
        yu[c] += K[m] * L.sc[1][3 * m + c];
        yv[c] += K[m] * L.sc[2][3 * m + c];
      }
    }
    const double c0 = yu[1] * yv[2] - yu[2] * yv[1];
    const double c1 = yu[2] * yv[0] - yu[0] * yv[2];
    const double c2 = yu[0] * yv[1] - yu[1] * yv[0];
    const double J = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    const double nu0 = c0 / J, nu1 = c1 / J, nu2 = c2 / J;
    const double d0 = dsp ? dsp[0] : x0 - y[0], d1 = dsp ? dsp[1] : x1 - y[1], d2 = dsp ? dsp[2] : x2 - y[2];
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    const double ir = 1.0 / sqrt(r2);
    const double ir3 = ir / r2;
    const double ir5 = ir3 / r2;
    kv[0] = ir * NQ_INV4PI;
    kv[1] = -d0 * ir3 * NQ_INV4PI;
    kv[2] = -d1 * ir3 * NQ_INV4PI;
    kv[3] = -d2 * ir3 * NQ_INV4PI;
    kv[4] = n0 * kv[1] + n1 * kv[2] + n2 * kv[3];
    const double m0 = n0 - nu0, m1 = n1 - nu1, m2 = n2 - nu2;
    const double nd = n0 * d0 + n1 * d1 + n2 * d2;
    const double md = m0 * d0 + m1 * d1 + m2 * d2;
    const double nm = n0 * m0 + n1 * m1 + n2 * m2;
    kv[5] = (3.0 * nd * md * ir5 - nm * ir3) * NQ_INV4PI;
    kv[6] = (nu0 * d0 + nu1 * d1 + nu2 * d2) * ir3 * NQ_INV4PI;  // D
    const double f = wgt * J;
#pragma unroll
    for (int t = 0; t < NKER; ++t) kv[t] *= f;
  } else {
#pragma unroll
    for (int m = 0; m < NPP; ++m) K[m] = 0.0;
  }
#pragma unroll
  for (int m = 0; m < NPP; ++m) L.sK[lane][m] = K[m];
#pragma unroll
  for (int t = 0; t < NKER; ++t) L.sKV[lane][t] = kv[t];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int o = lane + 64 * j;
    if (o < NKER * NPP) {
      const int c = o / NKER, t = o % NKER;
      double s = 0;
      for (int l = 0; l < 64; ++l) s += L.sK[l][c] * L.sKV[l][t];
      acc[j] += s;
    }
  }
  __syncthreads();
}

// modal moments -> Lagrange-basis values of one block:
// out[b][t] = sum_c Vinv[c][b] mom[c][t], plus pv[t - 1] for b = pv_b and
// t = 1..4, and -pv[3] for t = 6 (D: the 1/s part of S' with the opposite
// sign), when pv (in LDS, written before the call) is non-null
template <int KO>
__device__ inline void moments_out(QuadLds<KO>& L, int lane, const double* acc, const double* Vinv, double* out,
                                   const double* pv = nullptr, int pv_b = -1) {
  constexpr int NPP = QuadLds<KO>::NPP;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int o = lane + 64 * j;
    if (o < NKER * NPP) L.sM[o] = acc[j];
  }
  __syncthreads();
  for (int o = lane; o < NKER * NPP; o += 64) {
    const int b = o / NKER, t = o % NKER;
    double s = 0;
#pragma unroll
    for (int c = 0; c < NPP; ++c) s += Vinv[c * NPP + b] * L.sM[NKER * c + t];
    if (pv && b == pv_b && t >= 1 && t <= 4) s += pv[t - 1];
    if (pv && b == pv_b && t == 6) s -= pv[3];
    out[o] = s;
  }
}

template <int KO>
__global__ __launch_bounds__(64) void k_near_quad(NearQuadArgs q) {
  __shared__ QuadLds<KO> L;
  __shared__ double stk[NQ_STACK][6];  // subdivision stack: triangle vertices in (u, v)
  __shared__ int sdep[NQ_STACK];
  __shared__ double sv[4][3];          // chart at the vertices and the centroid
  const int lane = threadIdx.x;
  const int64_t w = blockIdx.x;
  if (w >= q.nwork) return;
  const int64_t i = q.row[w];
  load_patch<KO>(L, q.cX, q.cXu, q.cXv, q.ja, q.jb, q.jc, q.patch[w], lane);
  const double x0 = q.X[3 * i], x1 = q.X[3 * i + 1], x2 = q.X[3 * i + 2];
  const double n0 = q.nrm[3 * i], n1 = q.nrm[3 * i + 1], n2 = q.nrm[3 * i + 2];
  if (lane == 0) {
    stk[0][0] = 0; stk[0][1] = 0; stk[0][2] = 1; stk[0][3] = 0; stk[0][4] = 0; stk[0][5] = 1;
    sdep[0] = 0;
  }
  __syncthreads();
  double acc[4] = {0, 0, 0, 0};
  int top = 1;
  while (top > 0) {
    --top;
    double T[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) T[e] = stk[top][e];
    const int depth = sdep[top];
    if (lane < 4) {
      const double u = lane < 3 ? T[2 * lane] : (T[0] + T[2] + T[4]) / 3.0;
      const double v = lane < 3 ? T[2 * lane + 1] : (T[1] + T[3] + T[5]) / 3.0;
      double y[3];
      chart_pos<KO>(L, u, v, y);
      sv[lane][0] = y[0]; sv[lane][1] = y[1]; sv[lane][2] = y[2];
    }
    __syncthreads();
    auto dist = [&](int a, int b) {
      const double d0 = sv[a][0] - sv[b][0], d1 = sv[a][1] - sv[b][1], d2 = sv[a][2] - sv[b][2];
      return sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    };
    const double diam = fmax(dist(0, 1), fmax(dist(1, 2), dist(2, 0)));
    const double e0 = x0 - sv[3][0], e1 = x1 - sv[3][1], e2 = x2 - sv[3][2];
    const double dd = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
    __syncthreads();  // sv and the top of the stack are rewritten below
    if (dd >= q.adm * diam || depth >= q.max_depth) {
      const double e1u = T[2] - T[0], e1v = T[3] - T[1];
      const double e2u = T[4] - T[0], e2v = T[5] - T[1];
      const double area2 = fabs(e1u * e2v - e1v * e2u);
      for (int pt0 = 0; pt0 < q.nq; pt0 += 64) {
        const int pt = pt0 + lane;
        const bool act = pt < q.nq;
        double u = 0, v = 0, wgt = 0;
        if (act) {
          u = T[0] + q.ru[2 * pt] * e1u + q.ru[2 * pt + 1] * e2u;
          v = T[1] + q.ru[2 * pt] * e1v + q.ru[2 * pt + 1] * e2v;
          wgt = area2 * q.rw[pt];
        }
        quad_batch<KO>(L, lane, act, u, v, wgt, x0, x1, x2, n0, n1, n2, acc);
      }
    } else {
      // the four children, pushed in the host's order (the last is taken next)
      const double m01u = 0.5 * (T[0] + T[2]), m01v = 0.5 * (T[1] + T[3]);
      const double m12u = 0.5 * (T[2] + T[4]), m12v = 0.5 * (T[3] + T[5]);
      const double m20u = 0.5 * (T[4] + T[0]), m20v = 0.5 * (T[5] + T[1]);
      if (lane == 0) {
        const double ch[4][6] = {{T[0], T[1], m01u, m01v, m20u, m20v},
                                 {m01u, m01v, T[2], T[3], m12u, m12v},
                                 {m20u, m20v, m12u, m12v, T[4], T[5]},
                                 {m12u, m12v, m20u, m20v, m01u, m01v}};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
          for (int e = 0; e < 6; ++e) stk[top + c][e] = ch[c][e];
          sdep[top + c] = depth + 1;
        }
      }
      top += 4;
      __syncthreads();
    }
  }
  moments_out<KO>(L, lane, acc, q.Vinv, q.A + q.blk[w] * NKER * QuadLds<KO>::NPP);
}

template <int KO>
__global__ __launch_bounds__(64) void k_self_quad(SelfQuadArgs q) {
  constexpr int NPP = QuadLds<KO>::NPP;
  __shared__ QuadLds<KO> L;
  __shared__ double spv[64][4];
  __shared__ double spvs[4];
  __shared__ double sdc[2][NPP * 3];  // modal coefficients of the chart's derivatives
  __shared__ double smr[2][4];        // Gauss rule of the displacement integral
  const int lane = threadIdx.x;
  const int64_t i = blockIdx.x;
  if (i >= q.N) return;
  const int64_t blk = q.sblk[i];
  if (blk < 0) return;  // own patch not in the near list: no self block
  const int64_t p = i / NPP;
  const int a = (int)(i % NPP);
  load_patch<KO>(L, q.cX, q.cXu, q.cXv, q.ja, q.jb, q.jc, p, lane);
  for (int e = lane; e < 3 * NPP; e += 64) {
    sdc[0][e] = q.cDu[p * NPP * 3 + e];
    sdc[1][e] = q.cDv[p * NPP * 3 + e];
  }
  const int nm = q.nm;
  if (lane < nm) {
    smr[0][lane] = q.mg[lane];
    smr[1][lane] = q.mw[lane];
  }
  __syncthreads();
  const double u0 = q.uv[2 * a], v0 = q.uv[2 * a + 1];
  const double x0 = q.X[3 * i], x1 = q.X[3 * i + 1], x2 = q.X[3 * i + 2];
  const double n0 = q.nrm[3 * i], n1 = q.nrm[3 * i + 1], n2 = q.nrm[3 * i + 2];
  const double bu0 = q.dXu[3 * i], bu1 = q.dXu[3 * i + 1], bu2 = q.dXu[3 * i + 2];
  const double bv0 = q.dXv[3 * i], bv1 = q.dXv[3 * i + 1], bv2 = q.dXv[3 * i + 2];
  const double Ji = q.J[i];
  const int ns = q.ns, nt = q.nt;
  double sub = 0;
  for (int js = 0; js < ns; ++js) sub += q.gw[js] / q.g[js];
  // metric of the interpolated chart at the node
  const double G11 = bu0 * bu0 + bu1 * bu1 + bu2 * bu2;
  const double G12 = bu0 * bv0 + bu1 * bv1 + bu2 * bv2;
  const double G22 = bv0 * bv0 + bv1 * bv1 + bv2 * bv2;
  auto gdot = [&](double a1, double a2, double b1, double b2) {
    return a1 * (G11 * b1 + G12 * b2) + a2 * (G12 * b1 + G22 * b2);
  };
  double acc[4] = {0, 0, 0, 0};
  double pv[4] = {0, 0, 0, 0};
  for (int e = 0; e < 3; ++e) {
    // edge e of the reference triangle: (0,0)-(1,0), (1,0)-(0,1), (0,1)-(0,0)
    const double ax = e == 1 ? 1.0 : 0.0, ay = e == 2 ? 1.0 : 0.0;
    const double bx = e == 0 ? 1.0 : 0.0, by = e == 1 ? 1.0 : 0.0;
    const double ex = bx - ax, ey = by - ay;
    const double eG = sqrt(gdot(ex, ey, ex, ey));
    const double tstar = -gdot(ax - u0, ay - v0, ex, ey) / (eG * eG);
    const double fx = ax + tstar * ex, fy = ay + tstar * ey;
    const double h = sqrt(gdot(fx - u0, fy - v0, fx - u0, fy - v0));
    const double c0 = fabs((ax - u0) * ey - (ay - v0) * ex);
    const double ta = asinh((0.0 - tstar) * eG / h);
    const double tb = asinh((1.0 - tstar) * eG / h);
    // (a span that is not finite, from a degenerate chart, gets one panel)
    const double span = tb - ta;
    const int npan = span > 0.0 && span < 4096.0 * q.panel ? max(1, (int)ceil(span / q.panel)) : 1;
    const double dl = (tb - ta) / npan;
    const int npts = npan * nt * ns;
    for (int q0 = 0; q0 < npts; q0 += 64) {
      const int qq = q0 + lane;
      const bool act = qq < npts;
      double u = 0, v = 0, wgt = 0;
      double dsp[3] = {0, 0, 0};
      if (act) {
        const int js = qq % ns, jt = (qq / ns) % nt, ip = qq / (ns * nt);
        const double t = ta + dl * (ip + q.tg[jt]);
        const double wt = dl * q.tw[jt];
        const double sh = sinh(t), chh = cosh(t);
        const double du = fx + (h * sh / eG) * ex - u0, dv = fy + (h * sh / eG) * ey - v0;
        const double jac = c0 * h * chh / eG;
        const double s = q.g[js];
        u = u0 + s * du;
        v = v0 + s * dv;
        wgt = wt * q.gw[js] * jac * s;
        // x_i - X(u, v) = -s sum_j mw_j X'(u0 + mg_j s e) e, e = (du, dv)
        for (int jm = 0; jm < nm; ++jm) {
          double K[NPP];
          const double sj = smr[0][jm] * s;
          nq_basis<KO>(L.sj[0], L.sj[1], L.sj[2], u0 + sj * du, v0 + sj * dv, K);
          double t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
          for (int m = 0; m < NPP; ++m) {
            t0 += K[m] * (sdc[0][3 * m] * du + sdc[1][3 * m] * dv);
            t1 += K[m] * (sdc[0][3 * m + 1] * du + sdc[1][3 * m + 1] * dv);
            t2 += K[m] * (sdc[0][3 * m + 2] * du + sdc[1][3 * m + 2] * dv);
          }
          dsp[0] += smr[1][jm] * t0;
          dsp[1] += smr[1][jm] * t1;
          dsp[2] += smr[1][jm] * t2;
        }
        dsp[0] *= -s;
        dsp[1] *= -s;
        dsp[2] *= -s;
        if (js == 0) {
          // principal-value term of the gradient kernels at column a
          const double B0 = du * bu0 + dv * bv0, B1 = du * bu1 + dv * bv1, B2 = du * bu2 + dv * bv2;
          const double Bn = sqrt(B0 * B0 + B1 * B1 + B2 * B2);
          const double f = Ji * jac * NQ_INV4PI / (Bn * Bn * Bn);
          const double lg = log(Bn) - sub;
          const double fm0 = B0 * f, fm1 = B1 * f, fm2 = B2 * f;
          pv[0] += wt * fm0 * lg;
          pv[1] += wt * fm1 * lg;
          pv[2] += wt * fm2 * lg;
          pv[3] += wt * (fm0 * n0 + fm1 * n1 + fm2 * n2) * lg;
        }
      }
      quad_batch<KO>(L, lane, act, u, v, wgt, x0, x1, x2, n0, n1, n2, acc, dsp);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) spv[lane][t] = pv[t];
  __syncthreads();
  if (lane < 4) {
    double s = 0;
    for (int l = 0; l < 64; ++l) s += spv[l][lane];
    spvs[lane] = s;
  }
  // (moments_out's barrier orders spvs before its use)
  moments_out<KO>(L, lane, acc, q.Vinv, q.A + blk * NKER * NPP, spvs, a);
}

// C = A - B for one block per wavefront, B and B32 accumulated over the
// oversampled points of the patch 64 at a time; written in the packed
// layouts of the combine kernels (k = 4: S, Gx, Gy, Gz; k = 3: S, S', S''+D';
// k = 1: D).
__global__ __launch_bounds__(64) void k_far_rule(FarRuleArgs q) {
  __shared__ double skv[64][2 * NKER];  // kernel x weight of the staged points: FP64 rule, FP32-masked rule
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x;
  if (b >= q.nb) return;
  const int n_p = q.n_p, n_o = q.n_o;
  const int64_t i = q.brow[b];
  const int64_t p = q.patch[b];
  const double x0 = q.X[3 * i], x1 = q.X[3 * i + 1], x2 = q.X[3 * i + 2];
  const double n0 = q.nrm[3 * i], n1 = q.nrm[3 * i + 1], n2 = q.nrm[3 * i + 2];
  const float tx = (float)x0, ty = (float)x1, tz = (float)x2;
  double b64[4] = {0, 0, 0, 0}, b32[4] = {0, 0, 0, 0};
  for (int m0 = 0; m0 < n_o; m0 += 64) {
    const int m = m0 + lane;
    double kv[NKER] = {0, 0, 0, 0, 0, 0, 0};
    bool masked = true;
    if (m < n_o) {
      const int64_t sm = p * n_o + m;
      const double y0 = q.s[3 * sm], y1 = q.s[3 * sm + 1], y2 = q.s[3 * sm + 2];
      const double nu0 = q.nu[3 * sm], nu1 = q.nu[3 * sm + 1], nu2 = q.nu[3 * sm + 2];
      const double d0 = x0 - y0, d1 = x1 - y1, d2 = x2 - y2;
      const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
      const double ir = 1.0 / sqrt(r2);
      const double ir3 = ir / r2;
      const double ir5 = ir3 / r2;
      kv[0] = ir * NQ_INV4PI;
      kv[1] = -d0 * ir3 * NQ_INV4PI;
      kv[2] = -d1 * ir3 * NQ_INV4PI;
      kv[3] = -d2 * ir3 * NQ_INV4PI;
      kv[4] = n0 * kv[1] + n1 * kv[2] + n2 * kv[3];
      const double m0v = n0 - nu0, m1v = n1 - nu1, m2v = n2 - nu2;
      const double nd = n0 * d0 + n1 * d1 + n2 * d2;
      const double md = m0v * d0 + m1v * d1 + m2v * d2;
      const double nm = n0 * m0v + n1 * m1v + n2 * m2v;
      kv[5] = (3.0 * nd * md * ir5 - nm * ir3) * NQ_INV4PI;
      kv[6] = (nu0 * d0 + nu1 * d1 + nu2 * d2) * ir3 * NQ_INV4PI;
      const double wm = q.wo[sm];
#pragma unroll
      for (int t = 0; t < NKER; ++t) kv[t] *= wm;
      // the float32 near-field kernel's test, in its arithmetic
      const float dx = __fsub_rn(tx, (float)y0), dy = __fsub_rn(ty, (float)y1), dz = __fsub_rn(tz, (float)y2);
      const float fr2 = __fmaf_rn(dz, dz, __fmaf_rn(dy, dy, __fmul_rn(dx, dx)));
      masked = q.rm2 ? fr2 < q.rm2[sm] : false;
    }
#pragma unroll
    for (int t = 0; t < NKER; ++t) {
      skv[lane][t] = kv[t];
      skv[lane][NKER + t] = masked ? 0.0 : kv[t];
    }
    __syncthreads();
    const int lim = min(64, n_o - m0);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = lane + 64 * j;
      if (o < NKER * n_p) {
        const int k = o / NKER, t = o % NKER;
        double s64 = 0, s32 = 0;
        for (int l = 0; l < lim; ++l) {
          const double P = q.P[(int64_t)(m0 + l) * n_p + k];
          s64 += P * skv[l][t];
          s32 += P * skv[l][NKER + t];
        }
        b64[j] += s64;
        b32[j] += s32;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int o = lane + 64 * j;
    if (o < NKER * n_p) {
      const int k = o / NKER, t = o % NKER;
      const double a = q.A[b * NKER * n_p + o];
      const double c64 = a - b64[j];
      const float c32 = (float)(a - b32[j]);
      const int64_t e = b * n_p + k;
      if (t < 4) {
        if (q.v4_64) q.v4_64[4 * e + t] = c64;
        if (q.v4_32) q.v4_32[4 * e + t] = c32;
      }
      if (t == 0 || t == 4 || t == 5) {
        const int u = t == 0 ? 0 : t - 3;
        if (q.v3_64) q.v3_64[3 * e + u] = c64;
        if (q.v3_32) q.v3_32[3 * e + u] = c32;
      }
      if (t == 6) {
        if (q.vD_64) q.vD_64[e] = c64;
        if (q.vD_32) q.vD_32[e] = c32;
      }
    }
  }
}

}  // namespace

hipError_t launch_near_quad(const NearQuadArgs& q, hipStream_t st) {
  if (q.nwork <= 0) return hipSuccess;
  if (q.nwork > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid((unsigned)q.nwork), blk(64);
  switch (q.k) {
    case 1: hipLaunchKernelGGL(k_near_quad<1>, grid, blk, 0, st, q); break;
    case 2: hipLaunchKernelGGL(k_near_quad<2>, grid, blk, 0, st, q); break;
    case 3: hipLaunchKernelGGL(k_near_quad<3>, grid, blk, 0, st, q); break;
    case 4: hipLaunchKernelGGL(k_near_quad<4>, grid, blk, 0, st, q); break;
    case 5: hipLaunchKernelGGL(k_near_quad<5>, grid, blk, 0, st, q); break;
    case 6: hipLaunchKernelGGL(k_near_quad<6>, grid, blk, 0, st, q); break;
    case 7: hipLaunchKernelGGL(k_near_quad<7>, grid, blk, 0, st, q); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_self_quad(const SelfQuadArgs& q, hipStream_t st) {
  if (q.N <= 0) return hipSuccess;
  if (q.N > 0x7fffffff || q.ns < 1 || q.nt < 1 || !(q.panel > 0) || q.nm < 1 || q.nm > 4 || !q.cDu || !q.cDv)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)q.N), blk(64);
  switch (q.k) {
    case 1: hipLaunchKernelGGL(k_self_quad<1>, grid, blk, 0, st, q); break;
    case 2: hipLaunchKernelGGL(k_self_quad<2>, grid, blk, 0, st, q); break;
    case 3: hipLaunchKernelGGL(k_self_quad<3>, grid, blk, 0, st, q); break;
    case 4: hipLaunchKernelGGL(k_self_quad<4>, grid, blk, 0, st, q); break;
    case 5: hipLaunchKernelGGL(k_self_quad<5>, grid, blk, 0, st, q); break;
    case 6: hipLaunchKernelGGL(k_self_quad<6>, grid, blk, 0, st, q); break;
    case 7: hipLaunchKernelGGL(k_self_quad<7>, grid, blk, 0, st, q); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_far_rule(const FarRuleArgs& q, hipStream_t st) {
  if (q.nb <= 0) return hipSuccess;
  if (q.nb > 0x7fffffff || q.n_p < 1 || NKER * q.n_p > 256 || q.n_o < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_far_rule, dim3((unsigned)q.nb), dim3(64), 0, st, q);
  return hipGetLastError();
}

}  // namespace lb
