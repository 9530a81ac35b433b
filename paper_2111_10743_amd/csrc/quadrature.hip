// Near-patch quadrature of the locally corrected rule on the device
// (Section 4, eq. nys-lcq2: the accurate integrals A of the corrections
// C = A - B, for a target and a near patch other than its own).
//
// The rule is the host's (quadrature.cpp): recursive 4-way subdivision of the
// reference triangle, a triangle accepted as a leaf when its distance to the
// target is at least `adm` times its diameter (or at depth max_depth), and
// the conical Gauss rule (ru, rw) on every leaf.  The integrals accumulate
// modal moments int K psi_c J, turned into Lagrange-basis values with V^{-T}
// at the end.
//
// One wavefront per (target, patch) pair.  The subdivision stack is
// wave-uniform and lives in LDS; lanes 0..3 evaluate the chart at the three
// vertices and the centroid of the triangle on top; on a leaf, lane l takes
// point l of the rule (modal basis, chart, the six kernels) and stages its
// basis values and weighted kernel values in LDS, and lane l owns the
// moments (c, t) = (o / 6, o % 6) for o = l, l + 64, l + 128, l + 192.
// The order is a template parameter so that the n_p basis values of a point
// stay in registers.
#include "kernels.hpp"

#include <hip/hip_runtime.h>

namespace lb {

namespace {

constexpr int NQ_STACK = 72;  // >= 3 max_depth + 1 entries
constexpr double NQ_INV4PI = 0.07957747154594767;

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
__global__ __launch_bounds__(64) void k_near_quad(NearQuadArgs q) {
  constexpr int NPP = (KO + 1) * (KO + 2) / 2;
  constexpr int NMOM = 6 * NPP;
  constexpr int NJ = (KO + 1) * (KO + 1);
  __shared__ double sc[3][NPP * 3];   // modal coefficients of X, X_u, X_v of the patch
  __shared__ double stk[NQ_STACK][6];  // subdivision stack: triangle vertices in (u, v)
  __shared__ int sdep[NQ_STACK];
  __shared__ double sK[64][NPP + 1];   // basis values of the leaf's points
  __shared__ double sKV[64][6];        // weighted kernel values of the leaf's points
  __shared__ double sv[4][3];          // chart at the vertices and the centroid
  __shared__ double sM[NMOM];
  __shared__ double sj[3][NJ];         // Jacobi recurrence tables
  const int lane = threadIdx.x;
  const int64_t w = blockIdx.x;
  if (w >= q.nwork) return;
  const int64_t i = q.row[w];
  const int64_t p = q.patch[w];
  for (int e = lane; e < 3 * NPP; e += 64) {
    sc[0][e] = q.cX[p * NPP * 3 + e];
    sc[1][e] = q.cXu[p * NPP * 3 + e];
    sc[2][e] = q.cXv[p * NPP * 3 + e];
  }
  for (int e = lane; e < NJ; e += 64) {
    sj[0][e] = q.ja[e];
    sj[1][e] = q.jb[e];
    sj[2][e] = q.jc[e];
  }
  const double x0 = q.X[3 * i], x1 = q.X[3 * i + 1], x2 = q.X[3 * i + 2];
  const double n0 = q.nrm[3 * i], n1 = q.nrm[3 * i + 1], n2 = q.nrm[3 * i + 2];
  if (lane == 0) {
    stk[0][0] = 0; stk[0][1] = 0; stk[0][2] = 1; stk[0][3] = 0; stk[0][4] = 0; stk[0][5] = 1;
    sdep[0] = 0;
  }
  __syncthreads();
  double acc[4] = {0, 0, 0, 0};
  double K[NPP];
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
      nq_basis<KO>(sj[0], sj[1], sj[2], u, v, K);
      double y0 = 0, y1 = 0, y2 = 0;
#pragma unroll
      for (int m = 0; m < NPP; ++m) {
        y0 += K[m] * sc[0][3 * m];
        y1 += K[m] * sc[0][3 * m + 1];
        y2 += K[m] * sc[0][3 * m + 2];
      }
      sv[lane][0] = y0; sv[lane][1] = y1; sv[lane][2] = y2;
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
        double kv[6] = {0, 0, 0, 0, 0, 0};
        if (pt < q.nq) {
          const double u = T[0] + q.ru[2 * pt] * e1u + q.ru[2 * pt + 1] * e2u;
          const double v = T[1] + q.ru[2 * pt] * e1v + q.ru[2 * pt + 1] * e2v;
          nq_basis<KO>(sj[0], sj[1], sj[2], u, v, K);
          double y[3] = {0, 0, 0}, yu[3] = {0, 0, 0}, yv[3] = {0, 0, 0};
#pragma unroll
          for (int m = 0; m < NPP; ++m) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              y[c] += K[m] * sc[0][3 * m + c];
              yu[c] += K[m] * sc[1][3 * m + c];
              yv[c] += K[m] * sc[2][3 * m + c];
            }
          }
          const double c0 = yu[1] * yv[2] - yu[2] * yv[1];
          const double c1 = yu[2] * yv[0] - yu[0] * yv[2];
          const double c2 = yu[0] * yv[1] - yu[1] * yv[0];
          const double J = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
          const double nu0 = c0 / J, nu1 = c1 / J, nu2 = c2 / J;
          const double d0 = x0 - y[0], d1 = x1 - y[1], d2 = x2 - y[2];
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
          const double f = area2 * q.rw[pt] * J;
#pragma unroll
          for (int t = 0; t < 6; ++t) kv[t] *= f;
        } else {
#pragma unroll
          for (int m = 0; m < NPP; ++m) K[m] = 0.0;
        }
#pragma unroll
        for (int m = 0; m < NPP; ++m) sK[lane][m] = K[m];
#pragma unroll
        for (int t = 0; t < 6; ++t) sKV[lane][t] = kv[t];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int o = lane + 64 * j;
          if (o < NMOM) {
            const int c = o / 6, t = o % 6;
            double s = 0;
            for (int l = 0; l < 64; ++l) s += sK[l][c] * sKV[l][t];
            acc[j] += s;
          }
        }
        __syncthreads();
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
  // modal moments -> Lagrange-basis values: A[blk][b][t] = sum_c Vinv[c][b] mom[c][t]
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int o = lane + 64 * j;
    if (o < NMOM) sM[o] = acc[j];
  }
  __syncthreads();
  for (int o = lane; o < NMOM; o += 64) {
    const int b = o / 6, t = o % 6;
    double s = 0;
#pragma unroll
    for (int c = 0; c < NPP; ++c) s += q.Vinv[c * NPP + b] * sM[6 * c + t];
    q.A[q.blk[w] * NMOM + o] = s;
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

}  // namespace lb
