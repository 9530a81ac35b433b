// Surface calculus of node values on the device (Section 2) and the
// elementwise steps of the Hodge decomposition (harmonic vector field
// section).
//
// With the chart derivatives X_u, X_v given at the nodes and the metric E = X_u.X_u, F = X_u.X_v, G = X_v.X_v, det = EG - F^2:
//   grad psi = ((G psi_u - F psi_v) X_u + (E psi_v - F psi_u) X_v) / det,
//   div V    = det^(-1/2) (d_u (det^(1/2) V^1) + d_v (det^(1/2) V^2)),
// V^1 = (G V.X_u - F V.X_v) / det, V^2 = (E V.X_v - F V.X_u) / det the
// contravariant components of the tangential part of V.  The chart
// derivatives of node values differentiate the order-k interpolant on each
// patch: psi_u(node b) = sum_c Du[b][c] psi(node c), and the same with Dv.
#include "kernels.hpp"

#include <hip/hip_runtime.h>

namespace lb {

namespace {

constexpr int CALC_NPMAX = 64;

__device__ inline void surf_grad_at(const double* psi, const double* Du, const double* Dv, const double* Xu,
                                    const double* Xv, int n_p, int64_t i, double* g) {
  const int64_t base = (i / n_p) * n_p;
  const int b = (int)(i - base);
  double pu = 0, pv = 0;
  for (int c = 0; c < n_p; ++c) {
    const double v = psi[base + c];
    pu += Du[b * n_p + c] * v;
    pv += Dv[b * n_p + c] * v;
  }
  const double u0 = Xu[3 * i], u1 = Xu[3 * i + 1], u2 = Xu[3 * i + 2];
  const double v0 = Xv[3 * i], v1 = Xv[3 * i + 1], v2 = Xv[3 * i + 2];
  const double E = u0 * u0 + u1 * u1 + u2 * u2, F = u0 * v0 + u1 * v1 + u2 * v2, G = v0 * v0 + v1 * v1 + v2 * v2;
  const double det = E * G - F * F;
  const double a = (G * pu - F * pv) / det, bb = (E * pv - F * pu) / det;
  g[0] = a * u0 + bb * v0;
  g[1] = a * u1 + bb * v1;
  g[2] = a * u2 + bb * v2;
}

// grad[d][i][3] of psi[d][i]; one thread per (density, node)
__global__ void k_surf_grad(SurfCalcArgs q, int nd, const double* psi, double* grad) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nd * q.N) return;
  const int64_t d = t / q.N, i = t - d * q.N;
  double g[3];
  surf_grad_at(psi + d * q.N, q.Du, q.Dv, q.Xu, q.Xv, q.n_p, i, g);
  for (int c = 0; c < 3; ++c) grad[3 * t + c] = g[c];
}

// div[d][i] = sign * div_Gamma(V or n x V) at the nodes; one block of 64
// threads per (density, patch): thread c stages det^(1/2) V^1, det^(1/2) V^2
// of node c in LDS, thread b differentiates them at node b
__global__ __launch_bounds__(64) void k_surf_div(SurfCalcArgs q, int nd, const double* V, int cross_n, double sign,
                                                 double* div) {
  __shared__ double s1[CALC_NPMAX], s2[CALC_NPMAX], sJ[CALC_NPMAX];
  const int n_p = q.n_p;
  const int64_t NP = q.N / n_p;
  const int64_t d = blockIdx.x / NP, p = blockIdx.x - d * NP;
  const int c = threadIdx.x;
  if (c < n_p) {
    const int64_t i = p * n_p + c;
    const double* v = V + 3 * (d * q.N + i);
    double w0 = v[0], w1 = v[1], w2 = v[2];
    if (cross_n) {
      const double n0 = q.nrm[3 * i], n1 = q.nrm[3 * i + 1], n2 = q.nrm[3 * i + 2];
      const double x0 = n1 * w2 - n2 * w1, x1 = n2 * w0 - n0 * w2, x2 = n0 * w1 - n1 * w0;
      w0 = x0; w1 = x1; w2 = x2;
    }
    const double u0 = q.Xu[3 * i], u1 = q.Xu[3 * i + 1], u2 = q.Xu[3 * i + 2];
    const double v0 = q.Xv[3 * i], v1 = q.Xv[3 * i + 1], v2 = q.Xv[3 * i + 2];
    const double E = u0 * u0 + u1 * u1 + u2 * u2, F = u0 * v0 + u1 * v1 + u2 * v2, G = v0 * v0 + v1 * v1 + v2 * v2;
    const double det = E * G - F * F;
    const double cu = w0 * u0 + w1 * u1 + w2 * u2, cv = w0 * v0 + w1 * v1 + w2 * v2;
    const double J = sqrt(det);
    s1[c] = J * ((G * cu - F * cv) / det);
    s2[c] = J * ((E * cv - F * cu) / det);
    sJ[c] = J;
  }
  __syncthreads();
  if (c < n_p) {
    double a = 0, b = 0;
    for (int e = 0; e < n_p; ++e) {
      a += q.Du[c * n_p + e] * s1[e];
      b += q.Dv[c * n_p + e] * s2[e];
    }
    div[d * q.N + p * n_p + c] = sign * ((a + b) / sJ[c]);
  }
}

// H[f][i] = F[f][i] - grad alpha_f - n x grad beta_f; one thread per
// (field, node)
__global__ void k_hodge_h(SurfCalcArgs q, int nf, const double* Fv, const double* alpha, const double* beta,
                          double* H) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nf * q.N) return;
  const int64_t f = t / q.N, i = t - f * q.N;
  double ga[3], gb[3];
  surf_grad_at(alpha + f * q.N, q.Du, q.Dv, q.Xu, q.Xv, q.n_p, i, ga);
  surf_grad_at(beta + f * q.N, q.Du, q.Dv, q.Xu, q.Xv, q.n_p, i, gb);
  const double n0 = q.nrm[3 * i], n1 = q.nrm[3 * i + 1], n2 = q.nrm[3 * i + 2];
  const double c0 = n1 * gb[2] - n2 * gb[1], c1 = n2 * gb[0] - n0 * gb[2], c2 = n0 * gb[1] - n1 * gb[0];
  H[3 * t] = Fv[3 * t] - ga[0] - c0;
  H[3 * t + 1] = Fv[3 * t + 1] - ga[1] - c1;
  H[3 * t + 2] = Fv[3 * t + 2] - ga[2] - c2;
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_surf_grad(const SurfCalcArgs& q, int nd, const double* psi, double* grad, hipStream_t st) {
  const int64_t n = (int64_t)nd * q.N;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_surf_grad, dim3(nblocks(n, 256)), dim3(256), 0, st, q, nd, psi, grad);
  return hipGetLastError();
}

hipError_t launch_surf_div(const SurfCalcArgs& q, int nd, const double* V, int cross_n, double sign, double* div,
                           hipStream_t st) {
  if (q.n_p > CALC_NPMAX || q.N % q.n_p) return hipErrorInvalidValue;
  const int64_t nblk = (int64_t)nd * (q.N / q.n_p);
  if (nblk <= 0) return hipSuccess;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_surf_div, dim3((unsigned)nblk), dim3(64), 0, st, q, nd, V, cross_n, sign, div);
  return hipGetLastError();
}

hipError_t launch_hodge_h(const SurfCalcArgs& q, int nf, const double* F, const double* alpha, const double* beta,
                          double* H, hipStream_t st) {
  const int64_t n = (int64_t)nf * q.N;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hodge_h, dim3(nblocks(n, 256)), dim3(256), 0, st, q, nf, F, alpha, beta, H);
  return hipGetLastError();
}

}  // namespace lb

// ---------------------------------------------------------------------------
// A1 (Section 4.1, eq. ie-dis0): A1[tau] = div S[mu] + W(S tau) S[1] with
// mu = grad_Gamma S tau; the two elementwise steps between the applies.
// ---------------------------------------------------------------------------
namespace lb {
namespace {

// mu[3 d + l][i] = surf[d][i][l]
template <typename T>
__global__ void k_a1_split(int64_t N, int nd, const T* surf, T* mu) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nd * N) return;
  const int64_t d = t / N, i = t - d * N;
#pragma unroll
  for (int l = 0; l < 3; ++l) mu[(3 * d + l) * N + i] = surf[3 * t + l];
}

// out[d][i] = sum_l g[3 d + l][i][l] + eta[d][surface of i] phi0[i]
template <typename T>
__global__ void k_a1_finish(int64_t N, int nd, int nsurf, const int* surf_of, const T* g, const double* eta,
                            const T* phi0, T* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nd * N) return;
  const int64_t d = t / N, i = t - d * N;
  double s = 0;
#pragma unroll
  for (int l = 0; l < 3; ++l) s += (double)g[((3 * d + l) * N + i) * 3 + l];
  out[t] = (T)(s + eta[d * nsurf + surf_of[i]] * (double)phi0[i]);
}

}  // namespace

template <typename T>
hipError_t launch_a1_split(int64_t N, int nd, const T* surf, T* mu, hipStream_t st) {
  const int64_t n = (int64_t)nd * N;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_a1_split<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, N, nd, surf, mu);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_a1_finish(int64_t N, int nd, int nsurf, const int* surf_of, const T* g, const double* eta,
                            const T* phi0, T* out, hipStream_t st) {
  const int64_t n = (int64_t)nd * N;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_a1_finish<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, N, nd, nsurf, surf_of, g,
                     eta, phi0, out);
  return hipGetLastError();
}

template hipError_t launch_a1_split<float>(int64_t, int, const float*, float*, hipStream_t);
template hipError_t launch_a1_split<double>(int64_t, int, const double*, double*, hipStream_t);
template hipError_t launch_a1_finish<float>(int64_t, int, int, const int*, const float*, const double*, const float*,
                                            float*, hipStream_t);
template hipError_t launch_a1_finish<double>(int64_t, int, int, const int*, const double*, const double*,
                                             const double*, double*, hipStream_t);

}  // namespace lb
