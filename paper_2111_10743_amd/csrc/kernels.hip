// HIP kernels of the layer-potential apply (gfx950, wave64).
//
//  * strengths:     tau -> c = w^over (P tau) in source tree order (Section 4,
//                   eq. nys-lcq: oversampled interpolation of the density)
//  * FMM:           P2M, M2M, M2L, L2L, L2P for the charge/dipole vector FMM of
//                   Section 4, eq. (fmm-formula), uniform-depth octree
//  * near field:    direct sums over adjacent leaves (U-list) fused with L2P
//  * corrections:   block-CSR products with the stored near corrections of
//                   eq. (nys-lcq2), fused with the combination of Section 4.1
//                   (S, grad S, S', surface gradient) and Section 4.3 (A3)
//  * FP64 BLAS-1/2 helpers for GMRES (Section 6)
// Every output element has one owning thread; no floating-point atomics, so
// results are bitwise reproducible run to run.
#include "kernels.hpp"
#include "common.hpp"

#include <type_traits>

#include <hip/hip_runtime.h>
#include <cstdio>

namespace lb {

// A failed launch (bad grid, LDS size or argument) throws, so the C entry
// point returns LB_EHIP instead of reporting success with unwritten outputs
// (hipGetLastError clears the error, so it must be acted on here).
#define KCHECK()                                                                          \
  do {                                                                                    \
    hipError_t e_ = hipGetLastError();                                                    \
    if (e_ != hipSuccess)                                                                 \
      fail(LB_EHIP, "kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), __FILE__, __LINE__); \
  } while (0)

template <typename T> __device__ __forceinline__ T dev_rsqrt(T x);
template <> __device__ __forceinline__ float dev_rsqrt<float>(float x) { return __builtin_amdgcn_rsqf(x); }
// FP64: the hardware estimate (relative error ~5e-8 on gfx950) and one
// Newton step y (3 - x y^2) / 2, relative error ~4e-15 for normal x > 0
template <> __device__ __forceinline__ double dev_rsqrt<double>(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = __fma_rn(-x * y, y, 1.0);
  return __fma_rn(0.5 * y, e, y);
}

template <typename T> __device__ __forceinline__ T dev_fma(T a, T b, T c);
template <> __device__ __forceinline__ float dev_fma<float>(float a, float b, float c) { return __fmaf_rn(a, b, c); }
template <> __device__ __forceinline__ double dev_fma<double>(double a, double b, double c) { return __fma_rn(a, b, c); }

__device__ __forceinline__ int cidx(int n, int m) { return n * (n + 1) / 2 + m; }

template <typename T> struct Vec4;
template <> struct Vec4<float> { typedef float4 type; };
template <> struct Vec4<double> { typedef double4 type; };

// real layout index -> (n, m, part) with part 0 = Re, 1 = Im
__device__ __forceinline__ void rdecode(int c, int& n, int& m, int& part) {
  n = (int)sqrtf((float)c + 0.5f);
  while (n * n > c) --n;
  while ((n + 1) * (n + 1) <= c) ++n;
  int r = c - n * n;
  m = (r + 1) >> 1;
  part = (r == 0 || (r & 1)) ? 0 : 1;
}

// ---------------------------------------------------------------------------
// strengths
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_strengths(const T* __restrict__ tau, int ne, int64_t N, int n_p, int n_o,
                            const T* __restrict__ P, const T* __restrict__ wo,
                            const int* __restrict__ src_pos, int64_t No, T* __restrict__ str) {
  extern __shared__ unsigned char smraw[];
  T* tp = reinterpret_cast<T*>(smraw);
  const int pch = blockIdx.x;
  for (int t = threadIdx.x; t < ne * n_p; t += blockDim.x) {
    int e = t / n_p, k = t - e * n_p;
    tp[t] = tau[(int64_t)e * N + (int64_t)pch * n_p + k];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < ne * n_o; t += blockDim.x) {
    int e = t / n_o, m = t - e * n_o;
    const T* Pm = P + (int64_t)m * n_p;
    const T* te = tp + e * n_p;
    T acc = 0;
    for (int k = 0; k < n_p; ++k) acc += Pm[k] * te[k];
    int64_t gm = (int64_t)pch * n_o + m;
    str[(int64_t)e * No + src_pos[gm]] = wo[gm] * acc;
  }
}

template <typename T>
void launch_strengths(const T* tau, int ne, int64_t N, int NP, int n_p, int n_o, const T* P,
                      const T* wo, const int* src_pos, int64_t No, T* str, hipStream_t st) {
  size_t sm = sizeof(T) * ne * n_p;
  hipLaunchKernelGGL(k_strengths<T>, dim3(NP), dim3(256), sm, st, tau, ne, N, n_p, n_o, P, wo,
                     src_pos, No, str);
  KCHECK();
}

// ---------------------------------------------------------------------------
// solid harmonics Rt_n^m (normalized regular) of xi into LDS rows (re, im)
// ---------------------------------------------------------------------------
// Recurrence coefficients of the normalized regular solid harmonics
// (p <= 31), kept in LDS by each block:
//   Rt_m^m = sect[m] (x + i y) Rt_{m-1}^{m-1},  Rt_{m+1}^m = up[m] z Rt_m^m,
//   Rt_{n+1}^m = a[n,m] z Rt_n^m - b[n,m] r^2 Rt_{n-1}^m   (index cidx(n, m)),
// sect[m] = -sqrt((2m-1)/(2m)), up[m] = sqrt(2m+1),
// a = (2n+1) / sqrt((n+1+m)(n+1-m)), b = sqrt((n+m)(n-m)) / sqrt((n+1+m)(n+1-m)),
// evaluated in FP64 and rounded once.
constexpr int RECTAB_N = 2 * 32 + 2 * 528;
template <typename T>
struct RecTab {
  T* sect;
  T* up;
  T* a;
  T* b;
  __device__ explicit RecTab(T* base) : sect(base), up(base + 32), a(base + 64), b(base + 64 + 528) {}
};

// block-cooperative fill (the caller synchronizes before use)
template <typename T>
__device__ void fill_rectab(const RecTab<T>& rt, int p) {
  for (int c = threadIdx.x; c < (p + 1) * (p + 2) / 2; c += blockDim.x) {
    int n = 0;
    while ((n + 1) * (n + 2) / 2 <= c) ++n;
    const int m = c - n * (n + 1) / 2;
    const double dn = 1.0 / sqrt((double)((n + 1 + m) * (n + 1 - m)));
    rt.a[c] = (T)((2 * n + 1) * dn);
    rt.b[c] = (T)(sqrt((double)((n + m) * (n - m))) * dn);
  }
  for (int m = threadIdx.x; m <= p; m += blockDim.x) {
    rt.sect[m] = m > 0 ? (T)(-sqrt((double)(2 * m - 1) / (double)(2 * m))) : (T)1;
    rt.up[m] = (T)sqrt((double)(2 * m + 1));
  }
}

// Column m of the normalized regular harmonics, Rt_n^m for n = m..p, into
// LDS rows (re, im).  Rt_m^m = prod_{j<=m} (-(x+iy) sqrt((2j-1)/(2j))).
template <typename T>
__device__ void regular_column_to_lds(const RecTab<T>& rt, int p, int m, T x, T y, T z, T* re, T* im) {
  const T r2 = x * x + y * y + z * z;
  T mre = 1, mim = 0;
  for (int j = 1; j <= m; ++j) {
    const T f = rt.sect[j];
    const T nr = f * (x * mre - y * mim);
    const T ni = f * (x * mim + y * mre);
    mre = nr;
    mim = ni;
  }
  re[cidx(m, m)] = mre;
  im[cidx(m, m)] = mim;
  if (m + 1 > p) return;
  const T c1 = z * rt.up[m];
  T are = mre, aim = mim, bre = c1 * mre, bim = c1 * mim;
  re[cidx(m + 1, m)] = bre;
  im[cidx(m + 1, m)] = bim;
  for (int n = m + 1; n < p; ++n) {
    const int c = cidx(n, m);
    const T f1 = rt.a[c] * z, f2 = rt.b[c] * r2;
    const T cre = f1 * bre - f2 * are;
    const T cim = f1 * bim - f2 * aim;
    re[cidx(n + 1, m)] = cre;
    im[cidx(n + 1, m)] = cim;
    are = bre; aim = bim;
    bre = cre; bim = cim;
  }
}

// Rt_n^m for any m in [-n, n] from an LDS row of m >= 0 values
template <typename T>
__device__ __forceinline__ void rt_get(const T* re, const T* im, int n, int m, T& a, T& b) {
  if (m < -n || m > n || n < 0) { a = 0; b = 0; return; }
  if (m >= 0) { a = re[cidx(n, m)]; b = im[cidx(n, m)]; return; }
  T s = ((-m) & 1) ? (T)-1 : (T)1;
  a = s * re[cidx(n, -m)];
  b = -s * im[cidx(n, -m)];
}

// ---------------------------------------------------------------------------
// P2M: leaf sources -> multipole (charges and, in FMM_A3B, dipoles c * nu)
// grid (leaves with sources, nrhs); M [nbox][nrhs*nexp][L]
// ---------------------------------------------------------------------------
constexpr int P2M_TSMAX = 32;
constexpr int KMAX = 4;  // L <= 1024

template <typename T>
__global__ __launch_bounds__(256) void k_p2m(DevTree<T> t, int mode, int nrhs, const T* __restrict__ str,
                                             int64_t No, T* __restrict__ M, int P2M_TS) {
  extern __shared__ unsigned char smraw[];
  __shared__ T rtab[RECTAB_N];
  const RecTab<T> rt(rtab);
  fill_rectab(rt, t.p);
  __syncthreads();
  const int p = t.p, L = t.L, Lc = (p + 1) * (p + 2) / 2;
  T* Rre = reinterpret_cast<T*>(smraw);
  T* Rim = Rre + P2M_TS * Lc;
  T* sq = Rim + P2M_TS * Lc;     // [2][TS] strengths of this rhs
  T* sn = sq + 2 * P2M_TS;       // [3][TS] normals
  const int b = t.leaf_src_list[blockIdx.x];
  const int g = t.leaf_box[b];
  const int rhs = blockIdx.y;
  const int nexp = fmm_nexp(mode), nstr = fmm_nstr(mode);
  const T h = t.leaf_h[b];
  const T ih = (T)1 / h;
  const T cx = t.bcx[g], cy = t.bcy[g], cz = t.bcz[g];
  T acc[KMAX][3];
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
#pragma unroll
    for (int e = 0; e < 3; ++e) acc[k][e] = 0;
  const int beg = t.src_beg[b], end = t.src_end[b];
  for (int t0 = beg; t0 < end; t0 += P2M_TS) {
    const int nt = min(P2M_TS, end - t0);
    // harmonic tables of the tile: one thread per (source, column m)
    for (int task = threadIdx.x; task < nt * (p + 1); task += blockDim.x) {
      const int j = task / (p + 1), m = task - j * (p + 1);
      const int s = t0 + j;
      regular_column_to_lds<T>(rt, p, m, (t.sx[s] - cx) * ih, (t.sy[s] - cy) * ih, (t.sz[s] - cz) * ih, Rre + j * Lc,
                               Rim + j * Lc);
    }
    if (threadIdx.x < nt) {
      const int j = threadIdx.x;
      const int s = t0 + j;
      if (mode == FMM_ADJ) {  // charge, and the dipole vector in place of the normal
        sq[j] = str[(int64_t)(rhs * 4) * No + s];
        sn[j] = str[(int64_t)(rhs * 4 + 1) * No + s];
        sn[P2M_TS + j] = str[(int64_t)(rhs * 4 + 2) * No + s];
        sn[2 * P2M_TS + j] = str[(int64_t)(rhs * 4 + 3) * No + s];
      } else {
        for (int q = 0; q < nstr; ++q) sq[q * P2M_TS + j] = str[(int64_t)(rhs * nstr + q) * No + s];
        sn[j] = t.snx[s];
        sn[P2M_TS + j] = t.sny[s];
        sn[2 * P2M_TS + j] = t.snz[s];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int c = threadIdx.x + k * 256;
      if (c >= L) break;
      int n, m, part;
      rdecode(c, n, m, part);
      const T sgn = part ? (T)-1 : (T)1;  // conj
      // dipole factors (nu . grad Rt_n^m), see harmonics.hpp
      const T fa = sqrt((T)((n + m) * (n - m)));
      const T fb = (T)0.5 * sqrt((T)((n - m) * (n - m - 1) > 0 ? (n - m) * (n - m - 1) : 0));
      const T fc = (T)0.5 * sqrt((T)((n + m) * (n + m - 1) > 0 ? (n + m) * (n + m - 1) : 0));
      for (int jj = 0; jj < nt; ++jj) {
        const T* re = Rre + jj * Lc;
        const T* im = Rim + jj * Lc;
        const T v = part ? im[cidx(n, m)] : re[cidx(n, m)];
        if (mode == FMM_ADJ) {
          // q Rt + d . grad Rt / h with the dipole vector d in sn
          const T nx = sn[jj], ny = sn[P2M_TS + jj], nz = sn[2 * P2M_TS + jj];
          T a0, b0, a1, b1, a2, b2;
          rt_get(re, im, n - 1, m, a0, b0);
          rt_get(re, im, n - 1, m + 1, a1, b1);
          rt_get(re, im, n - 1, m - 1, a2, b2);
          const T gre = nz * fa * a0 + fb * (nx * a1 + ny * b1) - fc * (nx * a2 - ny * b2);
          const T gim = nz * fa * b0 + fb * (nx * b1 - ny * a1) - fc * (nx * b2 + ny * a2);
          acc[k][0] += sgn * (sq[jj] * v + (part ? gim : gre) * ih);
          continue;
        }
        acc[k][0] += sq[jj] * sgn * v;
        if (mode == FMM_A3B) {
          acc[k][1] += sq[P2M_TS + jj] * sgn * v;
          // nu . grad Rt_n^m = nz fa R_{n-1}^m + (nx - i ny) fb R_{n-1}^{m+1} - (nx + i ny) fc R_{n-1}^{m-1}
          const T nx = sn[jj], ny = sn[P2M_TS + jj], nz = sn[2 * P2M_TS + jj];
          T a0, b0, a1, b1, a2, b2;
          rt_get(re, im, n - 1, m, a0, b0);
          rt_get(re, im, n - 1, m + 1, a1, b1);
          rt_get(re, im, n - 1, m - 1, a2, b2);
          T gre = nz * fa * a0 + fb * (nx * a1 + ny * b1) - fc * (nx * a2 - ny * b2);
          T gim = nz * fa * b0 + fb * (nx * b1 - ny * a1) - fc * (nx * b2 + ny * a2);
          const T gv = part ? gim : gre;
          acc[k][2] += sq[P2M_TS + jj] * sgn * gv * ih;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int c = threadIdx.x + k * 256;
    if (c >= L) break;
    for (int e = 0; e < nexp; ++e) M[((int64_t)g * nrhs * nexp + rhs * nexp + e) * L + c] = acc[k][e];
  }
}

// P2M of the first transposed-A3 step (FMM_ADJ3): per source j with normal n,
// strengths v, w: expansion 1 += v (n . grad) conj Rt / h, expansion 2 +=
// v (n . grad)^2 conj Rt / h^2 + w (n . grad) conj Rt / h.  The directional
// derivative of Rt_n^m is a combination of Rt_{n-1}^{m-1,m,m+1}; applying it
// to that table again gives the second derivative.  Tiles of ts sources:
// harmonic table R and derivative table D in LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_p2m_adj3(DevTree<T> t, int nrhs, const T* __restrict__ str, int64_t No,
                                                  T* __restrict__ M, int ts) {
  extern __shared__ unsigned char smraw[];
  __shared__ T rtab[RECTAB_N];
  const RecTab<T> rt(rtab);
  fill_rectab(rt, t.p);
  __syncthreads();
  const int p = t.p, L = t.L, Lc = (p + 1) * (p + 2) / 2;
  T* Rre = reinterpret_cast<T*>(smraw);
  T* Rim = Rre + ts * Lc;
  T* Dre = Rim + ts * Lc;
  T* Dim = Dre + ts * Lc;
  T* sq = Dim + ts * Lc;  // [2][ts] v, w
  T* sn = sq + 2 * ts;    // [3][ts] normals
  const int b = t.leaf_src_list[blockIdx.x];
  const int g = t.leaf_box[b];
  const int rhs = blockIdx.y;
  const T h = t.leaf_h[b];
  const T ih = (T)1 / h;
  const T cx = t.bcx[g], cy = t.bcy[g], cz = t.bcz[g];
  T acc[KMAX][2];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) acc[k][0] = acc[k][1] = 0;
  const int beg = t.src_beg[b], end = t.src_end[b];
  for (int t0 = beg; t0 < end; t0 += ts) {
    const int nt = min(ts, end - t0);
    for (int task = threadIdx.x; task < nt * (p + 1); task += blockDim.x) {
      const int j = task / (p + 1), m = task - j * (p + 1);
      const int s = t0 + j;
      regular_column_to_lds<T>(rt, p, m, (t.sx[s] - cx) * ih, (t.sy[s] - cy) * ih, (t.sz[s] - cz) * ih, Rre + j * Lc,
                               Rim + j * Lc);
    }
    if (threadIdx.x < nt) {
      const int s = t0 + threadIdx.x;
      sq[threadIdx.x] = str[(int64_t)(rhs * 2) * No + s];
      sq[ts + threadIdx.x] = str[(int64_t)(rhs * 2 + 1) * No + s];
      sn[threadIdx.x] = t.snx[s];
      sn[ts + threadIdx.x] = t.sny[s];
      sn[2 * ts + threadIdx.x] = t.snz[s];
    }
    __syncthreads();
    // D_n^m = (n . grad) Rt_n^m, m >= 0
    for (int task = threadIdx.x; task < nt * Lc; task += blockDim.x) {
      const int j = task / Lc, ci = task - j * Lc;
      int n = (int)((sqrt(8.0 * ci + 1.0) - 1.0) * 0.5);
      while (n * (n + 1) / 2 > ci) --n;
      while ((n + 1) * (n + 2) / 2 <= ci) ++n;
      const int m = ci - n * (n + 1) / 2;
      const T fa = sqrt((T)((n + m) * (n - m)));
      const T fb = (T)0.5 * sqrt((T)((n - m) * (n - m - 1) > 0 ? (n - m) * (n - m - 1) : 0));
      const T fc = (T)0.5 * sqrt((T)((n + m) * (n + m - 1) > 0 ? (n + m) * (n + m - 1) : 0));
      const T nx = sn[j], ny = sn[ts + j], nz = sn[2 * ts + j];
      T a0, b0, a1, b1, a2, b2;
      rt_get(Rre + j * Lc, Rim + j * Lc, n - 1, m, a0, b0);
      rt_get(Rre + j * Lc, Rim + j * Lc, n - 1, m + 1, a1, b1);
      rt_get(Rre + j * Lc, Rim + j * Lc, n - 1, m - 1, a2, b2);
      Dre[j * Lc + ci] = nz * fa * a0 + fb * (nx * a1 + ny * b1) - fc * (nx * a2 - ny * b2);
      Dim[j * Lc + ci] = nz * fa * b0 + fb * (nx * b1 - ny * a1) - fc * (nx * b2 + ny * a2);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const int c = threadIdx.x + k * 256;
      if (c >= L) break;
      int n, m, part;
      rdecode(c, n, m, part);
      const T sgn = part ? (T)-1 : (T)1;  // conj
      const T fa = sqrt((T)((n + m) * (n - m)));
      const T fb = (T)0.5 * sqrt((T)((n - m) * (n - m - 1) > 0 ? (n - m) * (n - m - 1) : 0));
      const T fc = (T)0.5 * sqrt((T)((n + m) * (n + m - 1) > 0 ? (n + m) * (n + m - 1) : 0));
      for (int jj = 0; jj < nt; ++jj) {
        const T* dre = Dre + jj * Lc;
        const T* dim = Dim + jj * Lc;
        const T d1 = part ? dim[cidx(n, m)] : dre[cidx(n, m)];
        const T nx = sn[jj], ny = sn[ts + jj], nz = sn[2 * ts + jj];
        T a0, b0, a1, b1, a2, b2;
        rt_get(dre, dim, n - 1, m, a0, b0);
        rt_get(dre, dim, n - 1, m + 1, a1, b1);
        rt_get(dre, dim, n - 1, m - 1, a2, b2);
        const T gre = nz * fa * a0 + fb * (nx * a1 + ny * b1) - fc * (nx * a2 - ny * b2);
        const T gim = nz * fa * b0 + fb * (nx * b1 - ny * a1) - fc * (nx * b2 + ny * a2);
        const T d2 = part ? gim : gre;
        const T v = sq[jj], w = sq[ts + jj];
        acc[k][0] += sgn * v * d1 * ih;
        acc[k][1] += sgn * (v * d2 * ih * ih + w * d1 * ih);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int c = threadIdx.x + k * 256;
    if (c >= L) break;
    for (int e = 0; e < 2; ++e) M[((int64_t)g * nrhs * 2 + rhs * 2 + e) * L + c] = acc[k][e];
  }
}

// P2M tables of the sources of each leaf about the leaf centre (setup):
//   H[j][c] = conj(Rt_c(xi_j)),  Dp[j][c] = conj(nu_j . grad Rt_c(xi_j)) / h,
// xi_j = (y_j - centre) / h, real coefficient layout c < L.  A leaf multipole
// is then sum_j q_j H[j] (+ sum_j q2_j Dp[j] for the dipoles q2_j nu_j).
// grid: leaves with sources; tiles of ts sources through LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_p2m_build(DevTree<T> t, T* __restrict__ H, T* __restrict__ Dp, int ts) {
  extern __shared__ unsigned char smraw[];
  __shared__ T rtab[RECTAB_N];
  const RecTab<T> rt(rtab);
  fill_rectab(rt, t.p);
  __syncthreads();
  const int p = t.p, L = t.L, Lc = (p + 1) * (p + 2) / 2;
  T* Rre = reinterpret_cast<T*>(smraw);
  T* Rim = Rre + ts * Lc;
  T* sn = Rim + ts * Lc;  // [3][ts]
  const int b = t.leaf_src_list[blockIdx.x];
  const int g = t.leaf_box[b];
  const T h = t.leaf_h[b];
  const T ih = (T)1 / h;
  const T cx = t.bcx[g], cy = t.bcy[g], cz = t.bcz[g];
  const int beg = t.src_beg[b], end = t.src_end[b];
  for (int t0 = beg; t0 < end; t0 += ts) {
    const int nt = min(ts, end - t0);
    for (int task = threadIdx.x; task < nt * (p + 1); task += blockDim.x) {
      const int j = task / (p + 1), m = task - j * (p + 1);
      const int s = t0 + j;
      regular_column_to_lds<T>(rt, p, m, (t.sx[s] - cx) * ih, (t.sy[s] - cy) * ih, (t.sz[s] - cz) * ih, Rre + j * Lc,
                               Rim + j * Lc);
    }
    if (threadIdx.x < nt) {
      const int s = t0 + threadIdx.x;
      sn[threadIdx.x] = t.snx[s];
      sn[ts + threadIdx.x] = t.sny[s];
      sn[2 * ts + threadIdx.x] = t.snz[s];
    }
    __syncthreads();
    for (int task = threadIdx.x; task < nt * L; task += blockDim.x) {
      const int jj = task / L, c = task - jj * L;
      int n, m, part;
      rdecode(c, n, m, part);
      const T sgn = part ? (T)-1 : (T)1;  // conj
      const T* re = Rre + jj * Lc;
      const T* im = Rim + jj * Lc;
      const T v = part ? im[cidx(n, m)] : re[cidx(n, m)];
      // nu . grad Rt_n^m = nz fa R_{n-1}^m + (nx - i ny) fb R_{n-1}^{m+1} - (nx + i ny) fc R_{n-1}^{m-1}
      const T fa = sqrt((T)((n + m) * (n - m)));
      const T fb = (T)0.5 * sqrt((T)((n - m) * (n - m - 1) > 0 ? (n - m) * (n - m - 1) : 0));
      const T fc = (T)0.5 * sqrt((T)((n + m) * (n + m - 1) > 0 ? (n + m) * (n + m - 1) : 0));
      const T nx = sn[jj], ny = sn[ts + jj], nz = sn[2 * ts + jj];
      T a0, b0, a1, b1, a2, b2;
      rt_get(re, im, n - 1, m, a0, b0);
      rt_get(re, im, n - 1, m + 1, a1, b1);
      rt_get(re, im, n - 1, m - 1, a2, b2);
      const T gre = nz * fa * a0 + fb * (nx * a1 + ny * b1) - fc * (nx * a2 - ny * b2);
      const T gim = nz * fa * b0 + fb * (nx * b1 - ny * a1) - fc * (nx * b2 + ny * a2);
      const int64_t o = (int64_t)(t0 + jj) * L + c;
      H[o] = sgn * v;
      Dp[o] = sgn * (part ? gim : gre) * ih;
    }
    __syncthreads();
  }
}

template <typename T>
void launch_p2m_tables(const DevTree<T>& t, T* H, T* Dp, hipStream_t st) {
  if (t.depth < 2 || t.n_leaf_src == 0) return;
  const int Lc = (t.p + 1) * (t.p + 2) / 2;
  int ts = (int)((48 * 1024 / sizeof(T) - RECTAB_N) / (2 * Lc + 3));
  ts = ts < 1 ? 1 : (ts > 64 ? 64 : ts);
  const size_t sm = sizeof(T) * (size_t)ts * (2 * Lc + 3);
  hipLaunchKernelGGL(k_p2m_build<T>, dim3(t.n_leaf_src), dim3(256), sm, st, t, H, Dp, ts);
  KCHECK();
}

// P2M from the tables: M[g][rhs*nexp + e] = sum_j q_e[j] H[j] (+ Dp for the
// dipoles).  Each of the P2M_W waves of a block sums every P2M_W-th source
// of the leaf over 256 coefficients (4 per lane); the wave partials meet in
// LDS.  grid (leaves with sources, nrhs), block 64 * P2M_W
constexpr int P2M_W = 8;

template <typename T, bool A3B>
__global__ __launch_bounds__(64 * P2M_W) void k_p2m_tab(DevTree<T> t, int nrhs, const T* __restrict__ str,
                                                        int64_t No, const T* __restrict__ H,
                                                        const T* __restrict__ Dp, T* __restrict__ M) {
  constexpr int NE = A3B ? 3 : 1;
  __shared__ T red[NE][P2M_W][256];
  const int b = t.leaf_src_list[blockIdx.x];
  const int g = t.leaf_box[b];
  const int rhs = blockIdx.y;
  const int L = t.L;
  const int nstr = A3B ? 2 : 1;
  const int beg = t.src_beg[b], end = t.src_end[b];
  const T* q1 = str + (int64_t)(rhs * nstr) * No;
  const T* q2 = A3B ? str + (int64_t)(rhs * nstr + 1) * No : q1;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  T* out = M + ((int64_t)g * nrhs * NE + rhs * NE) * L;
  for (int c0 = 0; c0 < L; c0 += 256) {
    T a[NE][4];
#pragma unroll
    for (int e = 0; e < NE; ++e)
#pragma unroll
      for (int k = 0; k < 4; ++k) a[e][k] = 0;
    // coefficient of slot k of this lane, clamped into the row: lanes past
    // L sum a copy of coefficient L-1 and are never stored (no predicated
    // loads in the loop)
    int cc[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) cc[k] = min(c0 + lane + 64 * k, L - 1);
#pragma unroll(A3B && sizeof(T) == 8 ? 2 : 4)
    for (int j = beg + w; j < end; j += P2M_W) {
      const T s1 = q1[j];
      const T s2 = q2[j];
      const T* hr = H + (int64_t)j * L;
      const T* dr = Dp + (int64_t)j * L;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const T hv = hr[cc[k]];
        a[0][k] += s1 * hv;
        if (A3B) {
          a[1][k] += s2 * hv;
          a[2][k] += s2 * dr[cc[k]];
        }
      }
    }
#pragma unroll
    for (int e = 0; e < NE; ++e)
#pragma unroll
      for (int k = 0; k < 4; ++k) red[e][w][lane + 64 * k] = a[e][k];
    __syncthreads();
    const int c = c0 + threadIdx.x;
    if (threadIdx.x < 256 && c < L) {
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        T sum = 0;
#pragma unroll
        for (int v = 0; v < P2M_W; ++v) sum += red[e][v][threadIdx.x];
        out[e * L + c] = sum;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// M2L as batched GEMMs on the matrix cores.  All V-list pairs of all levels
// are grouped by offset (the translation matrix depends only on the offset
// in units of the box size): Y[:, c] = T_o M[src(c)] for every column c of
// the group (one column per (pair, expansion)), then a per-box reduction sums
// the columns of each target box and applies the level scale 1/h.
// v_mfma_*_16x16x4: lane l holds A[l%16][l/16] and B[l/16][l%16]; the
// result register v of lane l is D[4*(l/16)+v][l%16] for f32 and
// D[l/16+4v][l%16] for f64 (checked on gfx950).
// ---------------------------------------------------------------------------
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));
template <typename T> struct Mfma;
template <> struct Mfma<float> {
  typedef mf4 acc;
  static __device__ __forceinline__ acc op(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <> struct Mfma<double> {
  typedef md4 acc;
  static __device__ __forceinline__ acc op(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

constexpr int GM_COLS = 64;   // columns per block (4 waves x 16)
constexpr int GM_RB = 8;      // 16-row blocks per block (128 rows)
static_assert(GM_COLS == GEMM_TILE_COLS && GM_RB * 16 == GEMM_TILE_ROWS, "tile shape shared with the plans");
template <typename T> struct GmKc { static constexpr int v = 32; };   // k chunk staged in LDS
template <> struct GmKc<double> { static constexpr int v = 16; };

// work item w: (group, first column, first row, first k); group: offset id
// and column range.
// The tiles of k chunk i+1 are loaded into registers while the matrix cores
// work on chunk i from LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_gemm_grouped(const T* __restrict__ TT, int L, const int* __restrict__ work,
                                                      const int* __restrict__ grp_off, const int* __restrict__ grp_beg,
                                                      const int* __restrict__ pair_src, const int* __restrict__ grp_lo,
                                                      int kslice, int64_t ystride, int ne, const T* __restrict__ M,
                                                      T* __restrict__ Y) {
  constexpr int KC = GmKc<T>::v;
  constexpr int NA = KC * GM_RB * 16 / 256;  // A values per thread per chunk
  constexpr int NB = KC * GM_COLS / 256;     // B values per thread per chunk
  // FP64: two LDS buffers and one barrier per k chunk (measured: FP64 M2L
  // 2.85 -> 2.51 ms at 143k nodes); FP32 keeps one buffer (its three
  // blocks per CU: the second buffer costs it 0.200 -> 0.205 ms)
  constexpr int NBUF = sizeof(T) == 8 ? 2 : 1;
  __shared__ T As[NBUF][KC][GM_RB * 16];
  __shared__ T Bs[NBUF][GM_COLS][KC + 1];  // column-major, padded against bank conflicts
  __shared__ int srcrow[GM_COLS];
  // XCD-aware order: block b runs on XCD b % 8; each XCD takes a contiguous
  // range of the work list, so the column tiles that share a slab of a
  // translation matrix (and the row tiles that share the columns) run on
  // the same XCD and meet in its L2
  const int total = gridDim.x, bq = total / GEMM_NXCD, br = total - bq * GEMM_NXCD;
  const int xcd = blockIdx.x % GEMM_NXCD, loc = blockIdx.x / GEMM_NXCD;
  const int w = xcd < br ? xcd * (bq + 1) + loc : br * (bq + 1) + (xcd - br) * bq + loc;
  const int grp = work[4 * w];
  const int c0 = work[4 * w + 1];
  const int r0 = work[4 * w + 2];
  const int kb = work[4 * w + 3];
  const int cend = grp_beg[grp + 1] * ne;
  const int Lo = grp_lo ? grp_lo[grp] : L;  // coefficients in and out of this group's translation
  const int ke = kslice ? min(Lo, kb + kslice) : Lo;  // this block's part of the sum over k
  if (kslice) Y += (int64_t)(kb / kslice) * ystride;
  const T* Tm = TT + (int64_t)grp_off[grp] * L * L;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x < GM_COLS) {
    const int c = c0 + threadIdx.x;
    srcrow[threadIdx.x] = c < cend ? pair_src[c / ne] * ne + (c % ne) : -1;
  }
  __syncthreads();
  // this thread's tile elements, i = threadIdx.x + 256 u: A (kk, r) =
  // (i / 128, i % 128), B (c, kk) = (i / KC, i % KC).  Loads are unguarded
  // (indices clamped into the matrix and the source rows) and zeroed by a
  // select where k >= L or the column is empty.
  static_assert(256 % (GM_RB * 16) == 0 && 256 % KC == 0, "tile shape");
  const int ar = min(r0 + (int)(threadIdx.x % (GM_RB * 16)), L - 1);
  const int akk = threadIdx.x / (GM_RB * 16);
  const int bkk = threadIdx.x % KC;
  const T* bp[NB];
  T bv[NB];  // 1 for a column in use, else 0 (a factor, so that no load is predicated)
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int sr = srcrow[(threadIdx.x + 256 * u) / KC];
    bv[u] = sr >= 0 ? (T)1 : (T)0;
    bp[u] = M + (int64_t)(sr >= 0 ? sr : 0) * L;
  }
  T ra[NA], rb_[NB];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int k = k0 + akk + u * (256 / (GM_RB * 16));
      const T v = Tm[(int64_t)min(k, L - 1) * L + ar];
      ra[u] = k < ke ? v : (T)0;
    }
    const int k = k0 + bkk;
    const int kc = min(k, L - 1);
    const T kv = k < ke ? (T)1 : (T)0;
#pragma unroll
    for (int u = 0; u < NB; ++u) rb_[u] = bp[u][kc] * (bv[u] * kv);
  };
  typename Mfma<T>::acc acc[GM_RB];
#pragma unroll
  for (int rb = 0; rb < GM_RB; ++rb) acc[rb] = (typename Mfma<T>::acc){0, 0, 0, 0};
  auto store = [&](int bf) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int i = threadIdx.x + 256 * u;
      As[bf][i / (GM_RB * 16)][i % (GM_RB * 16)] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int i = threadIdx.x + 256 * u;
      Bs[bf][i / KC][i % KC] = rb_[u];
    }
  };
  auto compute = [&](int bf) {
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const T b = Bs[bf][wv * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int rb = 0; rb < GM_RB; ++rb) {
        const T a = As[bf][kk + (lane >> 4)][rb * 16 + (lane & 15)];
        acc[rb] = Mfma<T>::op(a, b, acc[rb]);
      }
    }
  };
  load(kb);
  if constexpr (NBUF == 2) {
    // chunk i+1 goes into registers while the matrix cores work on chunk i
    // from one buffer, then into the other buffer (read last in chunk i-1,
    // which every wave finished before the previous barrier)
    store(0);
    __syncthreads();
    int bf = 0;
    for (int k0 = kb; k0 < ke; k0 += KC) {
      const bool more = k0 + KC < ke;
      if (more) load(k0 + KC);
      compute(bf);
      if (more) store(bf ^ 1);
      __syncthreads();
      bf ^= 1;
    }
  } else {
    for (int k0 = kb; k0 < ke; k0 += KC) {
      __syncthreads();
      store(0);
      __syncthreads();
      if (k0 + KC < ke) load(k0 + KC);
      compute(0);
    }
  }
  const int c = c0 + wv * 16 + (lane & 15);
  if (c < cend) {
#pragma unroll
    for (int rb = 0; rb < GM_RB; ++rb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + rb * 16 + Mfma<T>::row(lane, v);
        if (r < Lo) Y[(int64_t)c * L + r] = acc[rb][v];
      }
  }
}

// out[g][e][r] (+)= f_g * sum over the triples p of box g of Y[p*ne + e][r],
// f_g = box_scale (2^level / side of the box's tree) when given, else 1
template <typename T>
__global__ __launch_bounds__(256) void k_col_reduce(const int* __restrict__ boxes, const double* __restrict__ box_scale,
                                                    const int* __restrict__ tptr, const int* __restrict__ tpairs,
                                                    const int* __restrict__ pair_lo, int nslice, int64_t ystride,
                                                    int ne, int L, int accumulate, const T* __restrict__ Y,
                                                    T* __restrict__ out) {
  // the box's triples and their orders are staged in LDS, so that the
  // column reads of several triples are in flight at once (a chain of
  // dependent index loads per triple would leave the kernel latency bound);
  // the sum keeps the triple order, so results do not depend on the staging
  constexpr int QC = 256;
  __shared__ int sp[QC];
  __shared__ int slo[QC];
  const int g = boxes[blockIdx.x];
  const T f = box_scale ? (T)box_scale[blockIdx.x] : (T)1;
  const int pb = tptr[blockIdx.x], pe = tptr[blockIdx.x + 1];
  for (int i0 = 0; i0 < ne * L; i0 += blockDim.x) {
    const int i = i0 + threadIdx.x;
    const bool act = i < ne * L;
    const int e = act ? i / L : 0, r = act ? i - e * L : 0;
    T a = 0;
    for (int q0 = pb; q0 < pe; q0 += QC) {
      const int nq = min(QC, pe - q0);
      __syncthreads();
      for (int j = threadIdx.x; j < nq; j += blockDim.x) {
        const int pq = tpairs[q0 + j];
        sp[j] = pq;
        slo[j] = pair_lo ? pair_lo[pq] : L;
      }
      __syncthreads();
      if (!act) continue;
      const T* Ye = Y + (int64_t)e * L + r;
      const int64_t cs = (int64_t)ne * L;  // column stride of a triple
      if (nslice == 1) {
        int q = 0;
        for (; q + 8 <= nq; q += 8) {
          T v[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            const T y = Ye[sp[q + j] * cs];  // rows past a triple's order hold no value: read, then dropped
            v[j] = r < slo[q + j] ? y : (T)0;
          }
#pragma unroll
          for (int j = 0; j < 8; ++j) a += v[j];
        }
        for (; q < nq; ++q)
          if (r < slo[q]) a += Ye[sp[q] * cs];
      } else {
        for (int q = 0; q < nq; ++q)
          if (r < slo[q])
            for (int sl = 0; sl < nslice; ++sl) a += Ye[sl * ystride + sp[q] * cs];
      }
    }
    if (act) {
      const int64_t o = ((int64_t)g * ne + e) * L + r;
      out[o] = accumulate ? out[o] + a * f : a * f;
    }
  }
}

template <typename T>
static void run_plan(const GemmPlan& pl, const T* TT, int L, int ne, const T* X, T* Y, T* out, hipStream_t st) {
  if (pl.nbox == 0) return;
  if (pl.npair > 0 && !pl.work[ne]) fail(LB_EINVAL, "translation plan has no work list for %d expansions", ne);
  const int64_t ystride = (int64_t)pl.npair * ne * L;  // one k slice of Y
  if (pl.nwork[ne] > 0) {
    dim3 grid(pl.nwork[ne]);
    hipLaunchKernelGGL(k_gemm_grouped<T>, grid, dim3(256), 0, st, TT, L, pl.work[ne], pl.grp_mat, pl.grp_beg,
                       pl.pair_src, pl.grp_lo, pl.kslice, ystride, ne, X, Y);
    KCHECK();
  }
  hipLaunchKernelGGL(k_col_reduce<T>, dim3(pl.nbox), dim3(256), 0, st, pl.boxes, pl.scaled ? pl.box_scale : nullptr,
                     pl.tptr, pl.tpairs, pl.pair_lo, pl.nslice, ystride, ne, L, pl.accumulate ? 1 : 0, (const T*)Y,
                     out);
  KCHECK();
}

// ---------------------------------------------------------------------------
// leaf evaluation: L2P (far) + direct sums over the U-list (near)
// grid (leaves with targets, nrhs); out [nrhs*nout][N] in target tree order
// ---------------------------------------------------------------------------
// Coefficient (n, m), any m in [-n, n], of a real-layout conjugate-symmetric
// expansion (see harmonics.hpp).
template <typename T>
__device__ __forceinline__ void coef_get(const T* v, int n, int m, T& re, T& im) {
  if (n < 0 || m < -n || m > n) { re = 0; im = 0; return; }
  const int am = m < 0 ? -m : m;
  re = am == 0 ? v[n * n] : v[n * n + 2 * am - 1];
  im = am == 0 ? (T)0 : v[n * n + 2 * am];
  if (m < 0) {
    const T sg = (am & 1) ? (T)-1 : (T)1;
    re = sg * re;
    im = -sg * im;
  }
}

// d/dx, d/dy, d/dz of a local expansion of order pin (unit box), written as
// expansions of order pin-1; the block's threads share the outputs.
//   d/dz: Lz_n^m = L_{n+1}^m sqrt((n+1+m)(n+1-m))
//   (d/dx + i d/dy): E_n^m = L_{n+1}^{m-1} sqrt((n-m+2)(n-m+1))
//   (d/dx - i d/dy): F_n^m = -L_{n+1}^{m+1} sqrt((n+m+2)(n+m+1))
template <typename T>
__device__ void derive3(const T* src, int pin, T* dx, T* dy, T* dz) {
  const int Lo = pin * pin;
  for (int c = threadIdx.x; c < Lo; c += blockDim.x) {
    int n, m, part;
    rdecode(c, n, m, part);
    T ar, ai, br, bi, cr, ci;
    coef_get(src, n + 1, m, ar, ai);
    coef_get(src, n + 1, m - 1, br, bi);
    coef_get(src, n + 1, m + 1, cr, ci);
    const T fz = sqrt((T)((n + 1 + m) * (n + 1 - m)));
    const T fe = sqrt((T)((n - m + 2) * (n - m + 1)));
    const T ff = -sqrt((T)((n + m + 2) * (n + m + 1)));
    const T er = fe * br, ei = fe * bi, gr = ff * cr, gi = ff * ci;
    // Gx = (E + F)/2, Gy = -i (E - F)/2
    const T xr = (T)0.5 * (er + gr), xi = (T)0.5 * (ei + gi);
    const T yr = (T)0.5 * (ei - gi), yi = -(T)0.5 * (er - gr);
    dx[c] = part ? xi : xr;
    dy[c] = part ? yi : yr;
    dz[c] = part ? fz * ai : fz * ar;
  }
}

// leaf kernel shape (compile-time; -D overrides for tuning sweeps)
#ifndef LB_LEAF_BS
#define LB_LEAF_BS 256
#endif
#ifndef LB_LEAF_CH
#define LB_LEAF_CH 512
#endif
#ifndef LB_LEAF_UNROLL
#define LB_LEAF_UNROLL (sizeof(T) == 4 ? 8 : 4)
#endif
constexpr int LEAF_BS = LB_LEAF_BS;            // threads per block
constexpr int LEAF_CH = LB_LEAF_CH;            // sources per LDS chunk
// the far-field values of a pass (4 per target slot) pass through the
// source chunk area, the smallest of which holds 5 values per source
static_assert(5 * LEAF_CH >= 4 * LEAF_BS, "source chunk area too small for the far-field values");

// Each target of a leaf gets F = min(leaf_fmax, 256 / targets) threads (a
// power of two, at most one wave; leaf_fmax is set by the autotuner) for
// the near field: thread (slot, f) sums the source indices j = f (mod F) of
// each LDS chunk for target slot `slot` of the current pass, and the F
// partial sums of a target (contiguous lanes) are then added by shuffles.
// The far field (L2P) takes one thread per target instead: split over F
// lanes of one wave by harmonic order, its terms would run one after the
// other with 1/F of the lanes active.
// LDS bytes of the L2P expansions of one block, rounded up to 16: the local
// expansions (nexp L), the gradient expansions the mode evaluates (3 p^2
// per expansion: all three in A3B, the first in GRAD and ADJ3), in A3B
// the Hessian expansions (6 (p-1)^2 and 3 (p-1)^2 scratch), and in GRAD the
// four expansions interleaved per coefficient (4 L, aligned to 16 bytes).
template <typename T>
__host__ __device__ inline size_t leaf_exp_bytes(int mode, int p) {
  const size_t L = (size_t)(p + 1) * (p + 1), Lg = (size_t)p * p, Lh = (size_t)(p - 1) * (p - 1);
  const size_t nexp = fmm_nexp(mode);
  size_t n = nexp * L;
  if (mode == FMM_GRAD || mode == FMM_ADJ3) n += 3 * Lg;
  if (mode == FMM_GRAD) n += 4 * L + 8;
  if (mode == FMM_A3B) n += nexp * 3 * Lg + 9 * Lh;
  return (sizeof(T) * n + 15) / 16 * 16;
}

// LDS bytes of the interleaved coefficients of the A3B far-only part (16
// values per real coefficient, aligned to 16 bytes), beyond leaf_exp_bytes.
template <typename T>
__host__ __device__ inline size_t leaf_z16_bytes(int p) {
  return sizeof(T) * ((size_t)16 * (p + 1) * (p + 1) + 8);
}

// Values of one (work item, density) slice of the leaf workspace D when the
// expansions do not fit in LDS: the gradient expansions (nexp 3 p^2), the
// Hessian and its scratch (9 (p-1)^2), and in GRAD the interleaved
// coefficients (4 L, at a multiple of 4 values so that they stay aligned).
__host__ __device__ inline int64_t leaf_d_vals(int mode, int p) {
  const int64_t L = (int64_t)(p + 1) * (p + 1), Lg = (int64_t)p * p, Lh = (int64_t)(p - 1) * (p - 1);
  const int64_t base = (int64_t)fmm_nexp(mode) * 3 * Lg + 9 * Lh;
  return mode == FMM_GRAD ? (base + 3) / 4 * 4 + 4 * L : base;
}

// PART: LEAF_BOTH (far and near, outputs written), LEAF_NEAR (near-field
// sums only, outputs written), LEAF_FAR (L2P only, added to the outputs);
// in A3B, when its expansions do not fit in LDS, the far part in two
// passes whose expansions do: LEAF_FAR1 (outputs 0-2: the gradient of
// expansion 0, expansion 1 and its gradient) and LEAF_FAR2 (output 3: the
// Hessian of expansion 1 and the gradient of expansion 2).
enum { LEAF_BOTH = 0, LEAF_NEAR = 1, LEAF_FAR = 2, LEAF_FAR1 = 3, LEAF_FAR2 = 4 };
template <typename T>
__host__ __device__ inline size_t leaf_far_split_bytes(int part, int p) {
  const size_t L = (size_t)(p + 1) * (p + 1), Lg = (size_t)p * p, Lh = (size_t)(p - 1) * (p - 1);
  return sizeof(T) * (part == LEAF_FAR1 ? L + 6 * Lg : 6 * Lh + 3 * Lg);
}

// Waves per SIMD the compiler must leave room for (caps the registers):
// 6 where that fits without spilling (measured: the FP32 gradient leaf
// kernel 0.498 -> 0.463 ms against 92 registers at 5 waves), else no cap.
template <typename T, int MODE>
constexpr int leaf_waves() {
  return sizeof(T) == 4 ? (MODE == FMM_ADJ ? 1 : 6) : (MODE == FMM_A3B || MODE == FMM_ADJ3 ? 1 : 6);
}

// one work item (leaf, target range, lanes per target) of the leaf kernel
template <typename T, int MODE, bool EXP_LDS, int PART>
__device__ __forceinline__ void leaf_item(const DevTree<T>& t, int nrhs, const T* __restrict__ str, int64_t No,
                                          const T* __restrict__ Lc, T* __restrict__ D, T* __restrict__ out, int64_t N,
                                          int widx) {
  extern __shared__ unsigned char smraw[];
  const int4 wk = t.leaf_work[widx];
  const int b = wk.x;
  const int g = t.leaf_box[b];
  const int rhs = blockIdx.y;
  const int p = t.p, L = t.L, Lg = p * p, Lh = (p - 1) * (p - 1);
  const int nexp = fmm_nexp(MODE), nstr = fmm_nstr(MODE), nout = fmm_nout(MODE);
  constexpr bool FARONLY = PART == LEAF_FAR || PART == LEAF_FAR1 || PART == LEAF_FAR2;
  const bool far = PART != LEAF_NEAR && t.leaf_lvl[b] >= 2;
  const int tbeg = wk.y, tend = wk.z;
  const int F = wk.w;                            // lanes per target: a power of two <= 64
  const int TPB = LEAF_BS / F;                   // target slots
  const int slot = threadIdx.x / F, f = threadIdx.x - (threadIdx.x / F) * F;
  // expansions for L2P: local [nexp][L], derived gradient [nexp][3][Lg] and
  // hessian [6][Lh] (+ 3 [Lh] scratch; A3B: expansion 1), in LDS after the
  // source chunk when EXP_LDS, else in this block's slice of D
  constexpr int REC = MODE == FMM_A3B || MODE == FMM_ADJ || MODE == FMM_ADJ3 ? 9 : 5;  // T values per source record
  T* tile = reinterpret_cast<T*>(smraw);  // (x, y, z, q1) [, (nx, ny, nz, q2)], rm2
  const T* gL = Lc + ((int64_t)g * nrhs * nexp + rhs * nexp) * L;
  const int64_t dstride = leaf_d_vals(MODE, p);
  T* sL;
  T* sG;
  if (EXP_LDS) {
    sL = tile + (FARONLY ? 0 : REC * LEAF_CH);  // the far-only kernels stage no sources
    sG = sL + nexp * L;
  } else {
    sL = const_cast<T*>(gL);
    sG = D + ((int64_t)widx * nrhs + rhs) * dstride;
  }
  T* sH = sG + nexp * 3 * Lg;
  typedef typename Vec4<T>::type T4;
  // GRAD: the interleaved coefficients after the gradient expansions, in
  // LDS at the next multiple of sizeof(T4), else at the end of the D slice
  // (slices start at multiples of 4 values)
  T4* sZ = EXP_LDS ? reinterpret_cast<T4*>(smraw) +
                         ((size_t)(sG + 3 * Lg - tile) * sizeof(T) + sizeof(T4) - 1) / sizeof(T4)
                   : reinterpret_cast<T4*>(sG + (nexp * 3 * Lg + 9 * Lh + 3) / 4 * 4);
  // A3B far-only part with the expansions in LDS: the 16 values of each
  // coefficient (expansion 1, the gradients of expansions 0, 1, 2 and the
  // Hessian of expansion 1) side by side after the Hessian scratch
  constexpr bool Z16 = MODE == FMM_A3B && PART == LEAF_FAR && EXP_LDS;
  T4* sZ16 = reinterpret_cast<T4*>(smraw) + ((size_t)(sH + 9 * Lh - tile) * sizeof(T) + sizeof(T4) - 1) / sizeof(T4);
  // A3B: the expansion values the L2P sums read (expansion 1, gradients of
  // 0, 1, 2, Hessian of 1); the split passes keep theirs in LDS
  const T* xP = sL + L;
  const T* xG1 = sG;
  const T* xG2 = sG + 3 * Lg;
  const T* xG3 = sG + 6 * Lg;
  const T* xH = sH;
  if (PART == LEAF_FAR1) {
    xP = tile;
    xG1 = tile + L;
    xG2 = tile + L + 3 * Lg;
  } else if (PART == LEAF_FAR2) {
    xH = tile;
    xG3 = tile + 6 * Lh;
  }
  // recurrence coefficients of the solid harmonics for L2P
  __shared__ T rtab[RECTAB_N];
  const RecTab<T> rt(rtab);
  if (far && MODE == FMM_A3B && PART == LEAF_FAR1) {
    fill_rectab(rt, p);
    T* lp = tile;
    for (int i = threadIdx.x; i < L; i += blockDim.x) lp[i] = gL[L + i];
    derive3(gL, p, lp + L, lp + L + Lg, lp + L + 2 * Lg);
    derive3(gL + L, p, lp + L + 3 * Lg, lp + L + 4 * Lg, lp + L + 5 * Lg);
    __syncthreads();
  } else if (far && MODE == FMM_A3B && PART == LEAF_FAR2) {
    // gradient of expansion 1 and scratch in this block's slice of D, the
    // Hessian and the gradient of expansion 2 in LDS
    fill_rectab(rt, p);
    T* dg = D + ((int64_t)widx * nrhs + rhs) * dstride;
    T* tmp = dg + 3 * Lg;
    T* lh = tile;
    derive3(gL + L, p, dg, dg + Lg, dg + 2 * Lg);
    derive3(gL + 2 * L, p, lh + 6 * Lh, lh + 6 * Lh + Lg, lh + 6 * Lh + 2 * Lg);
    __syncthreads();
    derive3(dg, p - 1, lh, lh + Lh, lh + 2 * Lh);                // xx, xy, xz
    derive3(dg + Lg, p - 1, tmp, lh + 3 * Lh, lh + 4 * Lh);      // (yx), yy, yz
    derive3(dg + 2 * Lg, p - 1, tmp + Lh, tmp + 2 * Lh, lh + 5 * Lh);  // (zx), (zy), zz
    __syncthreads();
  } else if (far) {
    fill_rectab(rt, p);
    if (EXP_LDS) {
      for (int i = threadIdx.x; i < nexp * L; i += blockDim.x) sL[i] = gL[i];
      __syncthreads();
    }
    if (MODE == FMM_GRAD || MODE == FMM_A3B) {
      for (int e = 0; e < nexp; ++e)
        derive3(sL + e * L, p, sG + (e * 3 + 0) * Lg, sG + (e * 3 + 1) * Lg, sG + (e * 3 + 2) * Lg);
    }
    if (MODE == FMM_GRAD) {
      // (phi, d/dx, d/dy, d/dz) of each real coefficient side by side, the
      // factors of the real-part evaluation folded in (2 Re and -2 Im for
      // m > 0), the gradients zero for n = p: one 4-vector read per part
      __syncthreads();
      for (int c = threadIdx.x; c < L; c += blockDim.x) {
        int n = 0;
        while ((n + 1) * (n + 1) <= c) ++n;
        const int r = c - n * n;  // 0: m = 0; odd: Re of m = (r+1)/2; even > 0: Im
        const T f = r == 0 ? (T)1 : ((r & 1) ? (T)2 : (T)-2);
        T4 z;
        z.x = f * sL[c];
        z.y = n < p ? f * sG[c] : (T)0;
        z.z = n < p ? f * sG[Lg + c] : (T)0;
        z.w = n < p ? f * sG[2 * Lg + c] : (T)0;
        sZ[c] = z;
      }
    }
    if (MODE == FMM_ADJ3) derive3(sL, p, sG, sG + Lg, sG + 2 * Lg);  // gradient of expansion 1
    if (MODE == FMM_A3B) {
      // second derivatives of expansion 1 from its gradient expansions; the
      // scratch after sH receives the unused d/dx of d/dy and d/dx, d/dy of d/dz
      __syncthreads();
      T* tmp = sH + 6 * Lh;
      const T* gx = sG + 3 * Lg;
      const T* gy = sG + 4 * Lg;
      const T* gz = sG + 5 * Lg;
      derive3(gx, p - 1, sH, sH + Lh, sH + 2 * Lh);          // xx, xy, xz
      derive3(gy, p - 1, tmp, sH + 3 * Lh, sH + 4 * Lh);     // (yx), yy, yz
      derive3(gz, p - 1, tmp + Lh, tmp + 2 * Lh, sH + 5 * Lh);  // (zx), (zy), zz
    }
    if (Z16) {
      __syncthreads();
      for (int c = threadIdx.x; c < L; c += blockDim.x) {
        int n = 0;
        while ((n + 1) * (n + 1) <= c) ++n;
        const int r = c - n * n;
        const T f = r == 0 ? (T)1 : ((r & 1) ? (T)2 : (T)-2);
        const T fg = n < p ? f : (T)0, fh = n < p - 1 ? f : (T)0;
        const int cg = n < p ? c : 0, ch = n < p - 1 ? c : 0;  // clamped: the factor is zero there
        T4 z0, z1, z2, z3;
        z0.x = f * xP[c];         z0.y = fg * xG1[cg];          z0.z = fg * xG1[Lg + cg];     z0.w = fg * xG1[2 * Lg + cg];
        z1.x = fg * xG2[cg];      z1.y = fg * xG2[Lg + cg];     z1.z = fg * xG2[2 * Lg + cg]; z1.w = fg * xG3[cg];
        z2.x = fg * xG3[Lg + cg]; z2.y = fg * xG3[2 * Lg + cg]; z2.z = fh * xH[ch];           z2.w = fh * xH[Lh + ch];
        z3.x = fh * xH[2 * Lh + ch]; z3.y = fh * xH[3 * Lh + ch]; z3.z = fh * xH[4 * Lh + ch]; z3.w = fh * xH[5 * Lh + ch];
        sZ16[4 * c] = z0; sZ16[4 * c + 1] = z1; sZ16[4 * c + 2] = z2; sZ16[4 * c + 3] = z3;
      }
    }
    __syncthreads();
  }
  const T h = t.leaf_h[b];
  const T ih = (T)1 / h;
  const T cx = t.bcx[g], cy = t.bcy[g], cz = t.bcz[g];
  // source records in LDS: (x, y, z, q1), (nx, ny, nz, q2) and rm2
  T4* rec1 = reinterpret_cast<T4*>(tile);
  T4* rec2 = rec1 + LEAF_CH;                                                   // A3B only
  // the mask radius is the target's in the transposed-tree modes (FMM_ADJ
  // with target radii, FMM_ADJ3), else the source's; TMASK sizes the records
  constexpr bool TMASK = MODE == FMM_ADJ || MODE == FMM_ADJ3;
  const bool tmask = MODE == FMM_ADJ3 || (MODE == FMM_ADJ && t.trm2 != nullptr);
  T* trm_ = reinterpret_cast<T*>(rec1 + (MODE == FMM_A3B || TMASK ? 2 : 1) * LEAF_CH);
  __shared__ int upref[28];
  const int u0 = t.ulist_ptr[b], nU = t.ulist_ptr[b + 1] - u0;
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int k = 0; k < nU; ++k) {
      upref[k] = acc;
      const int nb = t.ulist[u0 + k];
      acc += t.src_end[nb] - t.src_beg[nb];
    }
    upref[nU] = acc;
  }
  __syncthreads();
  const int utot = FARONLY ? 0 : upref[nU];
  // ---- far field: the local expansions at xi = (x - c)/h, one thread per
  // target, so that every lane of a wave runs the same (n, m) term: the
  // recurrence coefficients and expansion reads are wave-uniform and no
  // lane idles in a divergent branch ----
  auto far_target = [&](int i, T& o0, T& o1, T& o2, T& o3) __attribute__((always_inline)) {
    const T X = t.tx[i], Y = t.ty[i], Z = t.tz[i];
    T NX = 0, NY = 0, NZ = 0;
    if (MODE == FMM_A3B || MODE == FMM_ADJ3) { NX = t.tnx[i]; NY = t.tny[i]; NZ = t.tnz[i]; }
    const T x = (X - cx) * ih, y = (Y - cy) * ih, z = (Z - cz) * ih;
    const T r2 = x * x + y * y + z * z;
    if constexpr (MODE == FMM_GRAD) {
      // the interleaved, prefactored coefficients: column m = 0 (real
      // harmonics), then m >= 1 (real and imaginary parts)
      T pot = 0, gx = 0, gy = 0, gz = 0;
      T mre = 1, mim = 0;
      {
        T are = 0, bre = 1;
        for (int n = 0; n <= p; ++n) {
          if (n == 1) {
            are = bre; bre = z * rt.up[0] * bre;
          } else if (n > 1) {
            const int cc = cidx(n - 1, 0);
            const T c = rt.a[cc] * z * bre - rt.b[cc] * r2 * are;
            are = bre; bre = c;
          }
          const T4 v = sZ[n * n];
          pot += v.x * bre; gx += v.y * bre; gy += v.z * bre; gz += v.w * bre;
        }
      }
      for (int m = 1; m <= p; ++m) {
        const T fm = rt.sect[m];
        const T nr = fm * (x * mre - y * mim);
        const T ni = fm * (x * mim + y * mre);
        mre = nr; mim = ni;
        T are = 0, aim = 0, bre = mre, bim = mim;  // R_{n-1}, R_n with n = m
        for (int n = m; n <= p; ++n) {
          if (n == m + 1) {
            const T c1 = z * rt.up[m];
            are = bre; aim = bim; bre = c1 * bre; bim = c1 * bim;
          } else if (n > m + 1) {
            const int cc = cidx(n - 1, m);
            const T f1 = rt.a[cc] * z, f2 = rt.b[cc] * r2;
            const T cre = f1 * bre - f2 * are;
            const T cim = f1 * bim - f2 * aim;
            are = bre; aim = bim; bre = cre; bim = cim;
          }
          const T4 vr = sZ[n * n + 2 * m - 1], vi = sZ[n * n + 2 * m];
          pot += vr.x * bre + vi.x * bim;
          gx += vr.y * bre + vi.y * bim;
          gy += vr.z * bre + vi.z * bim;
          gz += vr.w * bre + vi.w * bim;
        }
      }
      o0 = pot; o1 = gx * ih; o2 = gy * ih; o3 = gz * ih;
      return;
    }
    if constexpr (Z16) {
      // the 16 interleaved, prefactored values per coefficient: column m = 0,
      // then m >= 1
      T acc[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) acc[k] = 0;
      auto add = [&](const T4* zc, T br, T bi, const T4* zs) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const T4 u = zc[q];
          if (zs) {
            const T4 v = zs[q];
            acc[4 * q] += u.x * br + v.x * bi; acc[4 * q + 1] += u.y * br + v.y * bi;
            acc[4 * q + 2] += u.z * br + v.z * bi; acc[4 * q + 3] += u.w * br + v.w * bi;
          } else {
            acc[4 * q] += u.x * br; acc[4 * q + 1] += u.y * br; acc[4 * q + 2] += u.z * br; acc[4 * q + 3] += u.w * br;
          }
        }
      };
      T mre = 1, mim = 0;
      {
        T are = 0, bre = 1;
        for (int n = 0; n <= p; ++n) {
          if (n == 1) {
            are = bre; bre = z * rt.up[0] * bre;
          } else if (n > 1) {
            const int cc = cidx(n - 1, 0);
            const T c = rt.a[cc] * z * bre - rt.b[cc] * r2 * are;
            are = bre; bre = c;
          }
          add(sZ16 + 4 * (n * n), bre, (T)0, nullptr);
        }
      }
      for (int m = 1; m <= p; ++m) {
        const T fm = rt.sect[m];
        const T nr = fm * (x * mre - y * mim);
        const T ni = fm * (x * mim + y * mre);
        mre = nr; mim = ni;
        T are = 0, aim = 0, bre = mre, bim = mim;
        for (int n = m; n <= p; ++n) {
          if (n == m + 1) {
            const T c1 = z * rt.up[m];
            are = bre; aim = bim; bre = c1 * bre; bim = c1 * bim;
          } else if (n > m + 1) {
            const int cc = cidx(n - 1, m);
            const T f1 = rt.a[cc] * z, f2 = rt.b[cc] * r2;
            const T cre = f1 * bre - f2 * are;
            const T cim = f1 * bim - f2 * aim;
            are = bre; aim = bim; bre = cre; bim = cim;
          }
          add(sZ16 + 4 * (n * n + 2 * m - 1), bre, bim, sZ16 + 4 * (n * n + 2 * m));
        }
      }
      // acc: pot, g1 (3), g2 (3), g3 (3), Hessian xx xy xz yy yz zz
      o0 = (NX * acc[1] + NY * acc[2] + NZ * acc[3]) * ih;
      o1 = acc[0];
      o2 = (NX * acc[4] + NY * acc[5] + NZ * acc[6]) * ih;
      const T nhn = NX * NX * acc[10] + 2 * NX * NY * acc[11] + 2 * NX * NZ * acc[12] + NY * NY * acc[13] +
                    2 * NY * NZ * acc[14] + NZ * NZ * acc[15];
      o3 = nhn * ih * ih + (NX * acc[7] + NY * acc[8] + NZ * acc[9]) * ih;
      return;
    }
    T pot = 0, pot2 = 0, g1[3] = {0, 0, 0}, g2[3] = {0, 0, 0}, g3[3] = {0, 0, 0}, hs[6] = {0, 0, 0, 0, 0, 0};
    T mre = 1, mim = 0;
    for (int m = 0; m <= p; ++m) {
      if (m > 0) {
        const T fm = rt.sect[m];
        T nr = fm * (x * mre - y * mim);
        T ni = fm * (x * mim + y * mre);
        mre = nr; mim = ni;
      }
      T are = 0, aim = 0, bre = mre, bim = mim;  // R_{n-1}, R_n with n = m
      for (int n = m; n <= p; ++n) {
        if (n > m) {
          T cre, cim;
          if (n == m + 1) {
            T c1 = z * rt.up[m];
            cre = c1 * bre; cim = c1 * bim;
          } else {
            const int cc = cidx(n - 1, m);
            const T f1 = rt.a[cc] * z, f2 = rt.b[cc] * r2;
            cre = f1 * bre - f2 * are;
            cim = f1 * bim - f2 * aim;
          }
          are = bre; aim = bim; bre = cre; bim = cim;
        }
        T rre, rim;
        int ire, iim;
        if (m == 0) { rre = bre; rim = 0; ire = n * n; iim = -1; }
        else { rre = 2 * bre; rim = -2 * bim; ire = n * n + 2 * m - 1; iim = n * n + 2 * m; }
#define ACC(dst, base, idxre, idxim) dst += (base)[idxre] * rre + ((idxim) >= 0 ? (base)[idxim] * rim : (T)0)
        if (MODE == FMM_POT || MODE == FMM_ADJ) {
          ACC(pot, sL, ire, iim);
        } else if (MODE == FMM_ADJ3) {
          ACC(pot, sL, ire, iim);
          ACC(pot2, sL + L, ire, iim);
          if (n < p) {
            ACC(g1[0], sG, ire, iim);
            ACC(g1[1], sG + Lg, ire, iim);
            ACC(g1[2], sG + 2 * Lg, ire, iim);
          }
        } else {  // A3B (GRAD returned above)
          if (PART != LEAF_FAR2) {
            ACC(pot, xP, ire, iim);  // phi_2
            if (n < p) {
              ACC(g1[0], xG1, ire, iim);
              ACC(g1[1], xG1 + Lg, ire, iim);
              ACC(g1[2], xG1 + 2 * Lg, ire, iim);
              ACC(g2[0], xG2, ire, iim);
              ACC(g2[1], xG2 + Lg, ire, iim);
              ACC(g2[2], xG2 + 2 * Lg, ire, iim);
            }
          }
          if (PART != LEAF_FAR1) {
            if (n < p) {
              ACC(g3[0], xG3, ire, iim);
              ACC(g3[1], xG3 + Lg, ire, iim);
              ACC(g3[2], xG3 + 2 * Lg, ire, iim);
            }
            if (n < p - 1) {
#pragma unroll
              for (int q = 0; q < 6; ++q) ACC(hs[q], xH + q * Lh, ire, iim);
            }
          }
        }
#undef ACC
      }
    }
    if (MODE == FMM_POT || MODE == FMM_ADJ) {
      o0 = pot;
    } else if (MODE == FMM_ADJ3) {
      o0 = pot;
      o1 = pot2 + (NX * g1[0] + NY * g1[1] + NZ * g1[2]) * ih;
    } else {
      o0 = (NX * g1[0] + NY * g1[1] + NZ * g1[2]) * ih;
      o1 = pot;
      o2 = (NX * g2[0] + NY * g2[1] + NZ * g2[2]) * ih;
      T nhn = NX * NX * hs[0] + 2 * NX * NY * hs[1] + 2 * NX * NZ * hs[2] + NY * NY * hs[3] +
              2 * NY * NZ * hs[4] + NZ * NZ * hs[5];
      o3 = nhn * ih * ih + (NX * g3[0] + NY * g3[1] + NZ * g3[2]) * ih;
    }
  };
  if (FARONLY) {
    if (far) {
      for (int i = tbeg + (int)threadIdx.x; i < tend; i += blockDim.x) {
        T o0 = 0, o1 = 0, o2 = 0, o3 = 0;
        far_target(i, o0, o1, o2, o3);
        const int64_t base = (int64_t)rhs * nout * N;
        if (PART == LEAF_FAR1) {
          out[base + i] += o0;
          out[base + N + i] += o1;
          out[base + 2 * N + i] += o2;
        } else if (PART == LEAF_FAR2) {
          out[base + 3 * N + i] += o3;
        } else {  // after the near-field kernel (stream ordered)
          out[base + i] += o0;
          if (nout > 1) out[base + N + i] += o1;
          if (nout > 2) {
            out[base + 2 * N + i] += o2;
            out[base + 3 * N + i] += o3;
          }
        }
      }
    }
    return;
  }
  for (int i0 = tbeg; i0 < tend; i0 += TPB) {
    const int i = i0 + slot;
    const bool act = i < tend;
    T X = 0, Y = 0, Z = 0, NX = 0, NY = 0, NZ = 0, TR = 0;
    if (act) { X = t.tx[i]; Y = t.ty[i]; Z = t.tz[i]; NX = t.tnx[i]; NY = t.tny[i]; NZ = t.tnz[i]; }
    if (tmask && act) TR = t.trm2[i];
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    if (far) {
      // the far field of the pass's targets, one per thread, through the
      // source chunk area (free until the near field restages it) to the
      // first lane of each target
      T* fb = tile;
      const int nf = min(TPB, tend - i0);
      __syncthreads();  // the previous pass may still read its last chunk
      if ((int)threadIdx.x < nf) {
        T o0 = 0, o1 = 0, o2 = 0, o3 = 0;
        far_target(i0 + threadIdx.x, o0, o1, o2, o3);
        fb[4 * threadIdx.x] = o0;
        fb[4 * threadIdx.x + 1] = o1;
        fb[4 * threadIdx.x + 2] = o2;
        fb[4 * threadIdx.x + 3] = o3;
      }
      __syncthreads();
      if (act && f == 0) { a0 = fb[4 * slot]; a1 = fb[4 * slot + 1]; a2 = fb[4 * slot + 2]; a3 = fb[4 * slot + 3]; }
      __syncthreads();  // before the near field restages the area
    }
    // ---- near field: U-list direct sums.  The U-list sources are gathered
    // into LDS in chunks of LEAF_CH (several neighbour boxes per chunk);
    // pairs are summed in T per chunk and the chunk sums in FP64 ----
    for (int c0 = 0; c0 < utot; c0 += LEAF_CH) {
      const int ns = min(LEAF_CH, utot - c0);
      __syncthreads();
      for (int k = 0; k < nU; ++k) {
        const int lo = max(c0, upref[k]), hi = min(c0 + ns, upref[k + 1]);
        if (lo >= hi) continue;
        const int sbase = t.src_beg[t.ulist[u0 + k]] - upref[k];
        for (int gj = lo + (int)threadIdx.x; gj < hi; gj += blockDim.x) {
        const int j = gj - c0;
        const int s = sbase + gj;
        T4 r1;
        r1.x = t.sx[s];
        r1.y = t.sy[s];
        r1.z = t.sz[s];
        r1.w = str[(int64_t)(rhs * nstr) * No + s];
        rec1[j] = r1;
        if (!tmask) trm_[j] = t.rm2[s];
        if (MODE == FMM_A3B || MODE == FMM_ADJ3) {
          T4 r2;
          r2.x = t.snx[s];
          r2.y = t.sny[s];
          r2.z = t.snz[s];
          r2.w = str[(int64_t)(rhs * nstr + 1) * No + s];
          rec2[j] = r2;
        }
        if (MODE == FMM_ADJ) {  // dipole vector
          T4 r2;
          r2.x = str[(int64_t)(rhs * nstr + 1) * No + s];
          r2.y = str[(int64_t)(rhs * nstr + 2) * No + s];
          r2.z = str[(int64_t)(rhs * nstr + 3) * No + s];
          r2.w = 0;
          rec2[j] = r2;
        }
        }
      }
      __syncthreads();
      if (act) {
        T q0 = 0, q1 = 0, q2 = 0, q3 = 0;
        // one (target, source jj) pair
        auto pair = [&](int jj) __attribute__((always_inline)) {
            const T4 r1 = rec1[jj];
            // the mask radius of the pair: the source's, or the target's on the transposed tree
            const T rm = tmask ? TR : trm_[jj];
            const T dx = X - r1.x;
            const T dy = Y - r1.y;
            const T dz = Z - r1.z;
            const T r2 = dev_fma(dz, dz, dev_fma(dy, dy, dx * dx));
            // pairs inside the mask radius are handled by the stored corrections
            // (rm > 0 always, so coincident points are skipped too)
            const bool skip = r2 < rm;
            const T ri = skip ? (T)0 : dev_rsqrt(skip ? (T)1 : r2);
            const T ri2 = ri * ri;
            const T ri3 = ri * ri2;
            if (MODE == FMM_POT) {
              q0 += r1.w * ri;
            } else if (MODE == FMM_ADJ) {
              const T4 dv = rec2[jj];
              q0 += r1.w * ri + (dv.x * dx + dv.y * dy + dv.z * dz) * ri3;
            } else if (MODE == FMM_ADJ3) {
              // source normal in rec2, target normal (NX, NY, NZ)
              const T4 nv = rec2[jj];
              const T nd = nv.x * dx + nv.y * dy + nv.z * dz;
              const T mx = nv.x - NX, my = nv.y - NY, mz = nv.z - NZ;
              const T md = mx * dx + my * dy + mz * dz;
              const T nm = nv.x * mx + nv.y * my + nv.z * mz;
              q0 += r1.w * nd * ri3;
              q1 += r1.w * ((T)3 * nd * md * ri3 * ri2 - nm * ri3) + nv.w * nd * ri3;
            } else if (MODE == FMM_GRAD) {
              const T q = r1.w;
              const T qr3 = q * ri3;
              q0 += q * ri;
              q1 -= qr3 * dx;
              q2 -= qr3 * dy;
              q3 -= qr3 * dz;
            } else {
              const T4 r2v = rec2[jj];
              const T c1 = r1.w, c2 = r2v.w;
              const T nd = NX * dx + NY * dy + NZ * dz;
              const T mx = NX - r2v.x, my = NY - r2v.y, mz = NZ - r2v.z;
              const T md = mx * dx + my * dy + mz * dz;
              const T nm = NX * mx + NY * my + NZ * mz;
              q0 -= c1 * nd * ri3;
              q1 += c2 * ri;
              q2 -= c2 * nd * ri3;
              q3 += c2 * ((T)3 * nd * md * ri3 * ri2 - nm * ri3);
            }
        };
        // the lane stride F as a compile-time constant, so that the unrolled
        // LDS reads take immediate offsets
        auto sweep = [&](auto fc) __attribute__((always_inline)) {
          constexpr int FF = decltype(fc)::value;
#pragma unroll LB_LEAF_UNROLL
          for (int jj = f; jj < ns; jj += FF) pair(jj);
        };
        switch (F) {
          case 1: sweep(std::integral_constant<int, 1>{}); break;
          case 2: sweep(std::integral_constant<int, 2>{}); break;
          case 4: sweep(std::integral_constant<int, 4>{}); break;
          case 8: sweep(std::integral_constant<int, 8>{}); break;
          case 16: sweep(std::integral_constant<int, 16>{}); break;
          case 32: sweep(std::integral_constant<int, 32>{}); break;
          default: sweep(std::integral_constant<int, 64>{}); break;
        }
        a0 += (double)q0; a1 += (double)q1; a2 += (double)q2; a3 += (double)q3;
      }
    }
    // sum the F partials of each target (contiguous lanes; F divides 64)
    for (int off = 1; off < F; off <<= 1) {
      a0 += __shfl_xor(a0, off, 64);
      a1 += __shfl_xor(a1, off, 64);
      a2 += __shfl_xor(a2, off, 64);
      a3 += __shfl_xor(a3, off, 64);
    }
    if (act && f == 0) {
      const int64_t base = (int64_t)rhs * nout * N;
      out[base + i] = (T)a0;
      if (nout > 1) out[base + N + i] = (T)a1;
      if (nout > 2) {
        out[base + 2 * N + i] = (T)a2;
        out[base + 3 * N + i] = (T)a3;
      }
    }
  }
}

// One work item per block; the near-field part of the overlapped apply
// takes the items b, b + gridDim.x, ... (heaviest first), so that a grid
// smaller than the item count leaves wave slots to the far-field kernels
// running at the same time on the other stream.
template <typename T, int MODE, bool EXP_LDS, int PART>
__global__ __launch_bounds__(LEAF_BS) __attribute__((amdgpu_waves_per_eu(leaf_waves<T, MODE>())))
void k_leaf(DevTree<T> t, int nrhs, const T* __restrict__ str, int64_t No, const T* __restrict__ Lc,
            T* __restrict__ D, T* __restrict__ out, int64_t N) {
  if (PART == LEAF_NEAR) {
    for (int w = blockIdx.x; w < t.n_leaf_work; w += gridDim.x) {
      leaf_item<T, MODE, EXP_LDS, PART>(t, nrhs, str, No, Lc, D, out, N, w);
      __syncthreads();  // the next item restages LDS
    }
  } else {
    leaf_item<T, MODE, EXP_LDS, PART>(t, nrhs, str, No, Lc, D, out, N, blockIdx.x);
  }
}

// Values per (work item, density) the leaf kernels of `mode` read and write
// in the workspace D: zero when every part keeps its expansions in LDS (the
// choices of launch_leaf below, taken for the part that also stages sources).
template <typename T>
int64_t leaf_d_stride(int mode, int p) {
  const size_t chunk = sizeof(T) * (mode == FMM_A3B || mode == FMM_ADJ || mode == FMM_ADJ3 ? 9 : 5) * LEAF_CH;
  if (chunk + leaf_exp_bytes<T>(mode, p) <= 40 * 1024) return 0;
  const size_t stat = sizeof(T) * RECTAB_N + 512;
  if (mode == FMM_A3B && leaf_far_split_bytes<T>(LEAF_FAR1, p) + stat <= 64 * 1024 &&
      leaf_far_split_bytes<T>(LEAF_FAR2, p) + stat <= 64 * 1024)
    return 0;
  return leaf_d_vals(mode, p);
}

template <typename T>
static void launch_leaf(const DevTree<T>& t, int mode, int part, int nrhs, const T* str, const T* Lc, T* D, T* out,
                        int64_t N, int64_t No, hipStream_t st) {
  const int p = t.p, L = t.L;
  const int nexp = fmm_nexp(mode);
  // LDS: staged sources (not in the far-only kernel), then the expansions
  // when both stay within 40 KiB (at least 4 blocks per CU: more LDS per
  // block costs more in occupancy than the global reads of the expansions,
  // e.g. 1.42 ms -> 1.74 ms for the FP64 gradient kernel at 45 KiB)
  const size_t chunk = part == LEAF_FAR ? 0
                       : sizeof(T) * (mode == FMM_A3B || mode == FMM_ADJ || mode == FMM_ADJ3 ? 9 : 5) * LEAF_CH;
  const size_t exps = part == LEAF_NEAR ? 0
                      : leaf_exp_bytes<T>(mode, p) + (part == LEAF_FAR && mode == FMM_A3B ? leaf_z16_bytes<T>(p) : 0);
  const bool lds = chunk + exps <= 40 * 1024;
  const size_t sml = lds ? chunk + exps : chunk;
  (void)L; (void)nexp;
  // A3B whose expansions do not fit: the far part in two passes that keep
  // theirs in LDS (within 64 KiB per block with the static tables)
  const size_t stat = sizeof(T) * RECTAB_N + 512;
  if (mode == FMM_A3B && !lds && part != LEAF_NEAR &&
      leaf_far_split_bytes<T>(LEAF_FAR1, p) + stat <= 64 * 1024 &&
      leaf_far_split_bytes<T>(LEAF_FAR2, p) + stat <= 64 * 1024) {
    if (part == LEAF_BOTH) launch_leaf<T>(t, mode, LEAF_NEAR, nrhs, str, Lc, D, out, N, No, st);
    const dim3 gf(t.n_leaf_work, nrhs);
    hipLaunchKernelGGL((k_leaf<T, FMM_A3B, true, LEAF_FAR1>), gf, dim3(LEAF_BS), leaf_far_split_bytes<T>(LEAF_FAR1, p),
                       st, t, nrhs, str, No, Lc, D, out, N);
    hipLaunchKernelGGL((k_leaf<T, FMM_A3B, true, LEAF_FAR2>), gf, dim3(LEAF_BS), leaf_far_split_bytes<T>(LEAF_FAR2, p),
                       st, t, nrhs, str, No, Lc, D, out, N);
    KCHECK();
    return;
  }
  const int gx = part == LEAF_NEAR && t.near_grid > 0 ? std::min(t.n_leaf_work, t.near_grid) : t.n_leaf_work;
  dim3 grid(gx, nrhs);
#define LEAF_LAUNCH(MD, PT)                                                                                    \
  if (lds)                                                                                                     \
    hipLaunchKernelGGL((k_leaf<T, MD, true, PT>), grid, dim3(LEAF_BS), sml, st, t, nrhs, str, No, Lc, D, out, N); \
  else                                                                                                         \
    hipLaunchKernelGGL((k_leaf<T, MD, false, PT>), grid, dim3(LEAF_BS), sml, st, t, nrhs, str, No, Lc, D, out, N);
#define LEAF_PARTS(MD)                    \
  if (part == LEAF_NEAR) {                \
    LEAF_LAUNCH(MD, LEAF_NEAR)            \
  } else if (part == LEAF_FAR) {          \
    LEAF_LAUNCH(MD, LEAF_FAR)             \
  } else {                                \
    LEAF_LAUNCH(MD, LEAF_BOTH)            \
  }
  if (mode == FMM_POT) {
    LEAF_PARTS(FMM_POT)
  } else if (mode == FMM_GRAD) {
    LEAF_PARTS(FMM_GRAD)
  } else if (mode == FMM_ADJ) {
    LEAF_PARTS(FMM_ADJ)
  } else if (mode == FMM_ADJ3) {
    LEAF_PARTS(FMM_ADJ3)
  } else {
    LEAF_PARTS(FMM_A3B)
  }
#undef LEAF_PARTS
#undef LEAF_LAUNCH
  KCHECK();
}

template <typename T>
void launch_fmm(const DevTree<T>& t, int mode, int nrhs, const T* str, T* M, T* Lc, T* D, T* out,
                int64_t N, int64_t No, hipStream_t st, PhaseTimer* tm) {
  PhaseTimer dummy;
  if (!tm) tm = &dummy;
  const int p = t.p, L = t.L, Lc_ = (p + 1) * (p + 2) / 2;
  const int ne = nrhs * fmm_nexp(mode);
  if (t.depth >= 2 && ne > t.m2l_plan->ne_max)
    fail(LB_EINVAL, "launch_fmm called with %d expansions (at most %d)", ne, t.m2l_plan->ne_max);
  // With a side stream, the near-field sums (which need only the strengths)
  // run there while this stream does P2M (unless fork_late), M2M, M2L and
  // L2L; the L2P kernel then adds the far field.  Timed applies stay serial.
  const bool ovl = t.side && t.depth >= 2 && !tm->on;
  auto fork = [&]() {
    (void)hipEventRecord(t.fork_ev, st);
    (void)hipStreamWaitEvent(t.side, t.fork_ev, 0);
    launch_leaf<T>(t, mode, LEAF_NEAR, nrhs, str, Lc, D, out, N, No, t.side);
    (void)hipEventRecord(t.join_ev, t.side);
  };
  if (ovl && !t.fork_late) fork();
  if (t.depth >= 2) {
    // source tile of P2M: harmonic tables of ts sources within 48 KiB of LDS
    int ts = (int)((48 * 1024 / sizeof(T) - RECTAB_N - 5 * P2M_TSMAX) / (2 * Lc_));
    ts = ts < 1 ? 1 : (ts > P2M_TSMAX ? P2M_TSMAX : ts);
    size_t sm = sizeof(T) * (2 * ts * Lc_ + 5 * ts);
    if (t.p2m_H && mode == FMM_ADJ3) fail(LB_EINVAL, "P2M tables are not built for the transposed tree");
    if (mode == FMM_ADJ3) {
      int ts3 = (int)((48 * 1024 / sizeof(T) - RECTAB_N - 5 * P2M_TSMAX) / (4 * Lc_));
      ts3 = ts3 < 1 ? 1 : (ts3 > P2M_TSMAX ? P2M_TSMAX : ts3);
      const size_t sm3 = sizeof(T) * (4 * (size_t)ts3 * Lc_ + 5 * ts3);
      hipLaunchKernelGGL(k_p2m_adj3<T>, dim3(t.n_leaf_src, nrhs), dim3(256), sm3, st, t, nrhs, str, No, M, ts3);
    } else if (t.p2m_H && mode == FMM_A3B)
      hipLaunchKernelGGL((k_p2m_tab<T, true>), dim3(t.n_leaf_src, nrhs), dim3(64 * P2M_W), 0, st, t, nrhs, str, No,
                         t.p2m_H, t.p2m_D, M);
    else if (t.p2m_H && mode != FMM_ADJ)
      hipLaunchKernelGGL((k_p2m_tab<T, false>), dim3(t.n_leaf_src, nrhs), dim3(64 * P2M_W), 0, st, t, nrhs, str, No,
                         t.p2m_H, t.p2m_D, M);
    else  // (FMM_ADJ on the forward tree: arbitrary dipole vectors, harmonics on the fly)
      hipLaunchKernelGGL(k_p2m<T>, dim3(t.n_leaf_src, nrhs), dim3(256), sm, st, t, mode, nrhs, str, No, M, ts);
    KCHECK();
    if (ovl && t.fork_late) fork();
    tm->mark(PH_M2M, st);
    T* Y = (T*)t.Y;
    for (int l = t.depth - 1; l >= 2; --l) run_plan<T>(t.m2m_plan[l], t.m2m, L, ne, M, Y, M, st);
    tm->mark(PH_M2L, st);
    for (int q = 0; q < t.m2l_parts; ++q) run_plan<T>(t.m2l_plan[q], t.m2l, L, ne, M, Y, Lc, st);
    tm->mark(PH_L2L, st);
    for (int l = 3; l <= t.depth; ++l) run_plan<T>(t.l2l_plan[l], t.l2l, L, ne, Lc, Y, Lc, st);
  } else {
    tm->mark(PH_M2M, st);
    tm->mark(PH_M2L, st);
    tm->mark(PH_L2L, st);
  }
  if (ovl) {  // join: the near-field sums are in `out`
    (void)hipStreamWaitEvent(st, t.join_ev, 0);
    launch_leaf<T>(t, mode, LEAF_FAR, nrhs, str, Lc, D, out, N, No, st);
  } else {
    tm->mark(PH_LEAF, st);
    launch_leaf<T>(t, mode, LEAF_BOTH, nrhs, str, Lc, D, out, N, No, st);
  }
}

// ---------------------------------------------------------------------------
// block-CSR corrections fused with the combination step; one wave per row
// ---------------------------------------------------------------------------
constexpr double INV4PI_D = 0.07957747154594767;  // 1/(4 pi)
constexpr int NDMAX = 4;

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Correction rows: one wave per target row.  The row's blocks of n_p
// contiguous columns are spread over the wave as segments of SW lanes
// (SW = 32 for n_p <= 32, else 64): f(entry, column, on) is called for
// every (block, node) pair of the row, with indices clamped into the row so
// that no load is predicated (on = false marks the clamped duplicates, whose
// contribution the caller zeroes).  The patch numbers of up to 64 blocks are
// loaded at once, one per lane, into this wave's 64-int LDS slice `pat`.
template <typename F>
__device__ __forceinline__ void row_blocks(int64_t b0, int64_t b1, int n_p, int lane, const int* __restrict__ patch,
                                           int* pat, F&& f) {
  const int SW = n_p <= 32 ? 32 : 64;
  const int sub = lane / SW, j0 = lane - sub * SW, nsub = 64 / SW, NJ = (n_p + SW - 1) / SW;
  // the row is the same for the whole wave: keep its bounds in scalar registers
  b0 = (int64_t)__builtin_amdgcn_readfirstlane((int)b0) |
       ((int64_t)__builtin_amdgcn_readfirstlane((int)(b0 >> 32)) << 32);
  const int nb = __builtin_amdgcn_readfirstlane((int)(b1 - b0));
  for (int base = 0; base < nb; base += 64) {
    const int nbb = min(64, nb - base);
    __builtin_amdgcn_wave_barrier();
    pat[lane] = patch[b0 + base + min(lane, nbb - 1)];
    __builtin_amdgcn_wave_barrier();
    if (NJ == 1) {  // n_p <= 64: one node per lane and block
      const int jc = min(j0, n_p - 1);
      const bool okj = j0 < n_p;
#pragma unroll 4
      for (int q0 = 0; q0 < nbb; q0 += nsub) {
        const int q = min(q0 + sub, nbb - 1);
        const int64_t pc = (int64_t)pat[q] * n_p;
        f((b0 + base + q) * n_p + jc, pc + jc, okj && q0 + sub < nbb);
      }
    } else {
      for (int q0 = 0; q0 < nbb; q0 += nsub) {
        const int q = min(q0 + sub, nbb - 1);
        const bool okb = q0 + sub < nbb;
        const int64_t pc = (int64_t)pat[q] * n_p;
        const int64_t eb = (b0 + base + q) * n_p;
        for (int jt = 0; jt < NJ; ++jt) {
          const int j = j0 + jt * SW;
          const int jc = min(j, n_p - 1);
          f(eb + jc, pc + jc, okb && j < n_p);
        }
      }
    }
  }
}

template <typename T, int ND>
__global__ __launch_bounds__(256) void k_combine_grad(int64_t N, int n_p, const int64_t* __restrict__ row_ptr,
                                                      const int* __restrict__ patch, const T* __restrict__ vals,
                                                      const T* __restrict__ sigma, const T* __restrict__ fmm,
                                                      const int* __restrict__ tgt_pos, const T* __restrict__ nrm,
                                                      T* pot, T* grad, T* dSdn, T* surf, T* corr) {
  typedef typename Vec4<T>::type T4;
  __shared__ int pat_s[4][64];
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= N) return;
  T acc[ND][4];
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[d][k] = 0;
  const T4* v4 = reinterpret_cast<const T4*>(vals);
  row_blocks(row_ptr[row], row_ptr[row + 1], n_p, lane, patch, pat_s[threadIdx.x >> 6], [&](int64_t e, int64_t col, bool on) {
    const T4 c = v4[e];
    const T m = on ? (T)1 : (T)0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const T x = sigma[(int64_t)d * N + col] * m;
      acc[d][0] += c.x * x; acc[d][1] += c.y * x; acc[d][2] += c.z * x; acc[d][3] += c.w * x;
    }
  });
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[d][k] = wave_sum(acc[d][k]);
  if (corr) {  // corrections only: the final step adds the far sums later
    if (lane == 0)
#pragma unroll
      for (int d = 0; d < ND; ++d)
#pragma unroll
        for (int k = 0; k < 4; ++k) corr[((int64_t)d * N + row) * 4 + k] = acc[d][k];
    return;
  }
  if (lane == 0) {
    const int tp = tgt_pos[row];
    const T n0 = nrm[3 * row], n1 = nrm[3 * row + 1], n2 = nrm[3 * row + 2];
    const T s = (T)INV4PI_D;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const T* f = fmm + (int64_t)d * 4 * N;
      const T P = f[tp] * s + acc[d][0];
      const T gx = f[N + tp] * s + acc[d][1];
      const T gy = f[2 * N + tp] * s + acc[d][2];
      const T gz = f[3 * N + tp] * s + acc[d][3];
      const T dn = n0 * gx + n1 * gy + n2 * gz;
      if (pot) pot[(int64_t)d * N + row] = P;
      if (grad) {
        grad[((int64_t)d * N + row) * 3] = gx;
        grad[((int64_t)d * N + row) * 3 + 1] = gy;
        grad[((int64_t)d * N + row) * 3 + 2] = gz;
      }
      if (dSdn) dSdn[(int64_t)d * N + row] = dn;
      if (surf) {
        surf[((int64_t)d * N + row) * 3] = gx - n0 * dn;
        surf[((int64_t)d * N + row) * 3 + 1] = gy - n1 * dn;
        surf[((int64_t)d * N + row) * 3 + 2] = gz - n2 * dn;
      }
    }
  }
}

// launch a kernel templated on the number of densities ND = 1..NDMAX
#define ND_DISPATCH(KERNEL, ND_, ...)                                                         \
  switch (ND_) {                                                                              \
    case 1: hipLaunchKernelGGL((KERNEL<T, 1>), __VA_ARGS__); break;                          \
    case 2: hipLaunchKernelGGL((KERNEL<T, 2>), __VA_ARGS__); break;                          \
    case 3: hipLaunchKernelGGL((KERNEL<T, 3>), __VA_ARGS__); break;                          \
    default: hipLaunchKernelGGL((KERNEL<T, 4>), __VA_ARGS__); break;                         \
  }

// the far sums (FMM outputs in tree order) plus the corrections computed
// before by k_combine_grad into corr [d][row][4]: the same values as the
// fused kernel (the same sums, added in the same order)
template <typename T>
__global__ void k_combine_grad_fin(int64_t N, int nd, const T* __restrict__ fmm, const T* __restrict__ corr,
                                   const int* __restrict__ tgt_pos, const T* __restrict__ nrm, T* pot, T* grad,
                                   T* dSdn, T* surf) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nd * N) return;
  const int64_t d = t / N, row = t - d * N;
  const int tp = tgt_pos[row];
  const T n0 = nrm[3 * row], n1 = nrm[3 * row + 1], n2 = nrm[3 * row + 2];
  const T s = (T)INV4PI_D;
  const T* f = fmm + d * 4 * N;
  const T* c = corr + t * 4;
  const T P = f[tp] * s + c[0];
  const T gx = f[N + tp] * s + c[1];
  const T gy = f[2 * N + tp] * s + c[2];
  const T gz = f[3 * N + tp] * s + c[3];
  const T dn = n0 * gx + n1 * gy + n2 * gz;
  if (pot) pot[t] = P;
  if (grad) { grad[3 * t] = gx; grad[3 * t + 1] = gy; grad[3 * t + 2] = gz; }
  if (dSdn) dSdn[t] = dn;
  if (surf) { surf[3 * t] = gx - n0 * dn; surf[3 * t + 1] = gy - n1 * dn; surf[3 * t + 2] = gz - n2 * dn; }
}

template <typename T>
void launch_combine_grad(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch,
                         const T* vals4, const T* sigma, const T* fmm, const int* tgt_pos,
                         const T* nrm, T* pot, T* grad, T* dSdn, T* surf, hipStream_t st) {
  for (int d0 = 0; d0 < nd; d0 += NDMAX) {
    int ndc = nd - d0 < NDMAX ? nd - d0 : NDMAX;
    ND_DISPATCH(k_combine_grad, ndc, dim3((N + 3) / 4), dim3(256), 0, st, N, n_p, row_ptr, patch, vals4,
                sigma + (int64_t)d0 * N, fmm + (int64_t)d0 * 4 * N, tgt_pos, nrm,
                pot ? pot + (int64_t)d0 * N : nullptr, grad ? grad + (int64_t)d0 * 3 * N : nullptr,
                dSdn ? dSdn + (int64_t)d0 * N : nullptr, surf ? surf + (int64_t)d0 * 3 * N : nullptr,
                (T*)nullptr)
  }
  KCHECK();
}

template <typename T>
void launch_corr_grad(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch, const T* vals4,
                      const T* sigma, T* corr, hipStream_t st) {
  for (int d0 = 0; d0 < nd; d0 += NDMAX) {
    int ndc = nd - d0 < NDMAX ? nd - d0 : NDMAX;
    ND_DISPATCH(k_combine_grad, ndc, dim3((N + 3) / 4), dim3(256), 0, st, N, n_p, row_ptr, patch, vals4,
                sigma + (int64_t)d0 * N, (const T*)nullptr, (const int*)nullptr, (const T*)nullptr, (T*)nullptr,
                (T*)nullptr, (T*)nullptr, (T*)nullptr, corr + (int64_t)d0 * 4 * N)
  }
  KCHECK();
}

template <typename T>
void launch_combine_grad_fin(int nd, int64_t N, const T* fmm, const T* corr, const int* tgt_pos, const T* nrm,
                             T* pot, T* grad, T* dSdn, T* surf, hipStream_t st) {
  const int64_t n = (int64_t)nd * N;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_combine_grad_fin<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, N, nd, fmm, corr,
                     tgt_pos, nrm, pot, grad, dSdn, surf);
  KCHECK();
}


// S only: pot = phi / (4 pi) + C_S sigma (vals3 column 0), FMM_POT output
template <typename T, int ND>
__global__ __launch_bounds__(256) void k_combine_pot(int64_t N, int n_p, const int64_t* __restrict__ row_ptr,
                                                     const int* __restrict__ patch, const T* __restrict__ vals,
                                                     const T* __restrict__ sigma, const T* __restrict__ fmm,
                                                     const int* __restrict__ tgt_pos, T* pot) {
  __shared__ int pat_s[4][64];
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= N) return;
  T acc[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) acc[d] = 0;
  row_blocks(row_ptr[row], row_ptr[row + 1], n_p, lane, patch, pat_s[threadIdx.x >> 6], [&](int64_t e, int64_t col, bool on) {
    const T c0 = vals[e * 3];
    const T m = on ? (T)1 : (T)0;
#pragma unroll
    for (int d = 0; d < ND; ++d) acc[d] += c0 * sigma[(int64_t)d * N + col] * m;
  });
#pragma unroll
  for (int d = 0; d < ND; ++d) acc[d] = wave_sum(acc[d]);
  if (lane == 0) {
    const int tp = tgt_pos[row];
#pragma unroll
    for (int d = 0; d < ND; ++d) pot[(int64_t)d * N + row] = fmm[(int64_t)d * N + tp] * (T)INV4PI_D + acc[d];
  }
}

template <typename T>
void launch_combine_pot(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch, const T* vals3,
                        const T* sigma, const T* fmm, const int* tgt_pos, T* pot, hipStream_t st) {
  for (int d0 = 0; d0 < nd; d0 += NDMAX) {
    int ndc = nd - d0 < NDMAX ? nd - d0 : NDMAX;
    ND_DISPATCH(k_combine_pot, ndc, dim3((N + 3) / 4), dim3(256), 0, st, N, n_p, row_ptr, patch, vals3,
                sigma + (int64_t)d0 * N, fmm + (int64_t)d0 * N, tgt_pos, pot + (int64_t)d0 * N)
    KCHECK();
  }
}

// A3 step 1: mu2 = S tau, mu1 = S' tau  (vals3 columns: S, S', S''+D')
template <typename T, int ND>
__global__ __launch_bounds__(256) void k_combine_a3a(int64_t N, int n_p, const int64_t* __restrict__ row_ptr,
                                                     const int* __restrict__ patch, const T* __restrict__ vals,
                                                     const T* __restrict__ tau, const T* __restrict__ fmm,
                                                     const int* __restrict__ tgt_pos, const T* __restrict__ nrm,
                                                     T* mu1, T* mu2, int64_t ldmu) {
  __shared__ int pat_s[4][64];
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= N) return;
  T aS[ND], aP[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) { aS[d] = 0; aP[d] = 0; }
  row_blocks(row_ptr[row], row_ptr[row + 1], n_p, lane, patch, pat_s[threadIdx.x >> 6], [&](int64_t e, int64_t col, bool on) {
    const T* c = vals + e * 3;
    const T c0 = c[0], c1 = c[1];
    const T m = on ? (T)1 : (T)0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const T x = tau[(int64_t)d * N + col] * m;
      aS[d] += c0 * x;
      aP[d] += c1 * x;
    }
  });
#pragma unroll
  for (int d = 0; d < ND; ++d) { aS[d] = wave_sum(aS[d]); aP[d] = wave_sum(aP[d]); }
  if (lane == 0) {
    const int tp = tgt_pos[row];
    const T n0 = nrm[3 * row], n1 = nrm[3 * row + 1], n2 = nrm[3 * row + 2];
    const T s = (T)INV4PI_D;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const T* f = fmm + (int64_t)d * 4 * N;
      mu2[(int64_t)d * ldmu + row] = f[tp] * s + aS[d];
      mu1[(int64_t)d * ldmu + row] = (n0 * f[N + tp] + n1 * f[2 * N + tp] + n2 * f[3 * N + tp]) * s + aP[d];
    }
  }
}

template <typename T>
void launch_combine_a3a(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch,
                        const T* vals3, const T* tau, const T* fmm, const int* tgt_pos,
                        const T* nrm, T* mu1, T* mu2, int64_t ldmu, hipStream_t st) {
  for (int d0 = 0; d0 < nd; d0 += NDMAX) {
    int ndc = nd - d0 < NDMAX ? nd - d0 : NDMAX;
    ND_DISPATCH(k_combine_a3a, ndc, dim3((N + 3) / 4), dim3(256), 0, st, N, n_p, row_ptr, patch, vals3,
                tau + (int64_t)d0 * N, fmm + (int64_t)d0 * 4 * N, tgt_pos, nrm, mu1 + (int64_t)d0 * ldmu,
                mu2 + (int64_t)d0 * ldmu, ldmu)
    KCHECK();
  }
}

// A3 step 2: per row y1 = S'mu1, y2 = S mu2, y3 = S'mu2, y4 = (S''+D')mu2;
// out = -tau/4 + y1 - y4 - 2 H y3 (the W S[S tau] term is added per surface
// afterwards from y2, kept in y2buf)
template <typename T, int ND>
__global__ __launch_bounds__(256) void k_combine_a3b(int64_t N, int n_p, const int64_t* __restrict__ row_ptr,
                                                     const int* __restrict__ patch, const T* __restrict__ vals,
                                                     const T* __restrict__ tau, const T* __restrict__ mu1,
                                                     const T* __restrict__ mu2, int64_t ldmu, const T* __restrict__ fmm,
                                                     const int* __restrict__ tgt_pos, const T* __restrict__ H,
                                                     T* out, T* y2buf) {
  __shared__ int pat_s[4][64];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * 4 + wv;
  if (row >= N) return;
  T a1[ND], a2[ND], a3[ND], a4[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) { a1[d] = a2[d] = a3[d] = a4[d] = 0; }
  row_blocks(row_ptr[row], row_ptr[row + 1], n_p, lane, patch, pat_s[wv], [&](int64_t e, int64_t col, bool on) {
    const T* c = vals + e * 3;
    const T cS = c[0], cP = c[1], cD = c[2];
    const T m = on ? (T)1 : (T)0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const T x1 = mu1[(int64_t)d * ldmu + col] * m;
      const T x2 = mu2[(int64_t)d * ldmu + col] * m;
      a1[d] += cP * x1;
      a2[d] += cS * x2;
      a3[d] += cP * x2;
      a4[d] += cD * x2;
    }
  });
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    a1[d] = wave_sum(a1[d]); a2[d] = wave_sum(a2[d]); a3[d] = wave_sum(a3[d]); a4[d] = wave_sum(a4[d]);
  }
  if (lane == 0) {
    const int tp = tgt_pos[row];
    const T s = (T)INV4PI_D;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const T* f = fmm + (int64_t)d * 4 * N;
      const T y1 = f[tp] * s + a1[d];
      const T y2 = f[N + tp] * s + a2[d];
      const T y3 = f[2 * N + tp] * s + a3[d];
      const T y4 = f[3 * N + tp] * s + a4[d];
      out[(int64_t)d * N + row] = -(T)0.25 * tau[(int64_t)d * N + row] + y1 - y4 - (T)2 * H[row] * y3;
      y2buf[(int64_t)d * N + row] = y2;
    }
  }
}

template <typename T>
void launch_combine_a3b(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch,
                        const T* vals3, const T* tau, const T* mu1, const T* mu2, int64_t ldmu, const T* fmm,
                        const int* tgt_pos, const T* H, const double* w, int nsurf, const int64_t* node_off,
                        const int* node_surf, const double* inv_area, T* out, T* y2buf, double* scal,
                        hipStream_t st) {
  const int nblk = (int)((N + 3) / 4);
  for (int d0 = 0; d0 < nd; d0 += NDMAX) {
    int ndc = nd - d0 < NDMAX ? nd - d0 : NDMAX;
    ND_DISPATCH(k_combine_a3b, ndc, dim3(nblk), dim3(256), 0, st, N, n_p, row_ptr, patch, vals3,
                tau + (int64_t)d0 * N, mu1 + (int64_t)d0 * ldmu, mu2 + (int64_t)d0 * ldmu, ldmu,
                fmm + (int64_t)d0 * 4 * N, tgt_pos, H, out + (int64_t)d0 * N, y2buf + (int64_t)d0 * N)
    KCHECK();
  }
  // W S[S tau] per surface: scal[d][q] = sum_{i in q} w_i y2_i / area_q
  launch_seg_dot<T>(nd, nsurf, N, node_off, y2buf, w, inv_area, scal, st);
  launch_seg_axpy<T>(nd, nsurf, N, node_surf, out, 1.0, nullptr, scal, out, st);
}

// ---------------------------------------------------------------------------
// A2 (Section 4.2): strengths in the layouts of the two FMM calls, and the
// corrections fused with the combination steps
// ---------------------------------------------------------------------------
// pass 1: from c [nd][No] (w^over P tau, tree order) the FMM_A3B strengths
// (charges 0 and c; its dipole c nu is formed from the tree's normals)
// [nd][2][No] and the FMM_ADJ strengths (no charge, dipole vector c nu)
// [nd][4][No]
template <typename T>
__global__ void k_a2_str1(int nd, int64_t No, const T* __restrict__ c, const T* __restrict__ nx,
                          const T* __restrict__ ny, const T* __restrict__ nz, T* __restrict__ s3, T* __restrict__ sd) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= No) return;
  const T a = nx[m], b = ny[m], e = nz[m];
  for (int d = 0; d < nd; ++d) {
    const T v = c[(int64_t)d * No + m];
    s3[(int64_t)(2 * d) * No + m] = 0;
    s3[(int64_t)(2 * d + 1) * No + m] = v;
    sd[(int64_t)(4 * d) * No + m] = 0;
    sd[(int64_t)(4 * d + 1) * No + m] = v * a;
    sd[(int64_t)(4 * d + 2) * No + m] = v * b;
    sd[(int64_t)(4 * d + 3) * No + m] = v * e;
  }
}

// pass 2: charge c2 and dipole vector c1 nu, [nd][4][No], from c1 and c2
// [nd][No] (c1 = w^over P mu1, c2 = w^over P mu2)
template <typename T>
__global__ void k_a2_str2(int nd, int64_t No, const T* __restrict__ c1, const T* __restrict__ c2,
                          const T* __restrict__ nx, const T* __restrict__ ny, const T* __restrict__ nz,
                          T* __restrict__ sd) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= No) return;
  const T a = nx[m], b = ny[m], e = nz[m];
  for (int d = 0; d < nd; ++d) {
    const T v1 = c1[(int64_t)d * No + m], v2 = c2[(int64_t)d * No + m];
    sd[(int64_t)(4 * d) * No + m] = v2;
    sd[(int64_t)(4 * d + 1) * No + m] = v1 * a;
    sd[(int64_t)(4 * d + 2) * No + m] = v1 * b;
    sd[(int64_t)(4 * d + 3) * No + m] = v1 * e;
  }
}

template <typename T>
void launch_a2_str1(int nd, int64_t No, const T* c, const T* nx, const T* ny, const T* nz, T* s3, T* sd,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_a2_str1<T>, dim3((unsigned)((No + 255) / 256)), dim3(256), 0, st, nd, No, c, nx, ny, nz, s3,
                     sd);
  KCHECK();
}

template <typename T>
void launch_a2_str2(int nd, int64_t No, const T* c1, const T* c2, const T* nx, const T* ny, const T* nz, T* sd,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_a2_str2<T>, dim3((unsigned)((No + 255) / 256)), dim3(256), 0, st, nd, No, c1, c2, nx, ny, nz,
                     sd);
  KCHECK();
}

// A2 step 1, one wave per row: S tau, S' tau, (S''+D') tau from the FMM_A3B
// outputs f3 [nd][4][N] (expansion 2 = charge tau, expansion 3 = dipole
// tau nu) and D tau from the FMM_ADJ output fd [nd][N], plus the
// corrections (vals3: S, S', S''+D'; valsD: D);
// mu1 = D tau, mu2 = -(S''+D') tau - 2 H S' tau, y = S tau (the W S tau
// term is added to mu2 per surface afterwards)
template <typename T, int ND>
__global__ __launch_bounds__(256) void k_combine_a2a(int64_t N, int n_p, const int64_t* __restrict__ row_ptr,
                                                     const int* __restrict__ patch, const T* __restrict__ vals3,
                                                     const T* __restrict__ valsD, const T* __restrict__ tau,
                                                     const T* __restrict__ f3, const T* __restrict__ fd,
                                                     const int* __restrict__ tgt_pos, const T* __restrict__ H,
                                                     T* mu1, T* mu2, T* y) {
  __shared__ int pat_s[4][64];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * 4 + wv;
  if (row >= N) return;
  T aS[ND], aP[ND], aK[ND], aD[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) { aS[d] = aP[d] = aK[d] = aD[d] = 0; }
  row_blocks(row_ptr[row], row_ptr[row + 1], n_p, lane, patch, pat_s[wv], [&](int64_t e, int64_t col, bool on) {
    const T* c = vals3 + e * 3;
    const T cS = c[0], cP = c[1], cK = c[2], cD = valsD[e];
    const T m = on ? (T)1 : (T)0;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const T x = tau[(int64_t)d * N + col] * m;
      aS[d] += cS * x;
      aP[d] += cP * x;
      aK[d] += cK * x;
      aD[d] += cD * x;
    }
  });
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    aS[d] = wave_sum(aS[d]); aP[d] = wave_sum(aP[d]); aK[d] = wave_sum(aK[d]); aD[d] = wave_sum(aD[d]);
  }
  if (lane == 0) {
    const int tp = tgt_pos[row];
    const T s = (T)INV4PI_D;
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      const T* f = f3 + (int64_t)d * 4 * N;
      const T vS = f[N + tp] * s + aS[d];
      const T vP = f[2 * N + tp] * s + aP[d];
      const T vK = f[3 * N + tp] * s + aK[d];
      const T vD = fd[(int64_t)d * N + tp] * s + aD[d];
      mu1[(int64_t)d * N + row] = vD;
      mu2[(int64_t)d * N + row] = -vK - (T)2 * H[row] * vP;
      y[(int64_t)d * N + row] = vS;
    }
  }
}

// A2 step 2: out = -tau/4 + S mu2 + D mu1 (D mu1 = D D tau) from the FMM_ADJ
// output fb [nd][N] (charge mu2, dipole vector mu1 nu) and the corrections
template <typename T, int ND>
__global__ __launch_bounds__(256) void k_combine_a2b(int64_t N, int n_p, const int64_t* __restrict__ row_ptr,
                                                     const int* __restrict__ patch, const T* __restrict__ vals3,
                                                     const T* __restrict__ valsD, const T* __restrict__ tau,
                                                     const T* __restrict__ mu1, const T* __restrict__ mu2,
                                                     const T* __restrict__ fb, const int* __restrict__ tgt_pos,
                                                     T* out) {
  __shared__ int pat_s[4][64];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t row = (int64_t)blockIdx.x * 4 + wv;
  if (row >= N) return;
  T a[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) a[d] = 0;
  row_blocks(row_ptr[row], row_ptr[row + 1], n_p, lane, patch, pat_s[wv], [&](int64_t e, int64_t col, bool on) {
    const T cS = vals3[e * 3], cD = valsD[e];
    const T m = on ? (T)1 : (T)0;
#pragma unroll
    for (int d = 0; d < ND; ++d)
      a[d] += (cS * mu2[(int64_t)d * N + col] + cD * mu1[(int64_t)d * N + col]) * m;
  });
#pragma unroll
  for (int d = 0; d < ND; ++d) a[d] = wave_sum(a[d]);
  if (lane == 0) {
    const int tp = tgt_pos[row];
    const T s = (T)INV4PI_D;
#pragma unroll
    for (int d = 0; d < ND; ++d)
      out[(int64_t)d * N + row] = -(T)0.25 * tau[(int64_t)d * N + row] + fb[(int64_t)d * N + tp] * s + a[d];
  }
}

template <typename T>
void launch_combine_a2a(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch, const T* vals3,
                        const T* valsD, const T* tau, const T* f3, const T* fd, const int* tgt_pos, const T* H,
                        T* mu1, T* mu2, T* y, hipStream_t st) {
  for (int d0 = 0; d0 < nd; d0 += NDMAX) {
    int ndc = nd - d0 < NDMAX ? nd - d0 : NDMAX;
    ND_DISPATCH(k_combine_a2a, ndc, dim3((N + 3) / 4), dim3(256), 0, st, N, n_p, row_ptr, patch, vals3, valsD,
                tau + (int64_t)d0 * N, f3 + (int64_t)d0 * 4 * N, fd + (int64_t)d0 * N, tgt_pos, H,
                mu1 + (int64_t)d0 * N, mu2 + (int64_t)d0 * N, y + (int64_t)d0 * N)
    KCHECK();
  }
}

template <typename T>
void launch_combine_a2b(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch, const T* vals3,
                        const T* valsD, const T* tau, const T* mu1, const T* mu2, const T* fb, const int* tgt_pos,
                        T* out, hipStream_t st) {
  for (int d0 = 0; d0 < nd; d0 += NDMAX) {
    int ndc = nd - d0 < NDMAX ? nd - d0 : NDMAX;
    ND_DISPATCH(k_combine_a2b, ndc, dim3((N + 3) / 4), dim3(256), 0, st, N, n_p, row_ptr, patch, vals3, valsD,
                tau + (int64_t)d0 * N, mu1 + (int64_t)d0 * N, mu2 + (int64_t)d0 * N, fb + (int64_t)d0 * N, tgt_pos,
                out + (int64_t)d0 * N)
    KCHECK();
  }
}

// ---------------------------------------------------------------------------
// adjoint applies (transposed far sum through the FMM on the transposed tree,
// transposed corrections, transposed oversampling)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_adj_strengths(int nd, int64_t N, const T* __restrict__ gpot, const T* __restrict__ ggrad,
                                const T* __restrict__ gdSdn, const T* __restrict__ gsurf, const T* __restrict__ nrm,
                                const int* __restrict__ src_pos, T* __restrict__ str, T* __restrict__ g4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const T n0 = nrm[3 * i], n1 = nrm[3 * i + 1], n2 = nrm[3 * i + 2];
  const int64_t pos = src_pos[i];
  for (int d = 0; d < nd; ++d) {
    const int64_t r = (int64_t)d * N + i;
    const T q = gpot ? gpot[r] : (T)0;
    T v0 = 0, v1 = 0, v2 = 0;
    if (ggrad) { v0 += ggrad[3 * r]; v1 += ggrad[3 * r + 1]; v2 += ggrad[3 * r + 2]; }
    if (gdSdn) { const T g = gdSdn[r]; v0 += n0 * g; v1 += n1 * g; v2 += n2 * g; }
    if (gsurf) {
      const T s0 = gsurf[3 * r], s1 = gsurf[3 * r + 1], s2 = gsurf[3 * r + 2];
      const T ns = n0 * s0 + n1 * s1 + n2 * s2;
      v0 += s0 - n0 * ns; v1 += s1 - n1 * ns; v2 += s2 - n2 * ns;
    }
    str[(int64_t)(4 * d) * N + pos] = q;
    str[(int64_t)(4 * d + 1) * N + pos] = v0;
    str[(int64_t)(4 * d + 2) * N + pos] = v1;
    str[(int64_t)(4 * d + 3) * N + pos] = v2;
    g4[4 * r] = q; g4[4 * r + 1] = v0; g4[4 * r + 2] = v1; g4[4 * r + 3] = v2;
  }
}

template <typename T>
void launch_adj_strengths(int nd, int64_t N, const T* gpot, const T* ggrad, const T* gdSdn, const T* gsurf,
                          const T* nrm, const int* src_pos, T* str, T* g4, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_strengths<T>, dim3((N + 255) / 256), dim3(256), 0, st, nd, N, gpot, ggrad, gdSdn, gsurf,
                     nrm, src_pos, str, g4);
  KCHECK();
}

// One wave per (patch, density): node k of the patch is lane k % SW (SW = 32
// for n_p <= 32, else 64); the two half-waves (n_p <= 32) split the
// oversampled points and the correction entries and are added at the end.
template <typename T>
__global__ __launch_bounds__(64) void k_adj_combine(int NP, int n_p, int n_o, int64_t N, int64_t No,
                                                    const T* __restrict__ P, const T* __restrict__ wo,
                                                    const T* __restrict__ psi, const int* __restrict__ tgt_pos,
                                                    const int64_t* __restrict__ cptr, const int* __restrict__ crow,
                                                    const int64_t* __restrict__ cblk, const T* __restrict__ vals4,
                                                    const T* __restrict__ g4, T* __restrict__ sbar) {
  typedef typename Vec4<T>::type T4;
  const int l = blockIdx.x, d = blockIdx.y;
  const int lane = threadIdx.x;
  const int SW = n_p <= 32 ? 32 : 64, nsub = 64 / SW;
  const int sub = lane / SW, k0 = lane - sub * SW;
  const T4* v4 = reinterpret_cast<const T4*>(vals4);
  const T4* gq = reinterpret_cast<const T4*>(g4) + (int64_t)d * N;
  const T* ps = psi + (int64_t)d * No;
  for (int k = k0; k < n_p; k += SW) {  // n_p > 64 needs several passes
    T far = 0, corr = 0;
    for (int m = sub; m < n_o; m += nsub) {
      const int64_t om = (int64_t)l * n_o + m;
      far += P[(int64_t)m * n_p + k] * wo[om] * ps[tgt_pos[om]];
    }
    for (int64_t e = cptr[l] + sub; e < cptr[l + 1]; e += nsub) {
      const T4 c = v4[cblk[e] * n_p + k];
      const T4 g = gq[crow[e]];
      corr += c.x * g.x + c.y * g.y + c.z * g.z + c.w * g.w;
    }
    T tot = far * (T)INV4PI_D + corr;
    if (nsub == 2) tot += __shfl_xor(tot, 32, 64);
    if (sub == 0) sbar[(int64_t)d * N + (int64_t)l * n_p + k] = tot;
  }
}

template <typename T>
void launch_adj_combine(int nd, int NP, int n_p, int n_o, int64_t N, int64_t No, const T* P, const T* wo,
                        const T* psi, const int* tgt_pos, const int64_t* cptr, const int* crow,
                        const int64_t* cblk, const T* vals4, const T* g4, T* sigma_bar, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_combine<T>, dim3(NP, nd), dim3(64), 0, st, NP, n_p, n_o, N, No, P, wo, psi, tgt_pos,
                     cptr, crow, cblk, vals4, g4, sigma_bar);
  KCHECK();
}

// ---- kernel-position derivative of S (see kernels.hpp) ----
template <typename T>
__global__ void k_scatter_perm(int64_t n, const T* __restrict__ in, const int* __restrict__ pos,
                               T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t d = blockIdx.y;
  out[d * n + pos[i]] = in[d * n + i];
}

template <typename T>
void launch_scatter_perm(int nd, int64_t n, const T* in, const int* pos, T* out, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_perm<T>, dim3((unsigned)((n + 255) / 256), nd), dim3(256), 0, st, n, in, pos, out);
  KCHECK();
}

// One 64-thread block per patch: the source part c_m grad psi(s_m) of the
// patch's oversampled points goes to LDS (summed over the densities), then
// node k of the patch adds gbar grad phi at the node and sum_m P_mk of it.
template <typename T>
__global__ __launch_bounds__(64) void k_xbar_S(int nd, int n_p, int n_o, int64_t N, int64_t No,
                                               const T* __restrict__ P, const T* __restrict__ str,
                                               const int* __restrict__ src_pos, const T* __restrict__ gphi,
                                               const int* __restrict__ tgt_pos, const T* __restrict__ gbar,
                                               const T* __restrict__ gpsi, const int* __restrict__ atgt_pos,
                                               T* __restrict__ xbar) {
  extern __shared__ unsigned char smraw[];
  double* sb = reinterpret_cast<double*>(smraw);  // [n_o][3]
  const int64_t l = blockIdx.x;
  for (int m = threadIdx.x; m < n_o; m += blockDim.x) {
    const int64_t om = l * n_o + m;
    const int64_t sp = src_pos[om], ap = atgt_pos[om];
    double a0 = 0, a1 = 0, a2 = 0;
    for (int d = 0; d < nd; ++d) {
      const double c = (double)str[(int64_t)d * No + sp];
      const T* g = gpsi + (int64_t)d * 4 * No;
      a0 += c * (double)g[No + ap];
      a1 += c * (double)g[2 * No + ap];
      a2 += c * (double)g[3 * No + ap];
    }
    sb[3 * m] = a0;
    sb[3 * m + 1] = a1;
    sb[3 * m + 2] = a2;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < n_p; k += blockDim.x) {
    const int64_t j = l * n_p + k;
    const int64_t tp = tgt_pos[j];
    double x0 = 0, x1 = 0, x2 = 0;
    for (int d = 0; d < nd; ++d) {
      const double gb = (double)gbar[(int64_t)d * N + j];
      const T* g = gphi + (int64_t)d * 4 * N;
      x0 += gb * (double)g[N + tp];
      x1 += gb * (double)g[2 * N + tp];
      x2 += gb * (double)g[3 * N + tp];
    }
    for (int m = 0; m < n_o; ++m) {
      const double pm = (double)P[(int64_t)m * n_p + k];
      x0 += pm * sb[3 * m];
      x1 += pm * sb[3 * m + 1];
      x2 += pm * sb[3 * m + 2];
    }
    xbar[3 * j] += (T)(x0 * INV4PI_D);
    xbar[3 * j + 1] += (T)(x1 * INV4PI_D);
    xbar[3 * j + 2] += (T)(x2 * INV4PI_D);
  }
}

template <typename T>
void launch_xbar_S(int nd, int NP, int n_p, int n_o, int64_t N, int64_t No, const T* P, const T* str,
                   const int* src_pos, const T* gphi, const int* tgt_pos, const T* gbar, const T* gpsi,
                   const int* atgt_pos, T* xbar, hipStream_t st) {
  hipLaunchKernelGGL(k_xbar_S<T>, dim3(NP), dim3(64), sizeof(double) * 3 * n_o, st, nd, n_p, n_o, N, No, P, str,
                     src_pos, gphi, tgt_pos, gbar, gpsi, atgt_pos, xbar);
  KCHECK();
}

// ---- transposed A3 (see kernels.hpp) ----
template <typename T>
__global__ void k_adj3_str1(int nd, int64_t N, const T* __restrict__ v, const T* __restrict__ H,
                            const int* __restrict__ src_pos, T* __restrict__ str, T* __restrict__ g2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t pos = src_pos[i];
  for (int d = 0; d < nd; ++d) {
    const T x = v[(int64_t)d * N + i];
    const T w = (T)2 * H[i] * x;
    str[(int64_t)(2 * d) * N + pos] = x;
    str[(int64_t)(2 * d + 1) * N + pos] = w;
    g2[2 * ((int64_t)d * N + i)] = x;
    g2[2 * ((int64_t)d * N + i) + 1] = w;
  }
}

template <typename T>
__global__ void k_adj3_str2(int nd, int64_t N, const T* __restrict__ a, const T* __restrict__ b,
                            const T* __restrict__ nrm, const int* __restrict__ src_pos, T* __restrict__ str,
                            T* __restrict__ g2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t pos = src_pos[i];
  for (int d = 0; d < nd; ++d) {
    const T x = a[(int64_t)d * N + i], y = b[(int64_t)d * N + i];
    str[(int64_t)(4 * d) * N + pos] = -y;
    str[(int64_t)(4 * d + 1) * N + pos] = x * nrm[3 * i];
    str[(int64_t)(4 * d + 2) * N + pos] = x * nrm[3 * i + 1];
    str[(int64_t)(4 * d + 3) * N + pos] = x * nrm[3 * i + 2];
    g2[2 * ((int64_t)d * N + i)] = x;
    g2[2 * ((int64_t)d * N + i) + 1] = y;
  }
}

// one wave per (patch, density), as k_adj_combine; STEP 1 writes a and b,
// STEP 2 the transposed A3
template <typename T, int STEP>
__global__ __launch_bounds__(64) void k_adj3_comb(int NP, int n_p, int n_o, int64_t N, int64_t No,
                                                  const T* __restrict__ P, const T* __restrict__ wo,
                                                  const T* __restrict__ psi, const int* __restrict__ tgt_pos,
                                                  const int64_t* __restrict__ cptr, const int* __restrict__ crow,
                                                  const int64_t* __restrict__ cblk, const T* __restrict__ vals3,
                                                  const T* __restrict__ g2, const T* __restrict__ v,
                                                  const T* __restrict__ z, const double* __restrict__ scal,
                                                  int nsurf, const int* __restrict__ node_surf,
                                                  T* __restrict__ o1, T* __restrict__ o2) {
  const int l = blockIdx.x, d = blockIdx.y;
  const int lane = threadIdx.x;
  const int SW = n_p <= 32 ? 32 : 64, nsub = 64 / SW;
  const int sub = lane / SW, k0 = lane - sub * SW;
  const int nps = STEP == 1 ? 2 : 1;  // far outputs per density
  const T* gq = g2 + (int64_t)d * N * 2;
  for (int k = k0; k < n_p; k += SW) {
    T f1 = 0, f2 = 0, c1 = 0, c2 = 0;
    for (int m = sub; m < n_o; m += nsub) {
      const int64_t om = (int64_t)l * n_o + m;
      const T pw = P[(int64_t)m * n_p + k] * wo[om];
      const int64_t tp = tgt_pos[om];
      f1 += pw * psi[((int64_t)d * nps) * No + tp];
      if (STEP == 1) f2 += pw * psi[((int64_t)d * nps + 1) * No + tp];
    }
    for (int64_t e = cptr[l] + sub; e < cptr[l + 1]; e += nsub) {
      const T* c = vals3 + (cblk[e] * n_p + k) * 3;  // S, S', S''+D'
      const T x = gq[2 * (int64_t)crow[e]], y = gq[2 * (int64_t)crow[e] + 1];
      if (STEP == 1) {
        c1 += c[1] * x;
        c2 += c[2] * x + c[1] * y;
      } else {
        c1 += c[1] * x - c[0] * y;
      }
    }
    T t1 = f1 * (T)INV4PI_D + c1, t2 = f2 * (T)INV4PI_D + c2;
    if (nsub == 2) {
      t1 += __shfl_xor(t1, 32, 64);
      if (STEP == 1) t2 += __shfl_xor(t2, 32, 64);
    }
    if (sub == 0) {
      const int64_t r = (int64_t)d * N + (int64_t)l * n_p + k;
      if (STEP == 1) {
        o1[r] = t1;
        o2[r] = t2;
      } else {
        const int64_t i = (int64_t)l * n_p + k;
        o1[r] = -(T)0.25 * v[r] + t1 + (T)scal[(int64_t)d * nsurf + node_surf[i]] * z[i];
      }
    }
  }
}

template <typename T>
void launch_adj3_str1(int nd, int64_t N, const T* v, const T* H, const int* src_pos, T* str, T* g2,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_adj3_str1<T>, dim3((N + 255) / 256), dim3(256), 0, st, nd, N, v, H, src_pos, str, g2);
  KCHECK();
}
template <typename T>
void launch_adj3_str2(int nd, int64_t N, const T* a, const T* b, const T* nrm, const int* src_pos, T* str, T* g2,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_adj3_str2<T>, dim3((N + 255) / 256), dim3(256), 0, st, nd, N, a, b, nrm, src_pos, str, g2);
  KCHECK();
}
template <typename T>
void launch_adj3_comb1(int nd, int NP, int n_p, int n_o, int64_t N, int64_t No, const T* P, const T* wo,
                       const T* psi, const int* tgt_pos, const int64_t* cptr, const int* crow, const int64_t* cblk,
                       const T* vals3, const T* g2, T* a, T* b, hipStream_t st) {
  hipLaunchKernelGGL((k_adj3_comb<T, 1>), dim3(NP, nd), dim3(64), 0, st, NP, n_p, n_o, N, No, P, wo, psi, tgt_pos,
                     cptr, crow, cblk, vals3, g2, (const T*)nullptr, (const T*)nullptr, (const double*)nullptr, 0,
                     (const int*)nullptr, a, b);
  KCHECK();
}
template <typename T>
void launch_adj3_comb2(int nd, int NP, int n_p, int n_o, int64_t N, int64_t No, const T* P, const T* wo,
                       const T* psi, const int* tgt_pos, const int64_t* cptr, const int* crow, const int64_t* cblk,
                       const T* vals3, const T* g2, const T* v, const T* z, const double* scal, int nsurf,
                       const int* node_surf, T* out, hipStream_t st) {
  hipLaunchKernelGGL((k_adj3_comb<T, 2>), dim3(NP, nd), dim3(64), 0, st, NP, n_p, n_o, N, No, P, wo, psi, tgt_pos,
                     cptr, crow, cblk, vals3, g2, v, z, scal, nsurf, node_surf, out, (T*)nullptr);
  KCHECK();
}

// ---------------------------------------------------------------------------
// FP64 vector helpers
// ---------------------------------------------------------------------------
constexpr int DOT_BLOCKS = 256;

__global__ void k_dots_partial(const double* V, int64_t ldv, int k, const double* w, int64_t N, double* partial) {
  __shared__ double red[256];
  const int j = blockIdx.y;
  const double* vj = V + (int64_t)j * ldv;
  double a = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) a += vj[i] * w[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = red[0];
}

__global__ void k_dots_final(const double* partial, int nb, double* out) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double a = 0;
  for (int b = threadIdx.x; b < nb; b += 256) a += partial[(int64_t)j * nb + b];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

void launch_dots(const double* V, int64_t ldv, int k, const double* w, int64_t N, double* out,
                 double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_dots_partial, dim3(DOT_BLOCKS, k), dim3(256), 0, st, V, ldv, k, w, N, partial);
  KCHECK();
  hipLaunchKernelGGL(k_dots_final, dim3(k), dim3(256), 0, st, partial, DOT_BLOCKS, out);
  KCHECK();
}

__global__ void k_gemv_sub(const double* V, int64_t ldv, int k, const double* h, double* w, int64_t N, double sign) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double a = 0;
  for (int j = 0; j < k; ++j) a += h[j] * V[(int64_t)j * ldv + i];
  w[i] += sign * a;
}

void launch_gemv_sub(const double* V, int64_t ldv, int k, const double* h, double* w, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_gemv_sub, dim3((N + 255) / 256), dim3(256), 0, st, V, ldv, k, h, w, N, -1.0);
  KCHECK();
}
void launch_gemv_add(const double* V, int64_t ldv, int k, const double* y, double* x, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_gemv_sub, dim3((N + 255) / 256), dim3(256), 0, st, V, ldv, k, y, x, N, 1.0);
  KCHECK();
}

__global__ void k_scale_copy(const double* w, double a, double* v, int64_t N) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) v[i] = a * w[i];
}
void launch_scale_copy(const double* w, double a, double* v, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_copy, dim3((N + 255) / 256), dim3(256), 0, st, w, a, v, N);
  KCHECK();
}

__global__ void k_axpby(double a, const double* x, double b, const double* y, double* z, int64_t N) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) z[i] = a * x[i] + b * y[i];
}
void launch_axpby(double a, const double* x, double b, const double* y, double* z, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3((N + 255) / 256), dim3(256), 0, st, a, x, b, y, z, N);
  KCHECK();
}

template <typename A, typename B>
__global__ void k_convert(const A* x, B* y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (B)x[i];
}
template <typename A, typename B>
void launch_convert(const A* x, B* y, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<A, B>), dim3((n + 255) / 256), dim3(256), 0, st, x, y, n);
  KCHECK();
}

__global__ void k_wmean_partial(const double* f, const double* w, int64_t N, double* partial) {
  __shared__ double red[256];
  double a = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) a += w[i] * f[i];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}
void launch_wmean(const double* f, const double* w, int64_t N, double* partial, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_wmean_partial, dim3(DOT_BLOCKS), dim3(256), 0, st, f, w, N, partial);
  KCHECK();
  hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(256), 0, st, partial, DOT_BLOCKS, out);
  KCHECK();
}

__global__ void k_sub_scalar(double* f, const double* s, double scale, int64_t N) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) f[i] -= scale * s[0];
}
void launch_sub_scalar(double* f, const double* s, double scale, int64_t N, hipStream_t st) {
  hipLaunchKernelGGL(k_sub_scalar, dim3((N + 255) / 256), dim3(256), 0, st, f, s, scale, N);
  KCHECK();
}

// ---- several GMRES systems at once (FP64).  System a owns the segment
// [xoff[a], xoff[a] + len[a]) of the operator's vectors and the basis
// vectors V + vbase[a] + j len[a], j = 0, 1, ...
constexpr int MSYS_BLOCKS = 32;

// win = basis vector j of every system in `act` order (all segments of win
// belong to some system; those of inactive systems are zeroed)
__global__ void k_msys_gather(int nsys, const int64_t* __restrict__ xoff, const int64_t* __restrict__ len,
                              const int64_t* __restrict__ vbase, const int* __restrict__ active, int j,
                              const double* __restrict__ V, double* __restrict__ win) {
  const int a = blockIdx.y;
  const int64_t n = len[a], o = xoff[a];
  const double* v = V + vbase[a] + (int64_t)j * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    win[o + t] = active[a] ? v[t] : 0.0;
}

// partial[(a k + jj) MB + bx] = sum over this block's share of V_jj(a) . w(a)
// (V_jj = w itself when vbase is null: the squared norm, k = 1)
__global__ void k_msys_dots_partial(int k, const int64_t* __restrict__ xoff, const int64_t* __restrict__ len,
                                    const int64_t* __restrict__ vbase, const double* __restrict__ V,
                                    const double* __restrict__ W, double* __restrict__ partial) {
  __shared__ double red[256];
  const int jj = blockIdx.y, a = blockIdx.z;
  const int64_t n = len[a];
  const double* w = W + xoff[a];
  const double* v = vbase ? V + vbase[a] + (int64_t)jj * n : w;
  double acc = 0;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)MSYS_BLOCKS * 256) acc += v[t] * w[t];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[((int64_t)a * k + jj) * MSYS_BLOCKS + blockIdx.x] = red[0];
}
__global__ void k_msys_dots_final(const double* __restrict__ partial, int count, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double acc = 0;
  for (int b = 0; b < MSYS_BLOCKS; ++b) acc += partial[(int64_t)i * MSYS_BLOCKS + b];
  out[i] = acc;
}

// w(a) += sign sum_jj h[a k + jj] V_jj(a)
__global__ void k_msys_gemv(int k, const int64_t* __restrict__ xoff, const int64_t* __restrict__ len,
                            const int64_t* __restrict__ vbase, const double* __restrict__ V,
                            const double* __restrict__ h, double sign, double* __restrict__ W) {
  const int a = blockIdx.y;
  const int64_t n = len[a];
  const double* v = V + vbase[a];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0;
    for (int jj = 0; jj < k; ++jj) acc += h[(int64_t)a * k + jj] * v[(int64_t)jj * n + t];
    W[xoff[a] + t] += sign * acc;
  }
}

// V_j(a) = s[a] w(a)
__global__ void k_msys_scale_copy(int j, const int64_t* __restrict__ xoff, const int64_t* __restrict__ len,
                                  const int64_t* __restrict__ vbase, const double* __restrict__ sc,
                                  const double* __restrict__ W, double* __restrict__ V) {
  const int a = blockIdx.y;
  const int64_t n = len[a];
  double* v = V + vbase[a] + (int64_t)j * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    v[t] = sc[a] * W[xoff[a] + t];
}

static inline int msys_grid_x(int64_t maxlen) {
  const int64_t b = (maxlen + 255) / 256;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 1024));
}

void launch_msys_gather(int nsys, int64_t maxlen, const int64_t* xoff, const int64_t* len, const int64_t* vbase,
                        const int* active, int j, const double* V, double* win, hipStream_t st) {
  hipLaunchKernelGGL(k_msys_gather, dim3(msys_grid_x(maxlen), nsys), dim3(256), 0, st, nsys, xoff, len, vbase, active,
                     j, V, win);
  KCHECK();
}
void launch_msys_dots(int nsys, int k, const int64_t* xoff, const int64_t* len, const int64_t* vbase,
                      const double* V, const double* W, double* partial, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_msys_dots_partial, dim3(MSYS_BLOCKS, k, nsys), dim3(256), 0, st, k, xoff, len, vbase, V, W,
                     partial);
  KCHECK();
  const int cnt = nsys * k;
  hipLaunchKernelGGL(k_msys_dots_final, dim3((cnt + 255) / 256), dim3(256), 0, st, partial, cnt, out);
  KCHECK();
}
void launch_msys_gemv(int nsys, int64_t maxlen, int k, const int64_t* xoff, const int64_t* len, const int64_t* vbase,
                      const double* V, const double* h, double sign, double* W, hipStream_t st) {
  hipLaunchKernelGGL(k_msys_gemv, dim3(msys_grid_x(maxlen), nsys), dim3(256), 0, st, k, xoff, len, vbase, V, h, sign,
                     W);
  KCHECK();
}
void launch_msys_scale_copy(int nsys, int64_t maxlen, int j, const int64_t* xoff, const int64_t* len,
                            const int64_t* vbase, const double* sc, const double* W, double* V, hipStream_t st) {
  hipLaunchKernelGGL(k_msys_scale_copy, dim3(msys_grid_x(maxlen), nsys), dim3(256), 0, st, j, xoff, len, vbase, sc,
                     W, V);
  KCHECK();
}

// ---- GMRES iterations driven on the device (Section 6) -------------------
// Every kernel reads the iteration number j from gm.iter, so one captured
// graph of an iteration (gather, operator, CGS2, Givens, next basis vector)
// is replayed for every j.  Systems that have stopped (gm.active[a] = 0)
// are skipped by every kernel; their segments of the operator input are 0.

// win(a) = V_j(a) for active systems, 0 otherwise
__global__ void k_gm_gather(GmresDev gm, const double* __restrict__ V, double* __restrict__ win) {
  const int a = blockIdx.y;
  const int j = *gm.iter;
  const int64_t n = gm.len[a], o = gm.xoff[a];
  const bool act = gm.active[a] != 0;
  const double* v = V + gm.vbase[a] + (int64_t)j * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    win[o + t] = act ? v[t] : 0.0;
}

// part[(a KM + jj) MB + bx] = this block's share of V_jj(a) . w(a) for
// jj <= j (basis), or of w(a) . w(a) (norm, jj = 0); active systems only
// unless `all`
__global__ void k_gm_dots_partial(GmresDev gm, int basis, int all, const double* __restrict__ V,
                                  const double* __restrict__ W, double* __restrict__ part) {
  __shared__ double red[256];
  const int a = blockIdx.y;
  if (!all && !gm.active[a]) return;
  const int k = basis ? *gm.iter + 1 : 1;
  const int64_t n = gm.len[a];
  const double* w = W + gm.xoff[a];
  for (int jj = 0; jj < k; ++jj) {
    const double* v = basis ? V + gm.vbase[a] + (int64_t)jj * n : w;
    double acc = 0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)MSYS_BLOCKS * 256)
      acc += v[t] * w[t];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[((int64_t)a * gm.km + jj) * MSYS_BLOCKS + blockIdx.x] = red[0];
    __syncthreads();
  }
}
// sum of the partial sums (fixed order): out[a KM + jj] (basis) or out[a]
// (norm)
__global__ void k_gm_dots_final(GmresDev gm, int basis, int all, const double* __restrict__ part,
                                double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)gm.ns * gm.km) return;
  const int a = (int)(i / gm.km), jj = (int)(i % gm.km);
  const int k = basis ? *gm.iter + 1 : 1;
  if ((!all && !gm.active[a]) || jj >= k) return;
  double acc = 0;
  for (int b = 0; b < MSYS_BLOCKS; ++b) acc += part[i * MSYS_BLOCKS + b];
  out[basis ? i : a] = acc;
}

// w(a) -= sum_{jj <= j} h[a KM + jj] V_jj(a), active systems
__global__ void k_gm_gemv_sub(GmresDev gm, const double* __restrict__ V, const double* __restrict__ h,
                              double* __restrict__ W) {
  const int a = blockIdx.y;
  if (!gm.active[a]) return;
  const int k = *gm.iter + 1;
  const int64_t n = gm.len[a];
  const double* v = V + gm.vbase[a];
  const double* ha = h + (int64_t)a * gm.km;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0;
    for (int jj = 0; jj < k; ++jj) acc += ha[jj] * v[(int64_t)jj * n + t];
    W[gm.xoff[a] + t] -= acc;
  }
}

// start: beta = |b(a)|, g_0 = beta, the first basis vector's scale, the
// iteration counter and the number of active systems (one block)
__global__ void k_gm_init(GmresDev gm, const int* __restrict__ skip) {
  __shared__ int cnt[256];
  int c = 0;
  for (int a = threadIdx.x; a < gm.ns; a += blockDim.x) {
    const double beta = sqrt(gm.nr[a]);
    const bool act = !skip[a] && beta > 0.0;
    gm.beta[a] = beta;
    gm.g[(int64_t)a * gm.km] = beta;
    gm.sc[a] = act ? 1.0 / beta : 0.0;
    gm.active[a] = act ? 1 : 0;
    gm.kdone[a] = 0;
    gm.relres[a] = act ? 1.0 : 0.0;
    c += act ? 1 : 0;
  }
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) cnt[threadIdx.x] += cnt[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *gm.iter = 0;
    *gm.nactive = cnt[0];
  }
}

// Givens step of iteration j for every active system (one block): the new
// Hessenberg column h1 + h2 (two Gram-Schmidt passes) and |w|, the earlier
// rotations applied to it, a new rotation, the residual estimate |g_{j+1}| /
// beta, the stopping test (below tol, breakdown or the last iteration), the
// scale of the next basis vector; then j + 1 and the active count.
__global__ void k_gm_givens(GmresDev gm) {
  __shared__ int cnt[256];
  const int j = *gm.iter;
  const int km = gm.km, mi = gm.maxit;
  const double tol = *gm.tol;
  int c = 0;
  for (int a = threadIdx.x; a < gm.ns; a += blockDim.x) {
    if (!gm.active[a]) continue;
    const double* h1 = gm.h1 + (int64_t)a * km;
    const double* h2 = gm.h2 + (int64_t)a * km;
    double* R = gm.R + (int64_t)a * mi * mi;  // R[r * mi + col]
    double* cs = gm.cs + (int64_t)a * mi;
    double* sn = gm.sn + (int64_t)a * mi;
    double* g = gm.g + (int64_t)a * km;
    const double hnrm = sqrt(gm.nr[a]);
    for (int r = 0; r <= j; ++r) R[r * mi + j] = h1[r] + h2[r];
    double below = hnrm;  // entry j + 1 of the column
    for (int r = 0; r < j; ++r) {
      const double x = R[r * mi + j], y = R[(r + 1) * mi + j];
      R[r * mi + j] = cs[r] * x + sn[r] * y;
      R[(r + 1) * mi + j] = -sn[r] * x + cs[r] * y;
    }
    const double x = R[j * mi + j];
    const double den = hypot(x, below);
    cs[j] = x / den;
    sn[j] = below / den;
    R[j * mi + j] = den;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    const double rel = fabs(g[j + 1]) / gm.beta[a];
    gm.relres[a] = rel;
    gm.kdone[a] = j + 1;
    const bool done = rel < tol || hnrm == 0.0 || j + 1 >= mi;
    gm.sc[a] = done ? 0.0 : 1.0 / hnrm;
    gm.active[a] = done ? 0 : 1;
    c += done ? 0 : 1;
  }
  cnt[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) cnt[threadIdx.x] += cnt[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *gm.nactive = cnt[0];
    *gm.iter = j + 1;
  }
}

// V_j(a) = sc[a] w(a) with j = the current counter (after the Givens step:
// the next basis vector), systems with sc[a] != 0
__global__ void k_gm_scale_copy(GmresDev gm, const double* __restrict__ W, double* __restrict__ V) {
  const int a = blockIdx.y;
  const double s = gm.sc[a];
  if (s == 0.0) return;
  const int j = *gm.iter;
  const int64_t n = gm.len[a];
  double* v = V + gm.vbase[a] + (int64_t)j * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    v[t] = s * W[gm.xoff[a] + t];
}

// y = R^{-1} g over the kdone[a] iterations of each system (one thread per
// system), written to h1[a KM + .]
__global__ void k_gm_backsolve(GmresDev gm) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= gm.ns) return;
  const int k = gm.kdone[a], mi = gm.maxit;
  const double* R = gm.R + (int64_t)a * mi * mi;
  const double* g = gm.g + (int64_t)a * gm.km;
  double* y = gm.h1 + (int64_t)a * gm.km;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int c = i + 1; c < k; ++c) s -= R[i * mi + c] * y[c];
    y[i] = s / R[i * mi + i];
  }
}

// x(a) = sum_{jj < kdone[a]} y_jj V_jj(a) (x(a) = 0 when kdone[a] = 0)
__global__ void k_gm_solution(GmresDev gm, const double* __restrict__ V, double* __restrict__ X) {
  const int a = blockIdx.y;
  const int k = gm.kdone[a];
  const int64_t n = gm.len[a];
  const double* v = V + gm.vbase[a];
  const double* y = gm.h1 + (int64_t)a * gm.km;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0;
    for (int jj = 0; jj < k; ++jj) acc += y[jj] * v[(int64_t)jj * n + t];
    X[gm.xoff[a] + t] = acc;
  }
}

void launch_gm_start(const GmresDev& gm, const double* B, const int* skip, double* V, hipStream_t st) {
  const int nf = (int)(((int64_t)gm.ns * gm.km + 255) / 256);
  hipLaunchKernelGGL(k_gm_dots_partial, dim3(MSYS_BLOCKS, gm.ns), dim3(256), 0, st, gm, 0, 1, V, B, gm.part);
  KCHECK();
  hipLaunchKernelGGL(k_gm_dots_final, dim3(nf), dim3(256), 0, st, gm, 0, 1, gm.part, gm.nr);
  KCHECK();
  hipLaunchKernelGGL(k_gm_init, dim3(1), dim3(256), 0, st, gm, skip);
  KCHECK();
  hipLaunchKernelGGL(k_gm_scale_copy, dim3(msys_grid_x(gm.maxlen), gm.ns), dim3(256), 0, st, gm, B, V);
  KCHECK();
}

void launch_gm_gather(const GmresDev& gm, const double* V, double* win, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_gather, dim3(msys_grid_x(gm.maxlen), gm.ns), dim3(256), 0, st, gm, V, win);
  KCHECK();
}

void launch_gm_arnoldi(const GmresDev& gm, double* V, double* W, hipStream_t st) {
  const dim3 gx(msys_grid_x(gm.maxlen), gm.ns), gd(MSYS_BLOCKS, gm.ns);
  const int nf = (int)(((int64_t)gm.ns * gm.km + 255) / 256);
  for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
    double* h = pass == 0 ? gm.h1 : gm.h2;
    hipLaunchKernelGGL(k_gm_dots_partial, gd, dim3(256), 0, st, gm, 1, 0, V, W, gm.part);
    KCHECK();
    hipLaunchKernelGGL(k_gm_dots_final, dim3(nf), dim3(256), 0, st, gm, 1, 0, gm.part, h);
    KCHECK();
    hipLaunchKernelGGL(k_gm_gemv_sub, gx, dim3(256), 0, st, gm, V, h, W);
    KCHECK();
  }
  hipLaunchKernelGGL(k_gm_dots_partial, gd, dim3(256), 0, st, gm, 0, 0, V, W, gm.part);
  KCHECK();
  hipLaunchKernelGGL(k_gm_dots_final, dim3(nf), dim3(256), 0, st, gm, 0, 0, gm.part, gm.nr);
  KCHECK();
  hipLaunchKernelGGL(k_gm_givens, dim3(1), dim3(256), 0, st, gm);
  KCHECK();
  hipLaunchKernelGGL(k_gm_scale_copy, gx, dim3(256), 0, st, gm, W, V);
  KCHECK();
}

void launch_gm_finish(const GmresDev& gm, const double* V, double* X, hipStream_t st) {
  hipLaunchKernelGGL(k_gm_backsolve, dim3((gm.ns + 63) / 64), dim3(64), 0, st, gm);
  KCHECK();
  hipLaunchKernelGGL(k_gm_solution, dim3(msys_grid_x(gm.maxlen), gm.ns), dim3(256), 0, st, gm, V, X);
  KCHECK();
}

// ---- per-surface reductions: surface q owns rows [off[q], off[q+1]) ----
// out[d][q] = scale[q] * sum_{i in q} x[d][i] (w ? w[i] : 1), one block per
// (surface, density), fixed summation order
constexpr int SEG_BS = 1024;  // threads per (surface, density) block of the segment sums
template <typename T>
__global__ __launch_bounds__(SEG_BS) void k_seg_dot(int nsurf, int64_t N, const int64_t* __restrict__ off,
                                                    const T* __restrict__ x, const double* __restrict__ w,
                                                    const double* __restrict__ scale, double* __restrict__ out) {
  // one wide block per (surface, density): eight independent partial sums
  // per thread keep eight loads of x (and w) in flight, so that a surface
  // of ~1e5 nodes is not a chain of dependent load latencies; the order of
  // the sums is fixed, so results are reproducible
  __shared__ double red[SEG_BS];
  const int q = blockIdx.x, d = blockIdx.y;
  const T* xd = x + (int64_t)d * N;
  const int64_t b = off[q], e = off[q + 1];
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t i = b + threadIdx.x;
  if (w) {
    for (; i + 7 * SEG_BS < e; i += 8 * SEG_BS)
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += (double)xd[i + u * SEG_BS] * w[i + u * SEG_BS];
    for (; i < e; i += SEG_BS) a[0] += (double)xd[i] * w[i];
  } else {
    for (; i + 7 * SEG_BS < e; i += 8 * SEG_BS)
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += (double)xd[i + u * SEG_BS];
    for (; i < e; i += SEG_BS) a[0] += (double)xd[i];
  }
  red[threadIdx.x] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  __syncthreads();
  for (int o = SEG_BS / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[(int64_t)d * nsurf + q] = red[0] * scale[q];
}
// y[d][i] = x[d][i] + alpha (w ? w[i] : 1) c[d][surf[i]]
template <typename T>
__global__ void k_seg_axpy(int nd, int nsurf, int64_t N, const int* __restrict__ surf, const T* __restrict__ x,
                           double alpha, const double* __restrict__ w, const double* __restrict__ c,
                           T* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int q = surf[i];
  const double f = alpha * (w ? w[i] : 1.0);
  for (int d = 0; d < nd; ++d)
    y[(int64_t)d * N + i] = (T)((double)x[(int64_t)d * N + i] + f * c[(int64_t)d * nsurf + q]);
}
template <typename T>
void launch_seg_dot(int nd, int nsurf, int64_t N, const int64_t* off, const T* x, const double* w,
                    const double* scale, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_dot<T>, dim3(nsurf, nd), dim3(SEG_BS), 0, st, nsurf, N, off, x, w, scale, out);
  KCHECK();
}
template <typename T>
void launch_seg_axpy(int nd, int nsurf, int64_t N, const int* surf, const T* x, double alpha, const double* w,
                     const double* c, T* y, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_axpy<T>, dim3((N + 255) / 256), dim3(256), 0, st, nd, nsurf, N, surf, x, alpha, w, c, y);
  KCHECK();
}

// explicit instantiations
#define INST(T)                                                                                                   \
  template void launch_strengths<T>(const T*, int, int64_t, int, int, int, const T*, const T*, const int*,        \
                                    int64_t, T*, hipStream_t);                                                    \
  template void launch_fmm<T>(const DevTree<T>&, int, int, const T*, T*, T*, T*, T*, int64_t, int64_t,       \
                              hipStream_t, PhaseTimer*);                                                  \
  template void launch_corr_grad<T>(int, int64_t, int, const int64_t*, const int*, const T*, const T*, T*,        \
                                    hipStream_t);                                                                 \
  template void launch_combine_grad_fin<T>(int, int64_t, const T*, const T*, const int*, const T*, T*, T*, T*, T*, \
                                           hipStream_t);                                                          \
  template void launch_combine_grad<T>(int, int64_t, int, const int64_t*, const int*, const T*, const T*,        \
                                       const T*, const int*, const T*, T*, T*, T*, T*, hipStream_t);             \
  template void launch_combine_a3a<T>(int, int64_t, int, const int64_t*, const int*, const T*, const T*,         \
                                      const T*, const int*, const T*, T*, T*, int64_t, hipStream_t);             \
  template void launch_combine_a3b<T>(int, int64_t, int, const int64_t*, const int*, const T*, const T*,         \
                                      const T*, const T*, int64_t, const T*, const int*, const T*, const double*, \
                                      int, const int64_t*, const int*, const double*, T*, T*, double*, hipStream_t);                                     \
  template void launch_p2m_tables<T>(const DevTree<T>&, T*, T*, hipStream_t);                                  \
  template int64_t leaf_d_stride<T>(int, int);                                                                  \
  template void launch_a2_str1<T>(int, int64_t, const T*, const T*, const T*, const T*, T*, T*, hipStream_t);  \
  template void launch_a2_str2<T>(int, int64_t, const T*, const T*, const T*, const T*, const T*, T*,          \
                                  hipStream_t);                                                                \
  template void launch_combine_a2a<T>(int, int64_t, int, const int64_t*, const int*, const T*, const T*,        \
                                      const T*, const T*, const T*, const int*, const T*, T*, T*, T*,           \
                                      hipStream_t);                                                            \
  template void launch_combine_a2b<T>(int, int64_t, int, const int64_t*, const int*, const T*, const T*,        \
                                      const T*, const T*, const T*, const T*, const int*, T*, hipStream_t);     \
  template void launch_combine_pot<T>(int, int64_t, int, const int64_t*, const int*, const T*, const T*, const T*, \
                                      const int*, T*, hipStream_t);                                             \
  template void launch_adj_strengths<T>(int, int64_t, const T*, const T*, const T*, const T*, const T*,          \
                                        const int*, T*, T*, hipStream_t);                                       \
  template void launch_adj_combine<T>(int, int, int, int, int64_t, int64_t, const T*, const T*, const T*,       \
                                      const int*, const int64_t*, const int*, const int64_t*, const T*, const T*, \
                                      T*, hipStream_t);                                                           \
  template void launch_scatter_perm<T>(int, int64_t, const T*, const int*, T*, hipStream_t);                    \
  template void launch_xbar_S<T>(int, int, int, int, int64_t, int64_t, const T*, const T*, const int*, const T*, \
                                 const int*, const T*, const T*, const int*, T*, hipStream_t);                  \
  template void launch_adj3_str1<T>(int, int64_t, const T*, const T*, const int*, T*, T*, hipStream_t);          \
  template void launch_adj3_str2<T>(int, int64_t, const T*, const T*, const T*, const int*, T*, T*, hipStream_t); \
  template void launch_adj3_comb1<T>(int, int, int, int, int64_t, int64_t, const T*, const T*, const T*,         \
                                     const int*, const int64_t*, const int*, const int64_t*, const T*, const T*, \
                                     T*, T*, hipStream_t);                                                        \
  template void launch_adj3_comb2<T>(int, int, int, int, int64_t, int64_t, const T*, const T*, const T*,         \
                                     const int*, const int64_t*, const int*, const int64_t*, const T*, const T*, \
                                     const T*, const T*, const double*, int, const int*, T*, hipStream_t);                         \
  template void launch_seg_dot<T>(int, int, int64_t, const int64_t*, const T*, const double*, const double*,     \
                                  double*, hipStream_t);                                                        \
  template void launch_seg_axpy<T>(int, int, int64_t, const int*, const T*, double, const double*, const double*, \
                                   T*, hipStream_t);
INST(float)
INST(double)
template void launch_convert<double, float>(const double*, float*, int64_t, hipStream_t);
template void launch_convert<float, double>(const float*, double*, int64_t, hipStream_t);

}  // namespace lb
