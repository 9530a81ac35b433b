// Host construction of the FMM translation matrices (real layout, see
// harmonics.hpp).  Addition theorems used (unnormalized harmonics):
//   M2M: M'_j^s = sum_{k,l} M_{j-k}^{s-l} conj(R_k^l(b)),    b = c_child - c_parent
//   M2L: L_k^l  = (-1)^{k+l} sum_{n,m} M_n^m S_{n+k}^{m-l}(A), A = c_target - c_source
//   L2L: L'_j^s = sum_{k>=j,l} L_k^l R_{k-j}^{l-s}(b),         b = c_child - c_parent
//   derivatives of a local expansion:
//     d/dz Rt_n^m = sqrt((n+m)(n-m)) Rt_{n-1}^m,
//     (d/dx + i d/dy) Rt_n^m =  sqrt((n-m)(n-m-1)) Rt_{n-1}^{m+1},
//     (d/dx - i d/dy) Rt_n^m = -sqrt((n+m)(n+m-1)) Rt_{n-1}^{m-1}.
#include "harmonics.hpp"
#include "common.hpp"

#include <cmath>
#include <complex>

namespace lb {

typedef std::complex<double> cd;

static inline int fidx(int n, int m) { return n * n + n + m; }  // full complex index

// log of c_n^m = sqrt((n+m)! (n-m)!), from a table of log-factorials
static std::vector<double> g_lfac;
static inline double lc(int n, int m) { return 0.5 * (g_lfac[n + m] + g_lfac[n - m]); }

// normalized regular harmonics Rt_n^m, 0 <= m <= n <= p, full array
static void regular(int p, const double* x, std::vector<cd>& F) {
  const double X = x[0], Y = x[1], Z = x[2], r2 = X * X + Y * Y + Z * Z;
  std::vector<cd> R((p + 1) * (p + 1));
  auto at = [&](int n, int m) -> cd& { return R[n * (p + 1) + m]; };
  at(0, 0) = 1.0;
  for (int m = 0; m <= p; ++m) {
    if (m > 0) at(m, m) = -cd(X, Y) * std::sqrt((2.0 * m - 1.0) / (2.0 * m)) * at(m - 1, m - 1);
    if (m + 1 <= p) at(m + 1, m) = Z * std::sqrt(2.0 * m + 1.0) * at(m, m);
    for (int n = m + 1; n < p; ++n)
      at(n + 1, m) = ((2.0 * n + 1.0) * Z * at(n, m) - r2 * std::sqrt((double)(n + m) * (n - m)) * at(n - 1, m)) /
                     std::sqrt((double)(n + 1 + m) * (n + 1 - m));
  }
  F.assign((p + 1) * (p + 1), 0.0);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m)
      F[fidx(n, m)] = m >= 0 ? at(n, m) : ((m & 1) ? -1.0 : 1.0) * std::conj(at(n, -m));
}

// normalized irregular harmonics St_n^m, full array up to degree p
static void irregular(int p, const double* x, std::vector<cd>& F) {
  const double X = x[0], Y = x[1], Z = x[2], r2 = X * X + Y * Y + Z * Z;
  std::vector<cd> S((p + 1) * (p + 1));
  auto at = [&](int n, int m) -> cd& { return S[n * (p + 1) + m]; };
  at(0, 0) = 1.0 / std::sqrt(r2);
  for (int m = 0; m <= p; ++m) {
    if (m > 0)  // S_m^m = -(2m-1)(x+iy)/r^2 S_{m-1}^{m-1}, c_m^m/c_{m-1}^{m-1} = sqrt(2m(2m-1))
      at(m, m) = -(2.0 * m - 1.0) * cd(X, Y) / r2 * at(m - 1, m - 1) / std::sqrt(2.0 * m * (2.0 * m - 1.0));
    if (m + 1 <= p) at(m + 1, m) = (2.0 * m + 1.0) * Z / r2 * at(m, m) / std::sqrt(2.0 * m + 1.0);
    for (int n = m + 1; n < p; ++n)
      at(n + 1, m) = ((2.0 * n + 1.0) * Z * at(n, m) - std::sqrt((double)(n + m) * (n - m)) * at(n - 1, m)) /
                     (r2 * std::sqrt((double)(n + 1 + m) * (n + 1 - m)));
  }
  F.assign((p + 1) * (p + 1), 0.0);
  for (int n = 0; n <= p; ++n)
    for (int m = -n; m <= n; ++m)
      F[fidx(n, m)] = m >= 0 ? at(n, m) : ((m & 1) ? -1.0 : 1.0) * std::conj(at(n, -m));
}

// Complex full map Tc[(pout+1)^2][(pin+1)^2] -> real [Lout][Lin], assuming a
// conjugate-symmetric input and output.
static void to_real(const std::vector<cd>& Tc, int pout, int pin, double* out) {
  const int Fin = (pin + 1) * (pin + 1), Lin = Fin, Lout = (pout + 1) * (pout + 1);
  for (int i = 0; i < Lout * Lin; ++i) out[i] = 0.0;
  for (int k = 0; k <= pout; ++k)
    for (int l = 0; l <= k; ++l) {
      const int rre = l == 0 ? k * k : k * k + 2 * l - 1;
      const int rim = k * k + 2 * l;
      for (int n = 0; n <= pin; ++n)
        for (int m = 0; m <= n; ++m) {
          cd ca, cb;  // coefficients of Re and Im of the input C_n^m
          const cd tp = Tc[(size_t)fidx(k, l) * Fin + fidx(n, m)];
          if (m == 0) {
            ca = tp;
          } else {
            const cd tm = Tc[(size_t)fidx(k, l) * Fin + fidx(n, -m)];
            const double sg = (m & 1) ? -1.0 : 1.0;
            ca = tp + sg * tm;
            cb = cd(0, 1) * (tp - sg * tm);
          }
          const int cre = m == 0 ? n * n : n * n + 2 * m - 1;
          const int cim = n * n + 2 * m;
          out[(size_t)rre * Lin + cre] += ca.real();
          if (m > 0) out[(size_t)rre * Lin + cim] += cb.real();
          if (l > 0) {
            out[(size_t)rim * Lin + cre] += ca.imag();
            if (m > 0) out[(size_t)rim * Lin + cim] += cb.imag();
          }
        }
    }
}

// derivative maps on full complex coefficients: order pin -> pin - 1
static void deriv_maps(int pin, std::vector<cd>& Gx, std::vector<cd>& Gy, std::vector<cd>& Gz) {
  const int Fin = (pin + 1) * (pin + 1), Fout = pin * pin;
  Gx.assign((size_t)Fout * Fin, 0.0);
  Gy.assign((size_t)Fout * Fin, 0.0);
  Gz.assign((size_t)Fout * Fin, 0.0);
  for (int n = 0; n < pin; ++n)
    for (int m = -n; m <= n; ++m) {
      const size_t row = (size_t)fidx(n, m) * Fin;
      Gz[row + fidx(n + 1, m)] = std::sqrt((double)(n + 1 + m) * (n + 1 - m));
      cd gp = 0.0, gm = 0.0;
      int ip = -1, im = -1;
      if (m - 1 >= -(n + 1)) { ip = fidx(n + 1, m - 1); gp = std::sqrt((double)(n - m + 2) * (n - m + 1)); }
      if (m + 1 <= n + 1) { im = fidx(n + 1, m + 1); gm = -std::sqrt((double)(n + m + 2) * (n + m + 1)); }
      // Gx = (G+ + G-)/2, Gy = -(i/2)(G+ - G-)
      if (ip >= 0) { Gx[row + ip] += 0.5 * gp; Gy[row + ip] += cd(0, -0.5) * gp; }
      if (im >= 0) { Gx[row + im] += 0.5 * gm; Gy[row + im] += cd(0, 0.5) * gm; }
    }
}

static std::vector<cd> matmul(const std::vector<cd>& A, const std::vector<cd>& B, int r, int k, int c) {
  std::vector<cd> C((size_t)r * c, 0.0);
  for (int i = 0; i < r; ++i)
    for (int t = 0; t < k; ++t) {
      cd a = A[(size_t)i * k + t];
      if (a == 0.0) continue;
      for (int j = 0; j < c; ++j) C[(size_t)i * c + j] += a * B[(size_t)t * c + j];
    }
  return C;
}

void Translations::build(int p_) {
  p = p_;
  L = (p + 1) * (p + 1);
  g_lfac.assign(4 * p + 8, 0.0);
  for (size_t i = 1; i < g_lfac.size(); ++i) g_lfac[i] = g_lfac[i - 1] + std::log((double)i);
  const int F = L;
  m2m.assign((size_t)8 * L * L, 0.0);
  l2l.assign((size_t)8 * L * L, 0.0);
  m2l.resize((size_t)343 * L * L);
  std::vector<cd> Tc((size_t)F * F), Rb;
  for (int oct = 0; oct < 8; ++oct) {
    double beta[3] = {(oct & 1) - 0.5, ((oct >> 1) & 1) - 0.5, ((oct >> 2) & 1) - 0.5};
    regular(p, beta, Rb);
    // M2M
    std::fill(Tc.begin(), Tc.end(), 0.0);
    for (int j = 0; j <= p; ++j)
      for (int s = -j; s <= j; ++s)
        for (int n = 0; n <= j; ++n)
          for (int m = -n; m <= n; ++m) {
            int k = j - n, l = s - m;
            if (l < -k || l > k) continue;
            double f = std::exp(lc(j, s) - lc(n, m) - lc(k, l) - j * std::log(2.0));
            Tc[(size_t)fidx(j, s) * F + fidx(n, m)] = f * std::conj(Rb[fidx(k, l)]);
          }
    to_real(Tc, p, p, &m2m[(size_t)oct * L * L]);
    // L2L
    std::fill(Tc.begin(), Tc.end(), 0.0);
    for (int j = 0; j <= p; ++j)
      for (int s = -j; s <= j; ++s)
        for (int k = j; k <= p; ++k)
          for (int l = -k; l <= k; ++l) {
            int kk = k - j, ll = l - s;
            if (ll < -kk || ll > kk) continue;
            double f = std::exp(lc(k, l) - lc(j, s) - lc(kk, ll) - k * std::log(2.0));
            Tc[(size_t)fidx(j, s) * F + fidx(k, l)] = f * Rb[fidx(kk, ll)];
          }
    to_real(Tc, p, p, &l2l[(size_t)oct * L * L]);
  }
  // M2L: T[(k,l)][(n,m)] = (-1)^{k+l} c_{n+k}^{m-l} / (c_k^l c_n^m) St_{n+k}^{m-l}(A);
  // the factor does not depend on the offset A: tabulated once
  std::vector<double> fac((size_t)F * F, 0.0);
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k <= p; ++k)
    for (int l = -k; l <= k; ++l)
      for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m) {
          const int nn = n + k, mm = m - l;
          if (mm < -nn || mm > nn) continue;
          const double sg = ((k + l) & 1) ? -1.0 : 1.0;
          fac[(size_t)fidx(k, l) * F + fidx(n, m)] = sg * std::exp(lc(nn, mm) - lc(k, l) - lc(n, m));
        }
#pragma omp parallel for schedule(dynamic, 1)
  for (int id = 0; id < 343; ++id) {
    const int ox = id / 49 - 3, oy = (id / 7) % 7 - 3, oz = id % 7 - 3;
    double* out = &m2l[(size_t)m2l_offset_id(ox, oy, oz) * L * L];
    if (std::abs(ox) <= 1 && std::abs(oy) <= 1 && std::abs(oz) <= 1) {
      for (size_t e = 0; e < (size_t)L * L; ++e) out[e] = 0.0;
      continue;
    }
    std::vector<cd> SA, Tc((size_t)F * F, 0.0);
    double A[3] = {(double)ox, (double)oy, (double)oz};
    irregular(2 * p, A, SA);
    for (int k = 0; k <= p; ++k)
      for (int l = -k; l <= k; ++l)
        for (int n = 0; n <= p; ++n)
          for (int m = -n; m <= n; ++m) {
            const int nn = n + k, mm = m - l;
            if (mm < -nn || mm > nn) continue;
            Tc[(size_t)fidx(k, l) * F + fidx(n, m)] = fac[(size_t)fidx(k, l) * F + fidx(n, m)] * SA[fidx(nn, mm)];
          }
    to_real(Tc, p, p, out);
  }
  // derivative maps
  std::vector<cd> Gx, Gy, Gz, Gx2, Gy2, Gz2;
  deriv_maps(p, Gx, Gy, Gz);
  const int Lg = p * p, Lh = (p - 1) * (p - 1);
  dgrad.assign((size_t)3 * Lg * L, 0.0);
  to_real(Gx, p - 1, p, &dgrad[0]);
  to_real(Gy, p - 1, p, &dgrad[(size_t)Lg * L]);
  to_real(Gz, p - 1, p, &dgrad[(size_t)2 * Lg * L]);
  deriv_maps(p - 1, Gx2, Gy2, Gz2);
  dhess.assign((size_t)6 * Lh * L, 0.0);
  const std::vector<cd>* first[6] = {&Gx, &Gy, &Gz, &Gy, &Gz, &Gz};
  const std::vector<cd>* second[6] = {&Gx2, &Gx2, &Gx2, &Gy2, &Gy2, &Gz2};
  for (int t = 0; t < 6; ++t) {
    std::vector<cd> Hc = matmul(*second[t], *first[t], Lh, Lg, L);
    to_real(Hc, p - 2, p, &dhess[(size_t)t * Lh * L]);
  }
}

}  // namespace lb
