// Translation operators of the Laplace FMM (the vector FMM of Section 4,
// eq. fmm-formula, for charges and dipoles), in a real coefficient layout.
//
// Solid harmonics (complex, Condon-Shortley Legendre functions P_n^m):
//   R_n^m(x) = r^n P_n^m(cos t) e^{i m f} / (n+m)!,
//   S_n^m(x) = (n-m)! P_n^m(cos t) e^{i m f} / r^{n+1},
// so that 1/|x - y| = sum_{n,m} conj(R_n^m(y)) S_n^m(x) for |y| < |x|.
// Stored coefficients use the normalized pair Rt = R c, St = S / c with
// c_n^m = sqrt((n+m)! (n-m)!), and box-size scaling: a multipole about the
// centre of a box of side h is Mh_n = sum_j q_j conj(Rt_n((y_j - c)/h)), a
// local expansion is Phi(x) = sum Lh_n Rt_n((x - c)/h).  With this scaling
// every translation matrix is independent of the level (M2L carries 1/h).
//
// Real layout of a conjugate-symmetric coefficient set of order p:
//   index n^2 -> Re C_n^0, n^2 + 2m - 1 -> Re C_n^m, n^2 + 2m -> Im C_n^m
//   (m = 1..n), L = (p+1)^2 reals.
#pragma once
#include <cstdint>
#include <memory>
#include <new>
#include <utility>
#include <vector>

namespace lb {

// Allocator that leaves value-initialized elements of trivially
// constructible type uninitialized: large host tables that are filled
// (in parallel) right after the allocation skip a serial zero-fill.
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U> struct rebind { using other = NoInitAlloc<U>; };
  NoInitAlloc() = default;
  template <class U> NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <class U> void construct(U* p) noexcept { ::new (static_cast<void*>(p)) U; }
  template <class U, class... A> void construct(U* p, A&&... a) { ::new (static_cast<void*>(p)) U(std::forward<A>(a)...); }
};
template <class T> using big_vector = std::vector<T, NoInitAlloc<T>>;

struct Translations {
  int p = 0, L = 0;
  std::vector<double> m2m;   // [8][L][L]   child octant -> parent
  std::vector<double> l2l;   // [8][L][L]   parent -> child octant
  big_vector<double> m2l;    // [343][L][L] offset (target - source) in {-3..3}^3, unit box
                             // (zero for the 27 offsets in {-1..1}^3)
  std::vector<double> dgrad; // [3][p^2][L]       d/dx, d/dy, d/dz (unit box)
  std::vector<double> dhess; // [6][(p-1)^2][L]   xx, xy, xz, yy, yz, zz (unit box)
  void build(int p);
};

inline int m2l_offset_id(int ox, int oy, int oz) { return ((ox + 3) * 7 + (oy + 3)) * 7 + (oz + 3); }
inline int octant_id(int bx, int by, int bz) { return bx | (by << 1) | (bz << 2); }

}  // namespace lb
