// Uniform-depth octree: 21-bit-per-axis Morton keys, stable sort of targets
// and sources by key, unique prefixes per level, parent/child links,
// U-lists (adjacent leaves holding sources) and V-lists (children of the
// parent's neighbours that are not neighbours, holding sources).
#include "octree.hpp"
#include "common.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace lb {

static inline uint64_t spread21(uint64_t x) {
  x &= 0x1fffff;
  x = (x | x << 32) & 0x1f00000000ffffULL;
  x = (x | x << 16) & 0x1f0000ff0000ffULL;
  x = (x | x << 8) & 0x100f00f00f00f00fULL;
  x = (x | x << 4) & 0x10c30c30c30c30c3ULL;
  x = (x | x << 2) & 0x1249249249249249ULL;
  return x;
}
static inline uint64_t morton(uint64_t ix, uint64_t iy, uint64_t iz) {
  return spread21(ix) | (spread21(iy) << 1) | (spread21(iz) << 2);
}
static inline uint32_t compact21(uint64_t x) {
  x &= 0x1249249249249249ULL;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ULL;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00fULL;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffULL;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffULL;
  x = (x ^ (x >> 32)) & 0x1fffff;
  return (uint32_t)x;
}

void Octree::set_frame(const double mn[3], const double mx[3]) {
  side = 0;
  for (int d = 0; d < 3; ++d) side = std::max(side, mx[d] - mn[d]);
  side = side * (1.0 + 1e-6) + 1e-12;
  for (int d = 0; d < 3; ++d) lo[d] = 0.5 * (mn[d] + mx[d]) - 0.5 * side;
}

int Octree::choose_depth(const int64_t* cnt, int64_t ns, int leaf_src, double min_leaf_side) const {
  int dep = 2;
  for (int l = 2; l <= 20; ++l) {
    dep = l;
    if (cnt[l] > 0 && (double)ns / (double)cnt[l] <= (double)leaf_src) break;
  }
  while (dep > 1 && box_side(dep) <= min_leaf_side) --dep;
  return dep;
}

void Octree::build(const double* tgt, int64_t nt, const double* src, int64_t ns, int leaf_src,
                   double min_leaf_side, int depth_req) {
  double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
  auto upd = [&](const double* p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
      for (int d = 0; d < 3; ++d) { mn[d] = std::min(mn[d], p[3 * i + d]); mx[d] = std::max(mx[d], p[3 * i + d]); }
  };
  upd(tgt, nt);
  upd(src, ns);
  set_frame(mn, mx);
  const double scale = (double)(1 << 21) / side;
  auto key21 = [&](const double* p) {
    uint64_t c[3];
    for (int d = 0; d < 3; ++d) {
      double t = std::floor((p[d] - lo[d]) * scale);
      c[d] = (uint64_t)std::min(std::max(t, 0.0), (double)((1 << 21) - 1));
    }
    return morton(c[0], c[1], c[2]);
  };
  std::vector<uint64_t> kt(nt), ks(ns);
  for (int64_t i = 0; i < nt; ++i) kt[i] = key21(&tgt[3 * i]);
  for (int64_t i = 0; i < ns; ++i) ks[i] = key21(&src[3 * i]);
  // choose depth
  if (depth_req >= 0) {
    depth = std::min(depth_req, 20);
  } else {
    std::vector<uint64_t> sk = ks;
    std::sort(sk.begin(), sk.end());
    int64_t cnt[21] = {0};
    for (int l = 2; l <= 20; ++l) {
      int shift = 3 * (21 - l);
      for (int64_t i = 0; i < ns; ++i)
        if (i == 0 || (sk[i] >> shift) != (sk[i - 1] >> shift)) ++cnt[l];
    }
    depth = choose_depth(cnt, ns, leaf_src, min_leaf_side);
  }
  const int shift = 3 * (21 - depth);
  // stable sort by leaf key
  tgt_perm.resize(nt);
  src_perm.resize(ns);
  std::iota(tgt_perm.begin(), tgt_perm.end(), 0);
  std::iota(src_perm.begin(), src_perm.end(), 0);
  std::stable_sort(tgt_perm.begin(), tgt_perm.end(), [&](int64_t a, int64_t b) { return (kt[a] >> shift) < (kt[b] >> shift); });
  std::stable_sort(src_perm.begin(), src_perm.end(), [&](int64_t a, int64_t b) { return (ks[a] >> shift) < (ks[b] >> shift); });
  tgt_pos.resize(nt);
  src_pos.resize(ns);
  for (int64_t j = 0; j < nt; ++j) tgt_pos[tgt_perm[j]] = j;
  for (int64_t j = 0; j < ns; ++j) src_pos[src_perm[j]] = j;
  // unique leaf keys
  std::vector<uint64_t> leafk;
  leafk.reserve(nt + ns);
  for (int64_t j = 0; j < nt; ++j) leafk.push_back(kt[tgt_perm[j]] >> shift);
  for (int64_t j = 0; j < ns; ++j) leafk.push_back(ks[src_perm[j]] >> shift);
  std::sort(leafk.begin(), leafk.end());
  leafk.erase(std::unique(leafk.begin(), leafk.end()), leafk.end());
  // levels bottom-up
  std::vector<std::vector<uint64_t>> lk(depth + 1);
  lk[depth] = leafk;
  for (int l = depth - 1; l >= 0; --l) {
    lk[l].clear();
    for (uint64_t k : lk[l + 1]) {
      uint64_t pk = k >> 3;
      if (lk[l].empty() || lk[l].back() != pk) lk[l].push_back(pk);
    }
  }
  lev_off.assign(depth + 2, 0);
  for (int l = 0; l <= depth; ++l) lev_off[l + 1] = lev_off[l] + (int)lk[l].size();
  const int nb = lev_off[depth + 1];
  bx.resize(nb); by.resize(nb); bz.resize(nb);
  parent.assign(nb, -1);
  child.assign((size_t)nb * 8, -1);
  has_src.assign(nb, 0);
  has_tgt.assign(nb, 0);
  auto find = [&](int l, uint64_t k) -> int {
    auto it = std::lower_bound(lk[l].begin(), lk[l].end(), k);
    if (it == lk[l].end() || *it != k) return -1;
    return lev_off[l] + (int)(it - lk[l].begin());
  };
  for (int l = 0; l <= depth; ++l)
    for (size_t i = 0; i < lk[l].size(); ++i) {
      int g = lev_off[l] + (int)i;
      uint64_t k = lk[l][i];
      bx[g] = compact21(k);
      by[g] = compact21(k >> 1);
      bz[g] = compact21(k >> 2);
      if (l > 0) {
        int pg = find(l - 1, k >> 3);
        parent[g] = pg;
        child[(size_t)pg * 8 + (k & 7)] = g;
      }
    }
  // leaf ranges
  const int nleaf = (int)lk[depth].size();
  tgt_beg.assign(nleaf, 0); tgt_end.assign(nleaf, 0);
  src_beg.assign(nleaf, 0); src_end.assign(nleaf, 0);
  {
    int64_t j = 0;
    for (int b = 0; b < nleaf; ++b) {
      tgt_beg[b] = (int)j;
      while (j < nt && (kt[tgt_perm[j]] >> shift) == lk[depth][b]) ++j;
      tgt_end[b] = (int)j;
    }
    j = 0;
    for (int b = 0; b < nleaf; ++b) {
      src_beg[b] = (int)j;
      while (j < ns && (ks[src_perm[j]] >> shift) == lk[depth][b]) ++j;
      src_end[b] = (int)j;
    }
  }
  max_leaf_tgt = max_leaf_src = 0;
  for (int b = 0; b < nleaf; ++b) {
    int g = lev_off[depth] + b;
    has_src[g] = src_end[b] > src_beg[b];
    has_tgt[g] = tgt_end[b] > tgt_beg[b];
    max_leaf_tgt = std::max(max_leaf_tgt, tgt_end[b] - tgt_beg[b]);
    max_leaf_src = std::max(max_leaf_src, src_end[b] - src_beg[b]);
  }
  for (int l = depth - 1; l >= 0; --l)
    for (int g = lev_off[l]; g < lev_off[l + 1]; ++g)
      for (int c = 0; c < 8; ++c) {
        int ch = child[(size_t)g * 8 + c];
        if (ch < 0) continue;
        has_src[g] |= has_src[ch];
        has_tgt[g] |= has_tgt[ch];
      }
  auto lookup = [&](int l, int x, int y, int z) -> int {
    int n = 1 << l;
    if (x < 0 || y < 0 || z < 0 || x >= n || y >= n || z >= n) return -1;
    return find(l, morton((uint64_t)x, (uint64_t)y, (uint64_t)z));
  };
  // U-lists
  ulist_ptr.assign(nleaf + 1, 0);
  ulist.clear();
  for (int b = 0; b < nleaf; ++b) {
    int g = lev_off[depth] + b;
    if (has_tgt[g])
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            int n = lookup(depth, bx[g] + dx, by[g] + dy, bz[g] + dz);
            if (n >= 0 && has_src[n]) ulist.push_back(n - lev_off[depth]);
          }
    ulist_ptr[b + 1] = (int)ulist.size();
  }
  // V-lists
  vlist_ptr.assign(nb + 1, 0);
  vlist_src.clear();
  vlist_off.clear();
  for (int g = 0; g < nb; ++g) {
    int l = 0;
    while (g >= lev_off[l + 1]) ++l;
    if (l >= 2 && has_tgt[g]) {
      int pg = parent[g];
      for (int dx = -1; dx <= 1; ++dx)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dz = -1; dz <= 1; ++dz) {
            int pn = lookup(l - 1, bx[pg] + dx, by[pg] + dy, bz[pg] + dz);
            if (pn < 0) continue;
            for (int c = 0; c < 8; ++c) {
              int ch = child[(size_t)pn * 8 + c];
              if (ch < 0 || !has_src[ch]) continue;
              int ox = bx[g] - bx[ch], oy = by[g] - by[ch], oz = bz[g] - bz[ch];
              if (std::abs(ox) <= 1 && std::abs(oy) <= 1 && std::abs(oz) <= 1) continue;
              vlist_src.push_back(ch);
              vlist_off.push_back(((ox + 3) * 7 + (oy + 3)) * 7 + (oz + 3));
            }
          }
    }
    vlist_ptr[g + 1] = (int)vlist_src.size();
  }
}

}  // namespace lb
