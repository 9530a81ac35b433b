// Uniform-depth octree over the FMM targets (Nystrom nodes) and sources
// (oversampled points) of one surface.  The tree itself is not described in
// the paper (it sits inside the point FMM of Section 4); surface point sets
// are quasi-uniform, so all leaves live on one level, which leaves only the
// U-list (adjacent leaves, direct sums) and the V-list (same-level
// well-separated boxes, M2L) -- no W/X lists.
#pragma once
#include <cstdint>
#include <vector>

namespace lb {

struct Octree {
  int depth = 0;                 // leaf level; boxes exist on levels 0..depth
  double lo[3] = {0, 0, 0};      // root cube corner
  double side = 1.0;             // root cube side
  std::vector<int> lev_off;      // [depth+2] global box id range of each level
  std::vector<int> bx, by, bz;   // integer coordinates of each box on its level
  std::vector<int> parent;       // [nbox], -1 at the root
  std::vector<int> child;        // [nbox][8], -1 when absent
  std::vector<uint8_t> has_src, has_tgt;
  // leaves (global ids lev_off[depth] ...), ranges in tree order
  std::vector<int> tgt_beg, tgt_end, src_beg, src_end;   // indexed by leaf number
  std::vector<int64_t> tgt_perm, src_perm;               // tree position -> input index
  std::vector<int64_t> tgt_pos, src_pos;                 // input index -> tree position
  std::vector<int> ulist_ptr, ulist;                     // per leaf: leaves with sources
  std::vector<int> vlist_ptr, vlist_src, vlist_off;      // per global box: V-list
  int max_leaf_tgt = 0, max_leaf_src = 0;

  // depth < 0: choose automatically (mean sources per leaf <= leaf_src, leaf
  // side > min_leaf_side).  depth 0 gives a single box (all pairs direct).
  void build(const double* tgt, int64_t nt, const double* src, int64_t ns, int leaf_src,
             double min_leaf_side, int depth);
  // The same tree built on the current HIP device (Morton keys, stable LSD
  // radix sorts, unique boxes per level, links and lists in HIP kernels);
  // the result is identical to build(): same frame, depth, orders and lists.
  void build_device(const double* tgt, int64_t nt, const double* src, int64_t ns, int leaf_src,
                    double min_leaf_side, int depth);
  // root cube from the bounding box of all points (both builds)
  void set_frame(const double mn[3], const double mx[3]);
  // automatic depth: the first level >= 2 whose mean number of sources per
  // non-empty leaf is <= leaf_src (cnt[l] = non-empty source boxes on level
  // l, l = 2..20), then coarsened while the leaf side is <= min_leaf_side
  int choose_depth(const int64_t* cnt, int64_t ns, int leaf_src, double min_leaf_side) const;
  double box_side(int level) const { return side / (double)(1 << level); }
  int nbox() const { return lev_off.back(); }
};

}  // namespace lb
