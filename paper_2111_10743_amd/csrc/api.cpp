// C ABI of the library (include/lb.h): setup, applies, the A3 operator and
// the GMRES solver, orchestrated on the caller's HIP stream.
#include "../../include/lb.h"
#include "common.hpp"
#include "harmonics.hpp"
#include "kernels.hpp"
#include "noalloc.hpp"
#include "octree.hpp"
#include "refelem.hpp"
#include "surface.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

namespace lb {

static thread_local std::string g_last_error;

static double wall_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}
void set_last_error(const std::string& msg) { g_last_error = msg; }

#define HIPTRY(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) fail(LB_EHIP, "%s failed: %s", #x, hipGetErrorString(e_)); \
  } while (0)

// device allocation that frees itself
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { if (p) (void)hipFree(p); }
  void alloc(size_t b) {
    if (b <= bytes && p) return;
    if (p) { (void)hipFree(p); p = nullptr; bytes = 0; }
    if (b == 0) b = 16;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) fail(LB_ENOMEM, "hipMalloc(%zu) failed: %s", b, hipGetErrorString(e));
    bytes = b;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // exactly b bytes (frees a larger buffer)
  void alloc_exact(size_t b) {
    if (b == 0) b = 16;
    if (p && b != bytes) { (void)hipFree(p); p = nullptr; bytes = 0; }
    alloc(b);
  }
};
template <typename T> static inline T* dptr(const DBuf& b) { return reinterpret_cast<T*>(b.p); }

struct PlanBuf {
  GemmPlan pl;
  DBuf grp_mat, grp_beg, pair_src, boxes, box_scale, tptr, tpairs, grp_lo, pair_lo, work[GEMM_NE_MAX + 1];
};

// Densities per FMM traversal: FP32 carries more expansions per traversal
// (wider M2L GEMMs, fewer traversals for many right-hand sides); the FP64
// column scratch of M2L would grow past what the N ~ 1M problems can hold.
template <typename T> constexpr int nemax() { return sizeof(T) == 4 ? GEMM_NE_MAX : 8; }
template <typename T> constexpr int chunk_fwd() { return sizeof(T) == 4 ? 16 : 8; }  // S, grad S
template <typename T> constexpr int chunk_a3() { return nemax<T>() / 3; }           // A3 (3 expansions)
// largest column scratch of the M2L plan (split into parts beyond it)
constexpr size_t M2L_Y_BUDGET = (size_t)8 << 30;

template <typename T, class A>
static void upload(DBuf& d, const std::vector<T, A>& h);

// Triples (matrix id, target box, source box) -> GemmPlan; `boxes` lists every
// target box that gets an output (boxes without triples get zeros unless
// the plan accumulates).
struct Triple { int mat, tgt, src; };
// mat_lo (nullable: all L): active size of each matrix id's translation.
// ne_max: work lists for 1..ne_max expansions per box.
static size_t build_plan(PlanBuf& pb, std::vector<Triple> tr, const std::vector<int>& boxes,
                         const std::vector<double>& scale, bool scaled, bool accumulate, int nbox_total, int L,
                         int ne_max, const std::vector<int>& mat_lo = {}, bool ksplit = false) {
  std::stable_sort(tr.begin(), tr.end(), [](const Triple& a, const Triple& b) {
    return a.mat != b.mat ? a.mat < b.mat : a.tgt < b.tgt;
  });
  std::vector<int> gmat, gbeg, psrc(tr.size());
  for (size_t i = 0; i < tr.size(); ++i) {
    psrc[i] = tr[i].src;
    if (i == 0 || tr[i].mat != tr[i - 1].mat) { gmat.push_back(tr[i].mat); gbeg.push_back((int)i); }
  }
  gbeg.push_back((int)tr.size());
  std::vector<int> slot(nbox_total, -1);
  for (size_t b = 0; b < boxes.size(); ++b) slot[boxes[b]] = (int)b;
  std::vector<int> tptr(boxes.size() + 1, 0), tpairs(tr.size());
  for (const Triple& q : tr) tptr[slot[q.tgt] + 1]++;
  for (size_t b = 0; b < boxes.size(); ++b) tptr[b + 1] += tptr[b];
  std::vector<int> fill(tptr.begin(), tptr.end() - 1);
  for (size_t i = 0; i < tr.size(); ++i) tpairs[fill[slot[tr[i].tgt]]++] = (int)i;
  std::vector<int> glo, plo;
  if (!mat_lo.empty()) {
    for (int m : gmat) glo.push_back(mat_lo[m]);
    for (const Triple& q : tr) plo.push_back(mat_lo[q.mat]);
    upload(pb.grp_lo, glo);
    upload(pb.pair_lo, plo);
  }
  upload(pb.grp_mat, gmat); upload(pb.grp_beg, gbeg); upload(pb.pair_src, psrc);
  upload(pb.boxes, boxes); upload(pb.box_scale, scale); upload(pb.tptr, tptr); upload(pb.tpairs, tpairs);
  GemmPlan& pl = pb.pl;
  pl.ngrp = (int)gmat.size();
  pl.npair = (int)tr.size();
  pl.nbox = (int)boxes.size();
  pl.grp_mat = dptr<int>(pb.grp_mat); pl.grp_beg = dptr<int>(pb.grp_beg); pl.pair_src = dptr<int>(pb.pair_src);
  pl.boxes = dptr<int>(pb.boxes); pl.box_scale = scaled ? dptr<double>(pb.box_scale) : nullptr;
  pl.tptr = dptr<int>(pb.tptr); pl.tpairs = dptr<int>(pb.tpairs);
  pl.grp_lo = glo.empty() ? nullptr : dptr<int>(pb.grp_lo);
  pl.pair_lo = plo.empty() ? nullptr : dptr<int>(pb.pair_lo);
  pl.scaled = scaled;
  pl.accumulate = accumulate;
  // k split (small plans): enough blocks to fill the device, slices of at
  // least 64 coefficients, a multiple of 32 (the k chunks of both precisions)
  pl.kslice = 0;
  pl.nslice = 1;
  if (ksplit && glo.empty()) {
    int64_t nb1 = 0;
    for (int g2 = 0; g2 < pl.ngrp; ++g2)
      nb1 += (int64_t)((L + GEMM_TILE_ROWS - 1) / GEMM_TILE_ROWS) *
             ((gbeg[g2 + 1] - gbeg[g2] + GEMM_TILE_COLS - 1) / GEMM_TILE_COLS);
    const int ks = (int)std::min<int64_t>(8, std::max<int64_t>(1, (2048 + nb1 - 1) / std::max<int64_t>(nb1, 1)));
    int kl = ((L + ks - 1) / ks + 31) / 32 * 32;
    kl = std::max(kl, 64);
    if (kl < L) {
      pl.kslice = kl;
      pl.nslice = (L + kl - 1) / kl;
    }
  }
  pl.ne_max = ne_max;
  for (int ne = 1; ne <= ne_max; ++ne) {
    // the expansion counts of the applies: up to chunk_fwd densities of one
    // expansion, and three expansions per density (A3's second pass, A2)
    if (ne > 16 && ne % 3 != 0) continue;
    std::vector<int> w;
    for (int g2 = 0; g2 < pl.ngrp; ++g2) {
      const int lo = glo.empty() ? L : glo[g2];
      for (int r0 = 0; r0 < lo; r0 += GEMM_TILE_ROWS)
        for (int c0 = gbeg[g2] * ne; c0 < gbeg[g2 + 1] * ne; c0 += GEMM_TILE_COLS)
          for (int kb = 0; kb < lo; kb += pl.kslice ? pl.kslice : lo) {
            w.push_back(g2);
            w.push_back(c0);
            w.push_back(r0);
            w.push_back(kb);
          }
    }
    upload(pb.work[ne], w);
    pl.work[ne] = dptr<int>(pb.work[ne]);
    pl.nwork[ne] = (int)(w.size() / 4);
  }
  return tr.size() * pl.nslice;
}

template <typename T, class A>
static void upload(DBuf& d, const std::vector<T, A>& h) {
  d.alloc(sizeof(T) * std::max<size_t>(h.size(), 1));
  if (!h.empty()) HIPTRY(hipMemcpy(d.p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
}
template <typename T, typename S>
static void upload_as(DBuf& d, const std::vector<S>& h) {
  std::vector<T> c(h.begin(), h.end());
  upload(d, c);
}

// An operator application v -> w captured once as a HIP graph and replayed
// (valid for the captured buffers and density count).
struct OpGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* in = nullptr;
  const void* out = nullptr;
  int n = 0;
  // further buffers and sizes the captured launches depend on (GMRES
  // iteration graphs: basis, state, system count, iteration cap)
  const void* aux0 = nullptr;
  const void* aux1 = nullptr;
  int64_t aux2 = 0;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    in = out = nullptr;
    n = 0;
    aux0 = aux1 = nullptr;
    aux2 = 0;
  }
};

// Everything one precision of the apply needs on the device.
template <typename T>
struct Prec {
  int p = 0, L = 0;
  int n_o = 0;      // oversampled points per patch of this precision's far rule
  int64_t No = 0;   // oversampled points in total
  std::vector<Octree> trees;  // one per surface
  DevTree<T> dt{};
  DBuf tx, ty, tz, tnx, tny, tnz, sx, sy, sz, snx, sny, snz, rm2, trm2, bcx, bcy, bcz;
  DBuf tgt_beg, tgt_end, src_beg, src_end, ulist_ptr, ulist, vlist_ptr, vlist_src, vlist_off;
  DBuf parent, child, child_src, leaf_tgt, leaf_src, lev_src, lev_src_ptr, lev_tgt, lev_tgt_ptr;
  DBuf leaf_box, leaf_lvl, leaf_h;
  DBuf tgt_pos, src_pos, P, wo, vals4, vals3, valsD, nrm, H;
  DBuf m2m, l2l, m2l, dgrad, dhess;
  // batched translation plans (M2L over all levels; M2M, L2L per level)
  std::vector<std::unique_ptr<PlanBuf>> m2l_pb, m2m_pb, l2l_pb;
  std::vector<GemmPlan> m2l_pl, m2m_pl, l2l_pl;
  DBuf Y;
  DBuf p2m_H, p2m_D;
  // work
  DBuf str, M, Lc, D, fmm, mu, y2, tmp_in, tmp_out;
  DBuf a2s;  // A2: strengths of tau, then of mu1 and mu2 [2][chunk_a3][No]
  int ws_rhs = 0;
  // position derivative: mask radii that exclude only coincident points
  // (forward tree) and gradient outputs at the targets (transposed tree)
  DBuf rm2_none, fmm4;
  // leaf-kernel work items (leaf, target range, lanes per target), built
  // from the per-target-leaf (leaf, tbeg, tend, U-list sources) of the trees
  DBuf leaf_work;
  std::vector<int> lw_leaf, lw_tbeg, lw_tend;
  std::vector<int64_t> lw_usrc;
  // tree parameters of the last build (the autotuner rebuilds with others)
  int build_leaf_src = 0, leaf_fmax = 64, leaf_split = 0;
  int fork_late = 0, near_grid = 0, corr_early = 0;  // overlapped-apply schedule (see DevTree)
  DBuf corr;  // early correction sums of the gradient apply [chunk][N][4]
  double m2l_flops = 0;  // algorithmic M2L flops per density (all V-list pairs, orders by offset)
  double min_leaf_side = 0.0;
  bool direct = false;
};

}  // namespace lb

using namespace lb;

struct lb_ctx {
  int k = 0, NP = 0, n_p = 0, n_o = 0;
  double t_setup = 0.0;  // wall-clock seconds of lb_setup / lb_setup_batch (or of the import)
  // surfaces: surface q owns patches [surf_patch[q], surf_patch[q+1]) (its
  // nodes and oversampled points follow in the same order)
  int n_surf = 1;
  std::vector<int> surf_patch;
  std::vector<double> surf_area;
  int64_t N = 0, No = 0;
  lb_opts opts{};
  std::unique_ptr<RefElem> re;    // order k, the FP64 far rule (q = over_q)
  std::unique_ptr<RefElem> re32;  // order k, the FP32 far rule (q = over_q32)
  Surface S;
  std::vector<double> C64;  // [nnzb][n_p][NKER]
  bool host_only = false;
  int device = 0;
  Prec<float> f32;
  Prec<double> f64;
  DBuf row_ptr, patch, w;
  // adjoint applies (built on first use): transposed trees, transposed
  // block-CSR of the corrections (per patch: (row, block) entries), the FP32
  // mask radii and the FP32 tree's minimum leaf side
  Prec<float> a32;
  Prec<double> a64;
  bool adj_built32 = false, adj_built64 = false;
  DBuf cptr, crow, cblk, g4;
  bool csr_t_built = false;
  // transposed A3: z = S^T S^T w per precision, step workspace
  DBuf z32, z64, a3t_a, a3t_b, a3t_scal;
  bool z_built32 = false, z_built64 = false;
  std::vector<float> rm2f;
  // surface calculus (built on first use): nodal differentiation matrices,
  // the chart derivatives given at the nodes and the normals, FP64
  DBuf c_Du, c_Dv, c_Xu, c_Xv, c_nrm;
  bool calc_built = false;
  // A1 workspace per precision: S[1], and the intermediate applies
  DBuf a1_phi0_32, a1_phi0_64, a1_pot, a1_g1, a1_surf, a1_mu, a1_g2, a1_eta;
  // solver workspace
  DBuf V, wv, partial, r, sig, ftmp, utmp, msys2;
  // device GMRES state (GmresDev), skip flags, pinned host word for the
  // per-iteration count of active systems
  DBuf gm_state, gm_skip;
  int* gm_host = nullptr;
  // per-surface row ranges: node_off [n_surf+1] (host and device), the
  // surface of every node, 1/area per surface; scratch for per-surface sums
  std::vector<int64_t> node_off_h;
  DBuf node_off, node_surf, inv_area, seg_scal;
  // GMRES operators replayed from captured HIP graphs (A3 and A3^T, FP64
  // and FP32), captured on the library's own stream
  hipStream_t cap_stream = nullptr;
  // near-field sums overlapped with the far-field passes: a non-blocking
  // side stream (default priority) and its fork/join events
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // GMRES iteration graphs (A3 and A3^T, FP64 and FP32) and the FP64
  // residual applies of the solves
  lb::OpGraph gI64, gI32, gIT64, gIT32, gR64, gRT64;
  lb::OpGraph gI64a2, gI32a2, gR64a2;  // the same for the A2 solves
  DBuf a2b;                             // A2 solves: the right-hand side S f
  void reset_graphs() {
    gI64.reset(); gI32.reset(); gIT64.reset(); gIT32.reset(); gR64.reset(); gRT64.reset();
    gI64a2.reset(); gI32a2.reset(); gR64a2.reset();
  }
  ~lb_ctx() {
    reset_graphs();
    if (gm_host) (void)hipHostFree(gm_host);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (side_stream) (void)hipStreamDestroy(side_stream);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
  }
};

namespace lb {

static void default_opts(lb_opts* o) {
  o->eta_near = 2.0;
  o->over_q = 0;
  o->over_q32 = 0;
  o->p_f32 = 14;
  o->p_f64 = 28;
  o->leaf_src = 1024;
  o->max_iter = 100;
  o->flags = 0;
  o->self_n = 16;
  o->near_q = 8;
  o->near_adm = 2.0;
  o->m2l_trunc32 = 2.5;
  o->m2l_trunc64 = 2.0;
}

template <typename T, class V>
static void transpose_blocks(const V& src, int nblk, int rows, int cols, big_vector<T>& dst) {
  dst.resize((size_t)nblk * rows * cols);
#pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < nblk; ++b)
    for (int c = 0; c < cols; ++c)
      for (int r = 0; r < rows; ++r)
        dst[(size_t)b * rows * cols + (size_t)c * rows + r] = (T)src[(size_t)b * rows * cols + (size_t)r * cols + c];
}

// pack [nnzb][n_p][NKER] corrections into the gradS (k=4: S, Gx, Gy, Gz),
// A3 (k=3: S, S', S''+D') and double-layer (k=1: D) layouts
template <typename T>
static void pack_vals(const std::vector<double>& C, int64_t nnz, std::vector<T>& v4, std::vector<T>& v3,
                      std::vector<T>& vD) {
  v4.resize((size_t)nnz * 4);
  v3.resize((size_t)nnz * 3);
  vD.resize((size_t)nnz);
  for (int64_t e = 0; e < nnz; ++e) {
    const double* c = &C[(size_t)e * NKER];
    v4[4 * e] = (T)c[0]; v4[4 * e + 1] = (T)c[1]; v4[4 * e + 2] = (T)c[2]; v4[4 * e + 3] = (T)c[3];
    v3[3 * e] = (T)c[0]; v3[3 * e + 1] = (T)c[4]; v3[3 * e + 2] = (T)c[5];
    vD[e] = (T)c[6];
  }
}

constexpr size_t P2M_TABLE_MAX = (size_t)64 << 30;

// Several octrees (one per surface) numbered as one forest: the boxes,
// leaves and tree positions of tree s follow those of trees 0..s-1; every
// list holds global numbers.  Trees never interact: each surface's far
// field is its own.
struct Forest {
  int depth = 0, nbox = 0, nleaf = 0;
  std::vector<int> box_level, tree_depth, parent, child, child_src;
  std::vector<double> box_cen, box_scale;      // [nbox][3], [nbox] 2^level / side of its tree
  std::vector<uint8_t> has_src, has_tgt;
  std::vector<int> leaf_box, leaf_lvl;
  std::vector<double> leaf_h;
  std::vector<int> tgt_beg, tgt_end, src_beg, src_end;  // per leaf, global tree positions
  std::vector<int64_t> tgt_perm, src_perm, tgt_pos, src_pos;
  std::vector<int> ulist_ptr, ulist, vlist_ptr, vlist_src, vlist_off;
};

static void merge_forest(const std::vector<Octree>& trees, const std::vector<int64_t>& toff,
                         const std::vector<int64_t>& soff, Forest& F) {
  F = Forest();
  F.ulist_ptr.push_back(0);
  F.vlist_ptr.push_back(0);
  int boff = 0, loff = 0;
  for (size_t s = 0; s < trees.size(); ++s) {
    const Octree& t = trees[s];
    const int nb = t.nbox(), nl = t.lev_off[t.depth + 1] - t.lev_off[t.depth];
    F.depth = std::max(F.depth, t.depth);
    for (int l = 0; l <= t.depth; ++l) {
      const double h = t.box_side(l);
      for (int g = t.lev_off[l]; g < t.lev_off[l + 1]; ++g) {
        F.box_level.push_back(l);
        F.tree_depth.push_back(t.depth);
        F.box_cen.push_back(t.lo[0] + (t.bx[g] + 0.5) * h);
        F.box_cen.push_back(t.lo[1] + (t.by[g] + 0.5) * h);
        F.box_cen.push_back(t.lo[2] + (t.bz[g] + 0.5) * h);
        F.box_scale.push_back((double)(1 << l) / t.side);
        F.parent.push_back(t.parent[g] < 0 ? -1 : t.parent[g] + boff);
        for (int c = 0; c < 8; ++c) {
          const int ch = t.child[(size_t)g * 8 + c];
          F.child.push_back(ch < 0 ? -1 : ch + boff);
          F.child_src.push_back(ch < 0 || !t.has_src[ch] ? -1 : ch + boff);
        }
        F.has_src.push_back(t.has_src[g]);
        F.has_tgt.push_back(t.has_tgt[g]);
        for (int v = t.vlist_ptr[g]; v < t.vlist_ptr[g + 1]; ++v) {
          F.vlist_src.push_back(t.vlist_src[v] + boff);
          F.vlist_off.push_back(t.vlist_off[v]);
        }
        F.vlist_ptr.push_back((int)F.vlist_src.size());
      }
    }
    for (int b = 0; b < nl; ++b) {
      F.leaf_box.push_back(t.lev_off[t.depth] + b + boff);
      F.leaf_lvl.push_back(t.depth);
      F.leaf_h.push_back(t.box_side(t.depth));
      F.tgt_beg.push_back(t.tgt_beg[b] + (int)toff[s]);
      F.tgt_end.push_back(t.tgt_end[b] + (int)toff[s]);
      F.src_beg.push_back(t.src_beg[b] + (int)soff[s]);
      F.src_end.push_back(t.src_end[b] + (int)soff[s]);
      for (int k = t.ulist_ptr[b]; k < t.ulist_ptr[b + 1]; ++k) F.ulist.push_back(t.ulist[k] + loff);
      F.ulist_ptr.push_back((int)F.ulist.size());
    }
    for (int64_t j : t.tgt_perm) F.tgt_perm.push_back(j + toff[s]);
    for (int64_t j : t.src_perm) F.src_perm.push_back(j + soff[s]);
    for (int64_t j : t.tgt_pos) F.tgt_pos.push_back(j + toff[s]);
    for (int64_t j : t.src_pos) F.src_pos.push_back(j + soff[s]);
    boff += nb;
    loff += nl;
  }
  F.nbox = boff;
  F.nleaf = loff;
}

// Active size (p_o + 1)^2 of the M2L translation of each offset o (in box
// widths, id ((ox+3)*7 + (oy+3))*7 + (oz+3)): the multipole of a box of
// half-diagonal a = sqrt(3)/2 seen from a box at centre distance d converges
// like rho(d)^n with rho(d) = a / (d - a), so the order that matches the
// error of the closest V-list offset (d = 2) at order p is
// p ln rho(2) / ln rho(d); `safety` multiplies it (0: full order for all).
static std::vector<int> m2l_orders(int p, double safety) {
  if (!(safety > 0)) return {};
  std::vector<int> lo(343);
  const double a = 0.5 * std::sqrt(3.0);
  const double l2 = std::log(a / (2.0 - a));
  for (int o = 0; o < 343; ++o) {
    const int ox = o / 49 - 3, oy = (o / 7) % 7 - 3, oz = o % 7 - 3;
    const double d = std::sqrt((double)(ox * ox + oy * oy + oz * oz));
    int po = p;
    if (d > 2.0) po = std::min(p, (int)std::ceil(safety * p * l2 / std::log(a / (d - a))));
    po = std::max(po, std::min(p, 4));
    lo[o] = (po + 1) * (po + 1);
  }
  return lo;
}

// Work items of the leaf kernel: one block evaluates targets [tbeg, tend) of
// one leaf with F lanes per target (F a power of two, 256 / F target slots).
// split = 0: one block per leaf, F the largest power of two <= fmax with
// F a <= 256 for a leaf of a targets.  split = s >= 1: a leaf whose U-list
// holds u sources is cut into m <= s items of ceil(a / m) targets, F the
// largest power of two <= min(fmax, 256 / ceil(a / m)), m minimizing
// m (u / F + 2 u / 256 + 8) (near-field iterations per lane, staging of the
// sources, a fixed cost per block).  Items are ordered heaviest first so
// that the grid does not end on a tail of large blocks.
template <typename T>
static void make_leaf_work(Prec<T>& P, int fmax, int split) {
  struct Item { int leaf, tbeg, tend, F; double cost; };
  std::vector<Item> it;
  for (size_t k = 0; k < P.lw_leaf.size(); ++k) {
    const int a = P.lw_tend[k] - P.lw_tbeg[k];
    const double u = (double)P.lw_usrc[k];
    int bm = 1, bF = 1;
    double bc = 1e300;
    if (split == 0) {
      bF = fmax;
      while (bF > 1 && bF * a > 256) bF >>= 1;
    }
    for (int m = 1; m <= split; ++m) {
      const int per = (a + m - 1) / m;
      int F = fmax;
      while (F > 1 && F * per > 256) F >>= 1;
      const double c = m * (u / F + 2.0 * u / 256.0 + 8.0);
      if (c < bc) { bc = c; bm = m; bF = F; }
    }
    const int per = (a + bm - 1) / bm;
    for (int i = 0; i < bm; ++i) {
      const int b0 = P.lw_tbeg[k] + i * per, b1 = std::min(P.lw_tend[k], b0 + per);
      if (b0 < b1) it.push_back({P.lw_leaf[k], b0, b1, bF, u / bF + 2.0 * u / 256.0 + 8.0});
    }
  }
  std::stable_sort(it.begin(), it.end(), [](const Item& x, const Item& y) { return x.cost > y.cost; });
  std::vector<int> w(4 * std::max<size_t>(it.size(), 1), 0);
  for (size_t i = 0; i < it.size(); ++i) {
    w[4 * i] = it[i].leaf; w[4 * i + 1] = it[i].tbeg; w[4 * i + 2] = it[i].tend; w[4 * i + 3] = it[i].F;
  }
  upload(P.leaf_work, w);
  P.dt.leaf_work = reinterpret_cast<const int4*>(P.leaf_work.p);
  P.dt.n_leaf_work = (int)it.size();
  P.leaf_fmax = fmax;
  P.leaf_split = split;
  P.dt.leaf_fmax = fmax;
}

// The far rule of a precision: FP64 the surface's primary rule, FP32 its own
// (coarser) one; the transposed trees use their forward precision's.
struct OverView {
  int n_o;
  int64_t No;
  const std::vector<double>* s;
  const std::vector<double>* nu;
  const std::vector<double>* wo;
  const std::vector<double>* P;
};
template <typename T>
static OverView over_view(const lb_ctx* ctx) {
  const Surface& S = ctx->S;
  if (sizeof(T) == 4)
    return {S.o32.n_o, S.o32.No, &S.o32.s, &S.o32.nu, &S.o32.wo, &S.o32.re->P};
  return {S.n_o, S.No, &S.s, &S.nu, &S.wo, &ctx->re->P};
}

// Device state of one precision: one octree per surface, merged into a
// forest.  With `fwd` set, the transposed problem of the adjoint applies:
// the Nystrom nodes are the sources and the oversampled points the targets
// (trees of the same depths over the same points, so the same boxes), the
// mask radius moves with the oversampled point to the target side, and the
// reference matrices, corrections and translation operators are those of
// `fwd`.
template <typename T>
static void build_prec(lb_ctx* ctx, Prec<T>& P, int p, const std::vector<double>& C, const std::vector<float>& rm2f,
                       double min_leaf_side, int leaf_src, bool direct, const Prec<T>* fwd = nullptr,
                       DBuf* dev_v4 = nullptr, DBuf* dev_v3 = nullptr, DBuf* dev_vD = nullptr) {
  const Surface& S = ctx->S;
  const bool adj = fwd != nullptr;
  const OverView ov = over_view<T>(ctx);
  P.p = p;
  P.L = (p + 1) * (p + 1);
  P.n_o = ov.n_o;
  P.No = ov.No;
  P.build_leaf_src = leaf_src;
  P.min_leaf_side = min_leaf_side;
  P.direct = direct;
  // (X, nrm) are the nodes, (s, nu) the oversampled points
  const std::vector<double>& TX = adj ? *ov.s : S.X;
  const std::vector<double>& TN = adj ? *ov.nu : S.nrm;
  const std::vector<double>& SX = adj ? S.X : *ov.s;
  const std::vector<double>& SN = adj ? S.nrm : *ov.nu;
  const int64_t N = adj ? ov.No : S.N, No = adj ? S.N : ov.No;  // targets, sources of these trees
  const int ns = ctx->n_surf;
  std::vector<int64_t> toff(ns + 1), soff(ns + 1);
  for (int q = 0; q <= ns; ++q) {
    const int64_t pn = (int64_t)ctx->surf_patch[q] * ctx->n_p, po = (int64_t)ctx->surf_patch[q] * ov.n_o;
    toff[q] = adj ? po : pn;
    soff[q] = adj ? pn : po;
  }
  P.trees.assign(ns, Octree());
  for (int q = 0; q < ns; ++q) {
    const int depth_req = adj ? fwd->trees[q].depth : (direct ? 0 : -1);
    const double* tq = TX.data() + 3 * toff[q];
    const double* sq = SX.data() + 3 * soff[q];
    const int64_t nt = toff[q + 1] - toff[q], nsr = soff[q + 1] - soff[q];
    if (ctx->opts.flags & LB_HOST_OCTREE)
      P.trees[q].build(tq, nt, sq, nsr, leaf_src, adj ? 0.0 : min_leaf_side, depth_req);
    else
      P.trees[q].build_device(tq, nt, sq, nsr, leaf_src, adj ? 0.0 : min_leaf_side, depth_req);
  }
  Forest F;
  merge_forest(P.trees, toff, soff, F);
  // without a mask (FP64) the smallest positive normal value still excludes
  // coincident points
  auto rmask = [&](int64_t m) { return rm2f.empty() ? std::numeric_limits<T>::min() : (T)rm2f[m]; };
  std::vector<T> a(N), b(N), c(N), d(N), e(N), f(N), tr(adj ? N : 0);
  for (int64_t j = 0; j < N; ++j) {
    int64_t i = F.tgt_perm[j];
    a[j] = (T)TX[3 * i]; b[j] = (T)TX[3 * i + 1]; c[j] = (T)TX[3 * i + 2];
    d[j] = (T)TN[3 * i]; e[j] = (T)TN[3 * i + 1]; f[j] = (T)TN[3 * i + 2];
    if (adj) tr[j] = rmask(i);
  }
  upload(P.tx, a); upload(P.ty, b); upload(P.tz, c); upload(P.tnx, d); upload(P.tny, e); upload(P.tnz, f);
  if (adj) upload(P.trm2, tr);
  std::vector<T> sa(No), sb(No), sc(No), sd(No), se(No), sf(No), sr(No);
  for (int64_t j = 0; j < No; ++j) {
    int64_t i = F.src_perm[j];
    sa[j] = (T)SX[3 * i]; sb[j] = (T)SX[3 * i + 1]; sc[j] = (T)SX[3 * i + 2];
    sd[j] = (T)SN[3 * i]; se[j] = (T)SN[3 * i + 1]; sf[j] = (T)SN[3 * i + 2];
    sr[j] = adj ? std::numeric_limits<T>::min() : rmask(i);
  }
  upload(P.sx, sa); upload(P.sy, sb); upload(P.sz, sc); upload(P.snx, sd); upload(P.sny, se); upload(P.snz, sf);
  upload(P.rm2, sr);
  const int nb = F.nbox;
  {
    std::vector<T> cx(nb), cy(nb), cz(nb);
    for (int g = 0; g < nb; ++g) { cx[g] = (T)F.box_cen[3 * g]; cy[g] = (T)F.box_cen[3 * g + 1]; cz[g] = (T)F.box_cen[3 * g + 2]; }
    upload(P.bcx, cx); upload(P.bcy, cy); upload(P.bcz, cz);
  }
  upload(P.tgt_beg, F.tgt_beg); upload(P.tgt_end, F.tgt_end);
  upload(P.src_beg, F.src_beg); upload(P.src_end, F.src_end);
  upload(P.ulist_ptr, F.ulist_ptr); upload(P.ulist, F.ulist);
  upload(P.vlist_ptr, F.vlist_ptr); upload(P.vlist_src, F.vlist_src); upload(P.vlist_off, F.vlist_off);
  upload(P.parent, F.parent); upload(P.child, F.child); upload(P.child_src, F.child_src);
  upload(P.leaf_box, F.leaf_box); upload(P.leaf_lvl, F.leaf_lvl); upload_as<T>(P.leaf_h, F.leaf_h);
  std::vector<int> lt, ls;
  for (int l = 0; l < F.nleaf; ++l) {
    if (F.has_tgt[F.leaf_box[l]]) lt.push_back(l);
    if (F.has_src[F.leaf_box[l]]) ls.push_back(l);
  }
  // heaviest leaves first, so that the block-per-leaf kernels (P2M, leaf
  // evaluation) do not end on a tail of large leaves
  {
    auto nsrc = [&](int l) { return F.src_end[l] - F.src_beg[l]; };
    std::stable_sort(ls.begin(), ls.end(), [&](int x, int y) { return nsrc(x) > nsrc(y); });
    P.lw_leaf.clear(); P.lw_tbeg.clear(); P.lw_tend.clear(); P.lw_usrc.clear();
    for (int l : lt) {
      int64_t us = 0;
      for (int k = F.ulist_ptr[l]; k < F.ulist_ptr[l + 1]; ++k) us += nsrc(F.ulist[k]);
      P.lw_leaf.push_back(l);
      P.lw_tbeg.push_back(F.tgt_beg[l]);
      P.lw_tend.push_back(F.tgt_end[l]);
      P.lw_usrc.push_back(us);
    }
  }
  upload(P.leaf_tgt, lt); upload(P.leaf_src, ls);
  std::vector<int> lsv, lsp(1, 0), ltv, ltp(1, 0);
  for (int l = 0; l <= F.depth; ++l) {
    for (int g = 0; g < nb; ++g) {
      if (F.box_level[g] != l) continue;
      if (F.has_src[g]) lsv.push_back(g);
      if (F.has_tgt[g]) ltv.push_back(g);
    }
    lsp.push_back((int)lsv.size());
    ltp.push_back((int)ltv.size());
  }
  upload(P.lev_src, lsv); upload(P.lev_src_ptr, lsp); upload(P.lev_tgt, ltv); upload(P.lev_tgt_ptr, ltp);
  // user-order maps
  std::vector<int> tp(N), sp(No);
  for (int64_t i = 0; i < N; ++i) tp[i] = (int)F.tgt_pos[i];
  for (int64_t i = 0; i < No; ++i) sp[i] = (int)F.src_pos[i];
  upload(P.tgt_pos, tp); upload(P.src_pos, sp);
  // node data and corrections do not depend on the tree: a rebuild (empty C)
  // keeps them where they are
  // (dev_v4, dev_v3, dev_vD: corrections already on the device in the packed
  // layouts, taken over)
  if (!adj && (!C.empty() || dev_v4)) {
    upload_as<T>(P.P, *ov.P);
    upload_as<T>(P.wo, *ov.wo);
    upload_as<T>(P.nrm, S.nrm);
    upload_as<T>(P.H, S.H);
    if (dev_v4) {
      std::swap(P.vals4.p, dev_v4->p); std::swap(P.vals4.bytes, dev_v4->bytes);
      std::swap(P.vals3.p, dev_v3->p); std::swap(P.vals3.bytes, dev_v3->bytes);
      std::swap(P.valsD.p, dev_vD->p); std::swap(P.valsD.bytes, dev_vD->bytes);
    } else {
      std::vector<T> v4, v3, vD;
      pack_vals(C, (int64_t)C.size() / NKER, v4, v3, vD);
      upload(P.vals4, v4);
      upload(P.vals3, v3);
      upload(P.valsD, vD);
    }
  }
  // translations (level independent: built once)
  if (F.depth >= 2 && !adj && !P.m2l.p) {
    Translations trn;
    trn.build(p);
    big_vector<T> m;
    transpose_blocks(trn.m2m, 8, P.L, P.L, m); upload(P.m2m, m);
    transpose_blocks(trn.l2l, 8, P.L, P.L, m); upload(P.l2l, m);
    transpose_blocks(trn.m2l, 343, P.L, P.L, m); upload(P.m2l, m);
    transpose_blocks(trn.dgrad, 3, p * p, P.L, m); upload(P.dgrad, m);
    transpose_blocks(trn.dhess, 6, (p - 1) * (p - 1), P.L, m); upload(P.dhess, m);
  }
  // batched translation plans over all trees
  if (F.depth >= 2) {
    size_t maxcols = 1;
    {
      std::vector<Triple> trp;
      std::vector<int> boxes;
      std::vector<double> scale;
      for (int g = 0; g < nb; ++g) {
        if (F.box_level[g] < 2 || !F.has_tgt[g]) continue;
        boxes.push_back(g);
        scale.push_back(F.box_scale[g]);
        for (int v = F.vlist_ptr[g]; v < F.vlist_ptr[g + 1]; ++v) trp.push_back({F.vlist_off[v], g, F.vlist_src[v]});
      }
      const std::vector<int> lo = m2l_orders(p, sizeof(T) == 4 ? ctx->opts.m2l_trunc32 : ctx->opts.m2l_trunc64);
      // algorithmic M2L work per density: a pair at offset o multiplies its
      // leading lo[o] coefficients by the leading lo[o] x lo[o] block
      P.m2l_flops = 0;
      for (const Triple& q : trp) {
        const double l = lo.empty() ? P.L : lo[q.mat];
        P.m2l_flops += 2.0 * l * l;
      }
      // parts of at most cap pairs (in (offset, target) order), so that the
      // column scratch of the deep trees of the N ~ 1M surfaces stays within
      // M2L_Y_BUDGET; the first part writes every target box, the others add
      std::stable_sort(trp.begin(), trp.end(), [](const Triple& a, const Triple& b) {
        return a.mat != b.mat ? a.mat < b.mat : a.tgt < b.tgt;
      });
      const size_t cap = std::max<size_t>(4096, M2L_Y_BUDGET / (sizeof(T) * (size_t)nemax<T>() * P.L));
      const size_t nparts = std::max<size_t>(1, (trp.size() + cap - 1) / cap);
      P.m2l_pb.clear();
      P.m2l_pl.clear();
      for (size_t q = 0; q < nparts; ++q) {
        const size_t b0 = trp.size() * q / nparts, b1 = trp.size() * (q + 1) / nparts;
        std::vector<Triple> part(trp.begin() + b0, trp.begin() + b1);
        std::vector<int> pboxes;
        std::vector<double> pscale;
        if (q == 0) {
          pboxes = boxes;
          pscale = scale;
        } else {
          std::vector<char> has(nb, 0);
          for (const Triple& t3 : part) has[t3.tgt] = 1;
          for (size_t b = 0; b < boxes.size(); ++b)
            if (has[boxes[b]]) { pboxes.push_back(boxes[b]); pscale.push_back(scale[b]); }
        }
        P.m2l_pb.emplace_back(new PlanBuf());
        maxcols = std::max(maxcols, build_plan(*P.m2l_pb.back(), part, pboxes, pscale, true, q > 0, nb, P.L,
                                               nemax<T>(), lo));
        P.m2l_pl.push_back(P.m2l_pb.back()->pl);
      }
    }
    P.m2m_pb.clear();
    P.l2l_pb.clear();
    P.m2m_pl.assign(F.depth + 1, GemmPlan());
    P.l2l_pl.assign(F.depth + 1, GemmPlan());
    for (int l = 0; l <= F.depth; ++l) {
      P.m2m_pb.emplace_back(new PlanBuf());
      P.l2l_pb.emplace_back(new PlanBuf());
    }
    for (int l = 2; l < F.depth; ++l) {  // M2M into level l from level l+1
      std::vector<Triple> trp;
      std::vector<int> boxes;
      for (int g = 0; g < nb; ++g) {
        // the leaves of shallower trees on this level keep their P2M multipoles
        if (F.box_level[g] != l || !F.has_src[g] || F.box_level[g] == F.tree_depth[g]) continue;
        boxes.push_back(g);
        for (int c = 0; c < 8; ++c) {
          const int ch = F.child[(size_t)g * 8 + c];
          if (ch >= 0 && F.has_src[ch]) trp.push_back({c, g, ch});
        }
      }
      maxcols = std::max(maxcols, build_plan(*P.m2m_pb[l], trp, boxes, {}, false, false, nb, P.L, nemax<T>(), {}, true));
      P.m2m_pl[l] = P.m2m_pb[l]->pl;
    }
    for (int l = 3; l <= F.depth; ++l) {  // L2L into level l from level l-1
      std::vector<Triple> trp;
      std::vector<int> boxes;
      for (int g = 0; g < nb; ++g) {
        if (F.box_level[g] != l || !F.has_tgt[g]) continue;
        const int pg = F.parent[g];
        int oct = -1;
        for (int c = 0; c < 8; ++c)
          if (F.child[(size_t)pg * 8 + c] == g) oct = c;
        if (oct < 0) fail(LB_EINVAL, "octree: box %d missing from its parent", g);
        boxes.push_back(g);
        trp.push_back({oct, g, pg});
      }
      maxcols = std::max(maxcols, build_plan(*P.l2l_pb[l], trp, boxes, {}, false, true, nb, P.L, nemax<T>(), {}, true));
      P.l2l_pl[l] = P.l2l_pb[l]->pl;
    }
    P.Y.alloc_exact(sizeof(T) * maxcols * nemax<T>() * (size_t)P.L);
  }
  // device tree descriptor
  DevTree<T>& D = P.dt;
  D.tx = dptr<T>(P.tx); D.ty = dptr<T>(P.ty); D.tz = dptr<T>(P.tz);
  D.tnx = dptr<T>(P.tnx); D.tny = dptr<T>(P.tny); D.tnz = dptr<T>(P.tnz);
  D.sx = dptr<T>(P.sx); D.sy = dptr<T>(P.sy); D.sz = dptr<T>(P.sz);
  D.snx = dptr<T>(P.snx); D.sny = dptr<T>(P.sny); D.snz = dptr<T>(P.snz);
  D.rm2 = dptr<T>(P.rm2);
  D.trm2 = adj ? dptr<T>(P.trm2) : nullptr;
  D.bcx = dptr<T>(P.bcx); D.bcy = dptr<T>(P.bcy); D.bcz = dptr<T>(P.bcz);
  D.tgt_beg = dptr<int>(P.tgt_beg); D.tgt_end = dptr<int>(P.tgt_end);
  D.src_beg = dptr<int>(P.src_beg); D.src_end = dptr<int>(P.src_end);
  D.ulist_ptr = dptr<int>(P.ulist_ptr); D.ulist = dptr<int>(P.ulist);
  D.vlist_ptr = dptr<int>(P.vlist_ptr); D.vlist_src = dptr<int>(P.vlist_src); D.vlist_off = dptr<int>(P.vlist_off);
  D.parent = dptr<int>(P.parent); D.child = dptr<int>(P.child); D.child_src = dptr<int>(P.child_src);
  D.leaf_tgt_list = dptr<int>(P.leaf_tgt); D.n_leaf_tgt = (int)lt.size();
  make_leaf_work<T>(P, P.leaf_fmax, P.leaf_split);
  D.leaf_src_list = dptr<int>(P.leaf_src); D.n_leaf_src = (int)ls.size();
  D.lev_box_src = dptr<int>(P.lev_src); D.lev_box_src_ptr = dptr<int>(P.lev_src_ptr);
  D.lev_box_tgt = dptr<int>(P.lev_tgt); D.lev_box_tgt_ptr = dptr<int>(P.lev_tgt_ptr);
  D.leaf_box = dptr<int>(P.leaf_box); D.leaf_lvl = dptr<int>(P.leaf_lvl); D.leaf_h = dptr<T>(P.leaf_h);
  D.depth = F.depth;
  D.nbox = nb;
  D.p = p;
  D.L = P.L;
  const Prec<T>& TRs = adj ? *fwd : P;  // owner of the translation operators
  D.m2m = dptr<T>(TRs.m2m); D.l2l = dptr<T>(TRs.l2l); D.m2l = dptr<T>(TRs.m2l);
  D.dgradT = dptr<T>(TRs.dgrad); D.dhessT = dptr<T>(TRs.dhess);
  D.m2l_plan = F.depth >= 2 ? P.m2l_pl.data() : nullptr;
  D.m2l_parts = F.depth >= 2 ? (int)P.m2l_pl.size() : 0;
  D.m2m_plan = F.depth >= 2 ? P.m2m_pl.data() : nullptr;
  D.l2l_plan = F.depth >= 2 ? P.l2l_pl.data() : nullptr;
  D.Y = P.Y.p;
  D.p2m_H = nullptr;
  D.p2m_D = nullptr;
  D.leaf_fmax = P.leaf_fmax;
  const bool overlap = !(ctx->opts.flags & LB_NO_OVERLAP);
  if (overlap && !ctx->side_stream) {
    HIPTRY(hipStreamCreateWithFlags(&ctx->side_stream, hipStreamNonBlocking));
    HIPTRY(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    HIPTRY(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
  }
  D.side = overlap ? ctx->side_stream : nullptr;
  D.fork_ev = ctx->ev_fork;
  D.join_ev = ctx->ev_join;
  D.fork_late = P.fork_late;
  D.near_grid = P.near_grid;
  D.corr_early = P.corr_early;
  // P2M tables (the geometry is fixed, so the leaf harmonics of every
  // source can be kept): built on the device when both fit in a quarter of
  // the free memory and under P2M_TABLE_MAX bytes
  if (F.depth >= 2 && !adj && !(ctx->opts.flags & LB_NO_P2M_TABLES)) {
    const size_t bytes = 2 * sizeof(T) * (size_t)No * P.L;
    size_t fr = 0, tot = 0;
    HIPTRY(hipMemGetInfo(&fr, &tot));
    if (bytes <= P2M_TABLE_MAX && (bytes <= fr / 4 || P.p2m_H.bytes >= bytes / 2)) {
      P.p2m_H.alloc(bytes / 2);
      P.p2m_D.alloc(bytes / 2);
      launch_p2m_tables<T>(D, dptr<T>(P.p2m_H), dptr<T>(P.p2m_D), nullptr);
      HIPTRY(hipDeviceSynchronize());
      D.p2m_H = dptr<T>(P.p2m_H);
      D.p2m_D = dptr<T>(P.p2m_D);
    }
  }
}

constexpr int CHUNK_GRAD = 8;
constexpr int CHUNK_A3T = 4;  // densities per transposed A3 traversal (two expansions each)

// Per-call workspace of the gradient apply for `chunk` densities per
// traversal: strengths, multipole and local expansions, derived leaf
// expansions, FMM outputs and the early correction sums.
template <typename T>
struct ApplyWs {
  T *str = nullptr, *M = nullptr, *Lc = nullptr, *D = nullptr, *fmm = nullptr, *corr = nullptr;
};

// element counts of the ApplyWs buffers for traversals of at most `chunk`
// densities (gradient or potential applies: one expansion per density; A3:
// three per density for at most chunk_a3 densities)
template <typename T>
static void ws_counts(const lb_ctx* ctx, const Prec<T>& P, int chunk, size_t cnt[6]) {
  const int c3 = std::min(chunk, chunk_a3<T>());
  const size_t ne = (size_t)std::max(chunk, 3 * c3);
  const int64_t dpd = std::max({(int64_t)chunk * leaf_d_stride<T>(FMM_GRAD, P.p),
                                (int64_t)chunk * leaf_d_stride<T>(FMM_POT, P.p),
                                (int64_t)c3 * leaf_d_stride<T>(FMM_A3B, P.p),
                                (int64_t)c3 * leaf_d_stride<T>(FMM_ADJ, P.p)});
  cnt[0] = (size_t)P.No * 2 * chunk;
  cnt[1] = (size_t)P.dt.nbox * ne * P.L;
  cnt[2] = cnt[1];
  cnt[3] = (size_t)std::max(P.dt.n_leaf_work, 1) * (size_t)dpd;
  cnt[4] = (size_t)ctx->N * 4 * chunk;
  cnt[5] = (size_t)ctx->N * 4 * chunk;
}

template <typename T>
static void ensure_ws(lb_ctx* ctx, Prec<T>& P, int chunk) {
  chunk = std::max(chunk, chunk_fwd<T>());
  if (P.ws_rhs >= chunk) return;
  const int64_t N = ctx->N;
  size_t cnt[6];
  ws_counts<T>(ctx, P, chunk, cnt);
  // exact sizes: a rebuild with a shallower tree gives back what a deeper
  // one took
  // (the A2 apply keeps two strength layouts, 2 + 4 values per density)
  P.str.alloc_exact(sizeof(T) * std::max(cnt[0], (size_t)P.No * 6 * std::min(chunk, chunk_a3<T>())));
  P.M.alloc_exact(sizeof(T) * cnt[1]);
  P.Lc.alloc_exact(sizeof(T) * cnt[2]);
  P.D.alloc_exact(sizeof(T) * std::max<size_t>(cnt[3], 1));
  P.fmm.alloc_exact(sizeof(T) * cnt[4]);
  P.corr.alloc_exact(sizeof(T) * cnt[5]);
  P.mu.alloc(sizeof(T) * (size_t)N * 2 * chunk);
  P.y2.alloc(sizeof(T) * (size_t)N * chunk);
  ctx->seg_scal.alloc(sizeof(double) * (size_t)chunk * ctx->n_surf + 8);
  P.ws_rhs = chunk;
  // per-block partial sums: the A3 combine (4 per row block) and the GMRES
  // dot products (256 blocks per basis vector)
  ctx->partial.alloc(sizeof(double) * std::max<size_t>((size_t)4 * ((N + 3) / 4) + 64,
                                                       (size_t)256 * (ctx->opts.max_iter + 2)));
}

template <typename T>
static ApplyWs<T> ctx_ws(Prec<T>& P) {
  ApplyWs<T> w;
  w.str = dptr<T>(P.str); w.M = dptr<T>(P.M); w.Lc = dptr<T>(P.Lc);
  w.D = dptr<T>(P.D); w.fmm = dptr<T>(P.fmm); w.corr = dptr<T>(P.corr);
  return w;
}

template <typename T>
static void apply_gradS_t(lb_ctx* ctx, Prec<T>& P, int nd, const T* sigma, T* pot, T* grad, T* dSdn, T* surf,
                          hipStream_t st, PhaseTimer* tm = nullptr, const ApplyWs<T>* ws = nullptr) {
  ApplyWs<T> W;
  if (ws) {
    W = *ws;
  } else {
    ensure_ws(ctx, P, CHUNK_GRAD);
    W = ctx_ws(P);
  }
  const int64_t N = ctx->N, No = P.No;
  // corr_early: the correction sums need only sigma, so they run first on
  // the side stream (ahead of the near field, which launch_fmm forks there
  // and joins back), and a light final step adds the far sums
  const bool early = P.corr_early && P.dt.side && P.dt.depth >= 2 && !tm;
  for (int d0 = 0; d0 < nd; d0 += chunk_fwd<T>()) {
    const int c = std::min(chunk_fwd<T>(), nd - d0);
    if (early) {
      HIPTRY(hipEventRecord(P.dt.fork_ev, st));
      HIPTRY(hipStreamWaitEvent(P.dt.side, P.dt.fork_ev, 0));
      launch_corr_grad<T>(c, N, ctx->n_p, dptr<int64_t>(ctx->row_ptr), dptr<int>(ctx->patch), dptr<T>(P.vals4),
                          sigma + (int64_t)d0 * N, W.corr, P.dt.side);
    }
    if (tm) tm->mark(PH_STR, st);
    launch_strengths<T>(sigma + (int64_t)d0 * N, c, N, ctx->NP, ctx->n_p, P.n_o, dptr<T>(P.P), dptr<T>(P.wo),
                        dptr<int>(P.src_pos), No, W.str, st);
    if (tm) tm->mark(PH_P2M, st);
    launch_fmm<T>(P.dt, FMM_GRAD, c, W.str, W.M, W.Lc, W.D, W.fmm, N, No, st, tm);
    if (tm) tm->mark(PH_COMB, st);
    if (early)
      launch_combine_grad_fin<T>(c, N, W.fmm, W.corr, dptr<int>(P.tgt_pos), dptr<T>(P.nrm),
                                 pot ? pot + (int64_t)d0 * N : nullptr, grad + (int64_t)d0 * 3 * N,
                                 dSdn ? dSdn + (int64_t)d0 * N : nullptr, surf ? surf + (int64_t)d0 * 3 * N : nullptr,
                                 st);
    else
      launch_combine_grad<T>(c, N, ctx->n_p, dptr<int64_t>(ctx->row_ptr), dptr<int>(ctx->patch), dptr<T>(P.vals4),
                             sigma + (int64_t)d0 * N, W.fmm, dptr<int>(P.tgt_pos), dptr<T>(P.nrm),
                             pot ? pot + (int64_t)d0 * N : nullptr, grad + (int64_t)d0 * 3 * N,
                             dSdn ? dSdn + (int64_t)d0 * N : nullptr, surf ? surf + (int64_t)d0 * 3 * N : nullptr, st);
    if (tm) tm->mark(PH_N, st);
  }
}

// S alone (potential-only FMM), chunk_fwd densities per traversal
template <typename T>
static void apply_S_t(lb_ctx* ctx, Prec<T>& P, int nd, const T* sigma, T* pot, hipStream_t st) {
  ensure_ws(ctx, P, CHUNK_GRAD);
  const int64_t N = ctx->N, No = P.No;
  for (int d0 = 0; d0 < nd; d0 += chunk_fwd<T>()) {
    const int c = std::min(chunk_fwd<T>(), nd - d0);
    launch_strengths<T>(sigma + (int64_t)d0 * N, c, N, ctx->NP, ctx->n_p, P.n_o, dptr<T>(P.P), dptr<T>(P.wo),
                        dptr<int>(P.src_pos), No, dptr<T>(P.str), st);
    launch_fmm<T>(P.dt, FMM_POT, c, dptr<T>(P.str), dptr<T>(P.M), dptr<T>(P.Lc), dptr<T>(P.D), dptr<T>(P.fmm), N, No,
                  st);
    launch_combine_pot<T>(c, N, ctx->n_p, dptr<int64_t>(ctx->row_ptr), dptr<int>(ctx->patch), dptr<T>(P.vals3),
                          sigma + (int64_t)d0 * N, dptr<T>(P.fmm), dptr<int>(P.tgt_pos), pot + (int64_t)d0 * N, st);
  }
}

// A3 (Section 4.3) for nd densities, chunk_a3 per traversal: the second FMM
// carries three expansions per density (charges mu1, mu2 and dipole mu2 nu).

template <typename T>
static void apply_A3_t(lb_ctx* ctx, Prec<T>& P, int nd, const T* tau, T* out, hipStream_t st) {
  ensure_ws(ctx, P, CHUNK_GRAD);
  const int64_t N = ctx->N, No = P.No;
  T* mu = dptr<T>(P.mu);  // [c][mu1; mu2]
  for (int d0 = 0; d0 < nd; d0 += chunk_a3<T>()) {
    const int c = std::min(chunk_a3<T>(), nd - d0);
    const T* td = tau + (int64_t)d0 * N;
    launch_strengths<T>(td, c, N, ctx->NP, ctx->n_p, P.n_o, dptr<T>(P.P), dptr<T>(P.wo), dptr<int>(P.src_pos), No,
                        dptr<T>(P.str), st);
    launch_fmm<T>(P.dt, FMM_GRAD, c, dptr<T>(P.str), dptr<T>(P.M), dptr<T>(P.Lc), dptr<T>(P.D), dptr<T>(P.fmm), N, No, st);
    launch_combine_a3a<T>(c, N, ctx->n_p, dptr<int64_t>(ctx->row_ptr), dptr<int>(ctx->patch), dptr<T>(P.vals3), td,
                          dptr<T>(P.fmm), dptr<int>(P.tgt_pos), dptr<T>(P.nrm), mu, mu + N, 2 * N, st);
    launch_strengths<T>(mu, 2 * c, N, ctx->NP, ctx->n_p, P.n_o, dptr<T>(P.P), dptr<T>(P.wo), dptr<int>(P.src_pos),
                        No, dptr<T>(P.str), st);
    launch_fmm<T>(P.dt, FMM_A3B, c, dptr<T>(P.str), dptr<T>(P.M), dptr<T>(P.Lc), dptr<T>(P.D), dptr<T>(P.fmm), N, No, st);
    launch_combine_a3b<T>(c, N, ctx->n_p, dptr<int64_t>(ctx->row_ptr), dptr<int>(ctx->patch), dptr<T>(P.vals3), td, mu,
                          mu + N, 2 * N, dptr<T>(P.fmm), dptr<int>(P.tgt_pos), dptr<T>(P.H), dptr<double>(ctx->w),
                          ctx->n_surf, dptr<int64_t>(ctx->node_off), dptr<int>(ctx->node_surf),
                          dptr<double>(ctx->inv_area), out + (int64_t)d0 * N, dptr<T>(P.y2),
                          dptr<double>(ctx->seg_scal), st);
  }
}

// A2 (Section 4.2, eq. ie-dis1) for nd densities, chunk_a3 per traversal:
// the first pass is the A3 second pass's FMM (charges 0 and tau, dipole
// tau nu: S, S', S''+D' of tau) plus a dipole-potential FMM (D tau); then
// mu1 = D tau, mu2 = -(S''+D'+2HS') tau + W S tau, and one FMM of the
// charge mu2 and dipole mu1 nu gives A2 tau = -tau/4 + S mu2 + D mu1 (the
// D^2 term of eq. ie-dis1 is D mu1 with a plus sign).
template <typename T>
static void a2_ws(lb_ctx* ctx, Prec<T>& P) {
  ensure_ws(ctx, P, CHUNK_GRAD);
  const int cmax = chunk_a3<T>();
  if ((size_t)6 * cmax * P.No > P.str.bytes / sizeof(T) || (size_t)2 * cmax * ctx->N > P.mu.bytes / sizeof(T))
    fail(LB_EINVAL, "A2 workspace too small");
  P.a2s.alloc(sizeof(T) * (size_t)P.No * 2 * cmax);
}

template <typename T>
static void apply_A2_t(lb_ctx* ctx, Prec<T>& P, int nd, const T* tau, T* out, hipStream_t st) {
  a2_ws<T>(ctx, P);
  const int64_t N = ctx->N, No = P.No;
  const int cmax = chunk_a3<T>();
  T* c1 = dptr<T>(P.a2s);
  T* c2 = c1 + (size_t)cmax * No;
  T* s3 = dptr<T>(P.str);                  // [c][2][No]
  T* sd = s3 + (size_t)2 * cmax * No;      // [c][4][No]
  T* mu1 = dptr<T>(P.mu);
  T* mu2 = mu1 + (size_t)cmax * N;
  T* fd = dptr<T>(P.corr);
  for (int d0 = 0; d0 < nd; d0 += cmax) {
    const int c = std::min(cmax, nd - d0);
    const T* td = tau + (int64_t)d0 * N;
    launch_strengths<T>(td, c, N, ctx->NP, ctx->n_p, P.n_o, dptr<T>(P.P), dptr<T>(P.wo), dptr<int>(P.src_pos), No,
                        c1, st);
    launch_a2_str1<T>(c, No, c1, dptr<T>(P.snx), dptr<T>(P.sny), dptr<T>(P.snz), s3, sd, st);
    launch_fmm<T>(P.dt, FMM_A3B, c, s3, dptr<T>(P.M), dptr<T>(P.Lc), dptr<T>(P.D), dptr<T>(P.fmm), N, No, st);
    launch_fmm<T>(P.dt, FMM_ADJ, c, sd, dptr<T>(P.M), dptr<T>(P.Lc), dptr<T>(P.D), fd, N, No, st);
    launch_combine_a2a<T>(c, N, ctx->n_p, dptr<int64_t>(ctx->row_ptr), dptr<int>(ctx->patch), dptr<T>(P.vals3),
                          dptr<T>(P.valsD), td, dptr<T>(P.fmm), fd, dptr<int>(P.tgt_pos), dptr<T>(P.H), mu1, mu2,
                          dptr<T>(P.y2), st);
    // W S tau (the average over each surface) onto mu2
    launch_seg_dot<T>(c, ctx->n_surf, N, dptr<int64_t>(ctx->node_off), dptr<T>(P.y2), dptr<double>(ctx->w),
                      dptr<double>(ctx->inv_area), dptr<double>(ctx->seg_scal), st);
    launch_seg_axpy<T>(c, ctx->n_surf, N, dptr<int>(ctx->node_surf), mu2, 1.0, nullptr,
                       dptr<double>(ctx->seg_scal), mu2, st);
    launch_strengths<T>(mu1, c, N, ctx->NP, ctx->n_p, P.n_o, dptr<T>(P.P), dptr<T>(P.wo), dptr<int>(P.src_pos), No,
                        c1, st);
    launch_strengths<T>(mu2, c, N, ctx->NP, ctx->n_p, P.n_o, dptr<T>(P.P), dptr<T>(P.wo), dptr<int>(P.src_pos), No,
                        c2, st);
    launch_a2_str2<T>(c, No, c1, c2, dptr<T>(P.snx), dptr<T>(P.sny), dptr<T>(P.snz), sd, st);
    launch_fmm<T>(P.dt, FMM_ADJ, c, sd, dptr<T>(P.M), dptr<T>(P.Lc), dptr<T>(P.D), fd, N, No, st);
    launch_combine_a2b<T>(c, N, ctx->n_p, dptr<int64_t>(ctx->row_ptr), dptr<int>(ctx->patch), dptr<T>(P.vals3),
                          dptr<T>(P.valsD), td, mu1, mu2, fd, dptr<int>(P.tgt_pos), out + (int64_t)d0 * N, st);
  }
}

// A1 (Section 4.1, eq. ie-dis0) for nd densities: S tau and grad_Gamma S tau
// (one gradient apply), mu = grad_Gamma S tau as three densities, the
// gradient apply of mu, and div S[mu] = sum_l (d_l S)[mu_l] plus
// W(S tau) S[1] (S[1] computed once per precision).
template <typename T>
static void apply_A1_t(lb_ctx* ctx, Prec<T>& P, DBuf& phi0, int nd, const T* tau, T* out, hipStream_t st) {
  const int64_t N = ctx->N;
  const int nsf = ctx->n_surf;
  if (!phi0.p) {
    std::vector<T> one((size_t)N, (T)1);
    DBuf d1;
    upload(d1, one);
    phi0.alloc(sizeof(T) * N);
    apply_S_t<T>(ctx, P, 1, dptr<T>(d1), dptr<T>(phi0), st);
    HIPTRY(hipStreamSynchronize(st));
  }
  ctx->a1_pot.alloc(sizeof(T) * (size_t)nd * N);
  ctx->a1_g1.alloc(sizeof(T) * (size_t)nd * N * 3);
  ctx->a1_surf.alloc(sizeof(T) * (size_t)nd * N * 3);
  ctx->a1_mu.alloc(sizeof(T) * (size_t)nd * N * 3);
  ctx->a1_g2.alloc(sizeof(T) * (size_t)nd * N * 9);
  ctx->a1_eta.alloc(sizeof(double) * (size_t)nd * nsf);
  T* pot = dptr<T>(ctx->a1_pot);
  apply_gradS_t<T>(ctx, P, nd, tau, pot, dptr<T>(ctx->a1_g1), nullptr, dptr<T>(ctx->a1_surf), st);
  HIPTRY(launch_a1_split<T>(N, nd, dptr<T>(ctx->a1_surf), dptr<T>(ctx->a1_mu), st));
  apply_gradS_t<T>(ctx, P, 3 * nd, dptr<T>(ctx->a1_mu), nullptr, dptr<T>(ctx->a1_g2), nullptr, nullptr, st);
  launch_seg_dot<T>(nd, nsf, N, dptr<int64_t>(ctx->node_off), pot, dptr<double>(ctx->w), dptr<double>(ctx->inv_area),
                    dptr<double>(ctx->a1_eta), st);
  HIPTRY(launch_a1_finish<T>(N, nd, nsf, dptr<int>(ctx->node_surf), dptr<T>(ctx->a1_g2), dptr<double>(ctx->a1_eta),
                             dptr<T>(phi0), out, st));
}

// ---------------------------------------------------------------------------
// Adjoint applies: sigma_bar = S^T gpot + (grad S)^T ggrad + S'^T gdSdn +
// (grad_Gamma S)^T gsurf, the exact transposes of the discrete operators of
// lb_apply_gradS (far sum, mask and corrections of the same precision), the
// far part through the FMM on the transposed tree.
// ---------------------------------------------------------------------------
template <typename T>
static void ensure_adjoint(lb_ctx* ctx, Prec<T>& F, Prec<T>& A, bool& built) {
  if (!ctx->csr_t_built) {
    const Surface& S = ctx->S;
    std::vector<int64_t> cp(ctx->NP + 1, 0), cb;
    std::vector<int> cr;
    for (int32_t pt : S.near_patch) cp[pt + 1]++;
    for (int l = 0; l < ctx->NP; ++l) cp[l + 1] += cp[l];
    cr.resize(S.near_patch.size());
    cb.resize(S.near_patch.size());
    std::vector<int64_t> fill(cp.begin(), cp.end() - 1);
    for (int64_t i = 0; i < ctx->N; ++i)
      for (int64_t b = S.near_ptr[i]; b < S.near_ptr[i + 1]; ++b) {
        const int64_t e = fill[S.near_patch[b]]++;
        cr[e] = (int)i;
        cb[e] = b;
      }
    upload(ctx->cptr, cp);
    upload(ctx->crow, cr);
    upload(ctx->cblk, cb);
    ctx->csr_t_built = true;
  }
  if (built) return;
  const bool fp32 = sizeof(T) == 4;
  build_prec<T>(ctx, A, F.p, std::vector<double>(), fp32 ? ctx->rm2f : std::vector<float>(), 0.0,
                ctx->opts.leaf_src, false, &F);
  const int nb = A.dt.nbox, L = A.L, p = A.p, c = CHUNK_GRAD;
  A.str.alloc(sizeof(T) * (size_t)ctx->N * 4 * c);
  A.M.alloc(sizeof(T) * (size_t)nb * c * L);
  A.Lc.alloc(sizeof(T) * (size_t)nb * c * L);
  // leaf workspace of the transposed traversals: FMM_ADJ with up to
  // CHUNK_GRAD densities, FMM_ADJ3 with up to CHUNK_A3T
  const int64_t dpd = std::max({(int64_t)c * leaf_d_stride<T>(FMM_ADJ, p),
                                (int64_t)CHUNK_A3T * leaf_d_stride<T>(FMM_ADJ3, p), (int64_t)1});
  A.D.alloc(sizeof(T) * (size_t)std::max(A.dt.n_leaf_work, 1) * (size_t)dpd);
  A.fmm.alloc(sizeof(T) * (size_t)F.No * c);
  HIPTRY(hipDeviceSynchronize());
  built = true;
}

template <typename T>
static void apply_adj_t(lb_ctx* ctx, Prec<T>& F, Prec<T>& A, bool& built, int nd, const T* gpot, const T* ggrad,
                        const T* gdSdn, const T* gsurf, T* sbar, hipStream_t st) {
  ensure_adjoint<T>(ctx, F, A, built);
  const int64_t N = ctx->N, No = F.No;
  ctx->g4.alloc(sizeof(T) * (size_t)N * 4 * CHUNK_GRAD);
  for (int d0 = 0; d0 < nd; d0 += CHUNK_GRAD) {
    const int c = std::min(CHUNK_GRAD, nd - d0);
    launch_adj_strengths<T>(c, N, gpot ? gpot + (int64_t)d0 * N : nullptr, ggrad ? ggrad + (int64_t)d0 * 3 * N : nullptr,
                            gdSdn ? gdSdn + (int64_t)d0 * N : nullptr, gsurf ? gsurf + (int64_t)d0 * 3 * N : nullptr,
                            dptr<T>(F.nrm), dptr<int>(A.src_pos), dptr<T>(A.str), dptr<T>(ctx->g4), st);
    // transposed tree: targets are the No oversampled points, sources the N nodes
    launch_fmm<T>(A.dt, FMM_ADJ, c, dptr<T>(A.str), dptr<T>(A.M), dptr<T>(A.Lc), dptr<T>(A.D), dptr<T>(A.fmm), No,
                  N, st);
    launch_adj_combine<T>(c, ctx->NP, ctx->n_p, F.n_o, N, No, dptr<T>(F.P), dptr<T>(F.wo), dptr<T>(A.fmm),
                          dptr<int>(A.tgt_pos), dptr<int64_t>(ctx->cptr), dptr<int>(ctx->crow),
                          dptr<int64_t>(ctx->cblk), dptr<T>(F.vals4), dptr<T>(ctx->g4), sbar + (int64_t)d0 * N, st);
  }
}

// ---------------------------------------------------------------------------
// Kernel-position derivative of S: X_bar = d<gbar, S sigma>/dX with the nodes
// and the far-rule points s = P X moving, weights, oversampled density and
// corrections fixed.  Two gradient FMMs without the near mask: grad phi at
// the nodes (forward tree, strengths w^over P sigma) and grad psi at the
// oversampled points (transposed tree, charges gbar at the nodes).
// ---------------------------------------------------------------------------
template <typename T>
static void apply_S_xbar_t(lb_ctx* ctx, Prec<T>& F, Prec<T>& A, bool& built, int nd, const T* sigma, const T* gbar,
                           T* xbar, hipStream_t st) {
  ensure_ws(ctx, F, CHUNK_GRAD);
  ensure_adjoint<T>(ctx, F, A, built);
  const int64_t N = ctx->N, No = F.No;
  if (!F.rm2_none.p) {
    upload(F.rm2_none, std::vector<T>((size_t)No, std::numeric_limits<T>::min()));
    A.fmm4.alloc(sizeof(T) * (size_t)No * 4 * CHUNK_GRAD);
  }
  DevTree<T> Fu = F.dt;
  Fu.rm2 = dptr<T>(F.rm2_none);
  HIPTRY(hipMemsetAsync(xbar, 0, sizeof(T) * 3 * (size_t)N, st));
  for (int d0 = 0; d0 < nd; d0 += CHUNK_GRAD) {
    const int c = std::min(CHUNK_GRAD, nd - d0);
    const T* sd = sigma + (int64_t)d0 * N;
    const T* gd = gbar + (int64_t)d0 * N;
    launch_strengths<T>(sd, c, N, ctx->NP, ctx->n_p, F.n_o, dptr<T>(F.P), dptr<T>(F.wo), dptr<int>(F.src_pos), No,
                        dptr<T>(F.str), st);
    launch_fmm<T>(Fu, FMM_GRAD, c, dptr<T>(F.str), dptr<T>(F.M), dptr<T>(F.Lc), dptr<T>(F.D), dptr<T>(F.fmm), N, No,
                  st);
    // transposed tree: targets are the No oversampled points, sources the N nodes
    launch_scatter_perm<T>(c, N, gd, dptr<int>(A.src_pos), dptr<T>(A.str), st);
    launch_fmm<T>(A.dt, FMM_GRAD, c, dptr<T>(A.str), dptr<T>(A.M), dptr<T>(A.Lc), dptr<T>(A.D), dptr<T>(A.fmm4), No,
                  N, st);
    launch_xbar_S<T>(c, ctx->NP, ctx->n_p, F.n_o, N, No, dptr<T>(F.P), dptr<T>(F.str), dptr<int>(F.src_pos),
                     dptr<T>(F.fmm), dptr<int>(F.tgt_pos), gd, dptr<T>(A.fmm4), dptr<int>(A.tgt_pos), xbar, st);
  }
}

// ---------------------------------------------------------------------------
// Autotuner: the depth of every octree (through the mean number of
// oversampled points per leaf, leaf_src) and the most lanes per target of
// the leaf kernel (leaf_fmax), chosen by timing the gradient apply with HIP
// events.  A rebuild keeps the corrections and node data, and drops what
// depends on the trees: workspaces, captured graphs, transposed trees.
// ---------------------------------------------------------------------------
template <typename T>
static void rebuild_trees(lb_ctx* ctx, Prec<T>& P, bool& adj_built, bool& z_built, int leaf_src) {
  HIPTRY(hipDeviceSynchronize());
  ctx->reset_graphs();
  // the old trees' workspaces go first (a deep candidate's are large)
  for (DBuf* b : {&P.str, &P.M, &P.Lc, &P.D, &P.fmm, &P.corr, &P.Y}) b->release();
  const bool fp32 = sizeof(T) == 4;
  build_prec<T>(ctx, P, P.p, std::vector<double>(), fp32 ? ctx->rm2f : std::vector<float>(), P.min_leaf_side,
                leaf_src, P.direct);
  P.ws_rhs = 0;
  adj_built = false;
  z_built = false;
  HIPTRY(hipDeviceSynchronize());
}

// new leaf-kernel work items (their count sizes the workspace; captured
// graphs hold the old buffers)
template <typename T>
static void set_leaf_shape(lb_ctx* ctx, Prec<T>& P, int fmax, int split) {
  HIPTRY(hipDeviceSynchronize());
  ctx->reset_graphs();
  make_leaf_work<T>(P, fmax, split);
  P.ws_rhs = 0;
  HIPTRY(hipDeviceSynchronize());
}

// overlapped-apply schedule (fork point, near-field grid); graphs captured
// with the old one are dropped
template <typename T>
static void set_schedule(lb_ctx* ctx, Prec<T>& P, int fork_late, int near_grid, int corr_early) {
  HIPTRY(hipDeviceSynchronize());
  ctx->reset_graphs();
  P.fork_late = fork_late;
  P.near_grid = near_grid;
  P.corr_early = corr_early;
  P.dt.fork_late = fork_late;
  P.dt.near_grid = near_grid;
  P.dt.corr_early = corr_early;
}

template <typename T>
static double time_apply(lb_ctx* ctx, Prec<T>& P, int nd, const DBuf& in, DBuf& out, int reps, hipStream_t st) {
  const int64_t N = ctx->N;
  const T* x = dptr<T>(in);
  T* o = dptr<T>(out);
  auto run = [&]() {
    apply_gradS_t<T>(ctx, P, nd, x, o, o + nd * N, o + 4 * nd * N, o + 5 * nd * N, st);
  };
  run();  // workspace allocation
  hipEvent_t e0, e1;
  HIPTRY(hipEventCreate(&e0));
  HIPTRY(hipEventCreate(&e1));
  HIPTRY(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) run();
  HIPTRY(hipEventRecord(e1, st));
  HIPTRY(hipEventSynchronize(e1));
  float ms = 0;
  HIPTRY(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return (double)ms / reps;
}

template <typename T>
static void autotune_t(lb_ctx* ctx, Prec<T>& P, bool& adj_built, bool& z_built, int nd, lb_tune_info& r,
                       hipStream_t st) {
  const int64_t N = ctx->N;
  DBuf in, out;
  in.alloc(sizeof(T) * (size_t)nd * N);
  out.alloc(sizeof(T) * (size_t)8 * nd * N);
  HIPTRY(hipMemsetAsync(in.p, 0, sizeof(T) * (size_t)nd * N, st));
  const int reps = 3;
  const int base_ls = P.build_leaf_src, base_fm = P.leaf_fmax, base_sp = P.leaf_split;
  std::vector<int> cand{base_ls};
  if (!P.direct)
    for (double f : {0.25, 0.5, 2.0, 4.0}) {
      const int v = std::max(16, (int)(base_ls * f));
      if (std::find(cand.begin(), cand.end(), v) == cand.end()) cand.push_back(v);
    }
  std::vector<std::vector<int>> seen;
  int best_ls = base_ls, best_fm = base_fm, best_sp = base_sp;
  double best = 1e300;
  r = lb_tune_info{};
  r.ms_default = -1.0;
  auto trial = [&](int ls, int fm, int sp, int depth) {
    set_leaf_shape<T>(ctx, P, fm, sp);
    const double ms = time_apply<T>(ctx, P, nd, in, out, reps, st);
    if (ls == base_ls && fm == base_fm && sp == base_sp && r.ms_default < 0) r.ms_default = ms;
    if (r.n_trials < LB_TUNE_MAX_TRIALS) {
      const int k = r.n_trials++;
      r.trial_leaf_src[k] = ls;
      r.trial_fmax[k] = fm;
      r.trial_split[k] = sp;
      r.trial_depth[k] = depth;
      r.trial_ms[k] = ms;
      r.trial_fork_late[k] = P.fork_late;
      r.trial_near_grid[k] = P.near_grid;
      r.trial_corr_early[k] = P.corr_early;
    }
    if (ms < best) { best = ms; best_ls = ls; best_fm = fm; best_sp = sp; }
  };
  // octree depth x lanes per target (one block per leaf), then the leaf
  // splitting of the best of those
  int best_depth = 0;
  for (size_t a = 0; a < cand.size(); ++a) {
    if (a > 0) rebuild_trees<T>(ctx, P, adj_built, z_built, cand[a]);
    std::vector<int> depths;
    for (const Octree& t : P.trees) depths.push_back(t.depth);
    if (std::find(seen.begin(), seen.end(), depths) != seen.end()) continue;
    seen.push_back(depths);
    const int dmax = *std::max_element(depths.begin(), depths.end());
    for (int fm : {64, 32, 16}) {
      const double b0 = best;
      trial(cand[a], fm, 0, dmax);
      if (best < b0) best_depth = dmax;
    }
  }
  if (P.build_leaf_src != best_ls) rebuild_trees<T>(ctx, P, adj_built, z_built, best_ls);
  const int fm0 = best_fm;
  for (int sp : {1, 2, 3}) trial(best_ls, fm0, sp, best_depth);
  set_leaf_shape<T>(ctx, P, best_fm, best_sp);
  // schedule of the overlapped apply at the best shape: the near-field
  // kernel forked after the strengths or after P2M, on every work item or
  // on 4 or 6 blocks per compute unit (leaving wave slots to the far field)
  int best_fl = P.fork_late, best_ng = P.near_grid, best_ce = P.corr_early;
  if (ctx->side_stream && !P.direct) {
    int dev = 0, ncu = 0;
    HIPTRY(hipGetDevice(&dev));
    HIPTRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    const int fl0 = P.fork_late, ng0 = P.near_grid, ce0 = P.corr_early;
    for (int ce : {0, 1})
      for (int fl : {0, 1})
        for (int ng : {0, 4 * ncu, 6 * ncu}) {
          if (fl == fl0 && ng == ng0 && ce == ce0) continue;  // timed above
          set_schedule<T>(ctx, P, fl, ng, ce);
          const double ms = time_apply<T>(ctx, P, nd, in, out, reps, st);
          if (r.n_trials < LB_TUNE_MAX_TRIALS) {
            const int k = r.n_trials++;
            r.trial_leaf_src[k] = best_ls;
            r.trial_fmax[k] = best_fm;
            r.trial_split[k] = best_sp;
            r.trial_depth[k] = best_depth;
            r.trial_ms[k] = ms;
            r.trial_fork_late[k] = fl;
            r.trial_near_grid[k] = ng;
            r.trial_corr_early[k] = ce;
          }
          if (ms < best) { best = ms; best_fl = fl; best_ng = ng; best_ce = ce; }
        }
    set_schedule<T>(ctx, P, best_fl, best_ng, best_ce);
  }
  r.leaf_src = best_ls;
  r.leaf_fmax = best_fm;
  r.leaf_split = best_sp;
  r.fork_late = best_fl;
  r.near_grid = best_ng;
  r.corr_early = best_ce;
  r.ms_best = best;
  r.depth = 0;
  for (const Octree& t : P.trees) r.depth = std::max(r.depth, t.depth);
  HIPTRY(hipStreamSynchronize(st));
}

template <typename T>
static void set_tuning_t(lb_ctx* ctx, Prec<T>& P, bool& adj_built, bool& z_built, const lb_tune_info& c) {
  if (P.direct && c.leaf_src != P.build_leaf_src) fail(LB_EINVAL, "a direct context keeps its one-leaf tree");
  if (c.leaf_src != P.build_leaf_src) rebuild_trees<T>(ctx, P, adj_built, z_built, c.leaf_src);
  set_leaf_shape<T>(ctx, P, c.leaf_fmax, c.leaf_split);
  set_schedule<T>(ctx, P, c.fork_late, c.near_grid, c.corr_early);
}

// ---------------------------------------------------------------------------
// Transposed A3 (adjoint of apply_A3_t, the same discrete operator):
//   A3^T v = -v/4 + S'^T S'^T v - S^T (S''+D')^T v - S^T S'^T (2 H v)
//            + (sum_i v_i / area) S^T S^T w
// in two transposed FMMs: step 1 (FMM_ADJ3) a = S'^T v and
// b = (S''+D')^T v + S'^T (2 H v); step 2 (FMM_ADJ) S'^T a - S^T b.
// ---------------------------------------------------------------------------

template <typename T>
static void apply_A3T_t(lb_ctx* ctx, Prec<T>& F, Prec<T>& A, bool& built, DBuf& zb, bool& zbuilt, int nd,
                        const T* v, T* out, hipStream_t st) {
  ensure_ws(ctx, F, CHUNK_GRAD);  // allocates ctx->partial (column sums below)
  ensure_adjoint<T>(ctx, F, A, built);
  const int64_t N = ctx->N, No = F.No;
  if (!zbuilt) {
    DBuf wt, z1;
    wt.alloc(sizeof(T) * N);
    z1.alloc(sizeof(T) * N);
    zb.alloc(sizeof(T) * N);
    std::vector<T> wh(ctx->S.w.begin(), ctx->S.w.end());
    HIPTRY(hipMemcpy(wt.p, wh.data(), sizeof(T) * N, hipMemcpyHostToDevice));
    apply_adj_t<T>(ctx, F, A, built, 1, dptr<T>(wt), nullptr, nullptr, nullptr, dptr<T>(z1), st);
    apply_adj_t<T>(ctx, F, A, built, 1, dptr<T>(z1), nullptr, nullptr, nullptr, dptr<T>(zb), st);
    HIPTRY(hipStreamSynchronize(st));
    zbuilt = true;
  }
  ctx->a3t_a.alloc(sizeof(double) * (size_t)N * CHUNK_A3T);
  ctx->a3t_b.alloc(sizeof(double) * (size_t)N * CHUNK_A3T);
  ctx->a3t_scal.alloc(sizeof(double) * CHUNK_A3T * ctx->n_surf);
  ctx->g4.alloc(sizeof(T) * (size_t)N * 4 * CHUNK_GRAD);
  T* a = dptr<T>(ctx->a3t_a);
  T* b = dptr<T>(ctx->a3t_b);
  T* g2 = dptr<T>(ctx->g4);
  for (int d0 = 0; d0 < nd; d0 += CHUNK_A3T) {
    const int c = std::min(CHUNK_A3T, nd - d0);
    const T* vd = v + (int64_t)d0 * N;
    launch_adj3_str1<T>(c, N, vd, dptr<T>(F.H), dptr<int>(A.src_pos), dptr<T>(A.str), g2, st);
    launch_fmm<T>(A.dt, FMM_ADJ3, c, dptr<T>(A.str), dptr<T>(A.M), dptr<T>(A.Lc), dptr<T>(A.D), dptr<T>(A.fmm), No,
                  N, st);
    launch_adj3_comb1<T>(c, ctx->NP, ctx->n_p, F.n_o, N, No, dptr<T>(F.P), dptr<T>(F.wo), dptr<T>(A.fmm),
                         dptr<int>(A.tgt_pos), dptr<int64_t>(ctx->cptr), dptr<int>(ctx->crow),
                         dptr<int64_t>(ctx->cblk), dptr<T>(F.vals3), g2, a, b, st);
    launch_seg_dot<T>(c, ctx->n_surf, N, dptr<int64_t>(ctx->node_off), vd, nullptr, dptr<double>(ctx->inv_area),
                      dptr<double>(ctx->a3t_scal), st);
    launch_adj3_str2<T>(c, N, a, b, dptr<T>(F.nrm), dptr<int>(A.src_pos), dptr<T>(A.str), g2, st);
    launch_fmm<T>(A.dt, FMM_ADJ, c, dptr<T>(A.str), dptr<T>(A.M), dptr<T>(A.Lc), dptr<T>(A.D), dptr<T>(A.fmm), No,
                  N, st);
    launch_adj3_comb2<T>(c, ctx->NP, ctx->n_p, F.n_o, N, No, dptr<T>(F.P), dptr<T>(F.wo), dptr<T>(A.fmm),
                         dptr<int>(A.tgt_pos), dptr<int64_t>(ctx->cptr), dptr<int>(ctx->crow),
                         dptr<int64_t>(ctx->cblk), dptr<T>(F.vals3), g2, vd, dptr<T>(zb),
                         dptr<double>(ctx->a3t_scal), ctx->n_surf, dptr<int>(ctx->node_surf), out + (int64_t)d0 * N,
                         st);
  }
}

// ---------------------------------------------------------------------------
// Apply `body` (kernel launches only, on the stream it is given) to in -> out
// through a captured HIP graph.  A call with new buffers or a new density
// count runs the body eagerly on `st` (which also makes every allocation
// the body needs), then captures it on the library's stream for the
// following calls; LB_NO_GRAPH runs it eagerly always.
// ---------------------------------------------------------------------------
// capture `body` (kernel launches only) on the library's capture stream
// into G and instantiate it
template <typename Body>
static void capture(lb_ctx* ctx, OpGraph& G, Body&& body) {
  if (!ctx->cap_stream) HIPTRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  HIPTRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
  try {
    body(ctx->cap_stream);
  } catch (...) {
    // close the capture so the stream stays usable, then report the failure
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(ctx->cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  HIPTRY(hipStreamEndCapture(ctx->cap_stream, &G.graph));
  HIPTRY(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
}

template <typename Body>
static void graphed(lb_ctx* ctx, OpGraph& G, Body&& body, const void* in, const void* out, int n, hipStream_t st) {
  if (ctx->opts.flags & LB_NO_GRAPH) {
    body(st);
    return;
  }
  if (G.exec && G.in == in && G.out == out && G.n == n) {
    HIPTRY(hipGraphLaunch(G.exec, st));
    return;
  }
  G.reset();
  body(st);
  capture(ctx, G, body);
  G.in = in;
  G.out = out;
  G.n = n;
}

// ---------------------------------------------------------------------------
// GMRES (Section 6) for several independent systems at once: x0 = 0, no
// restart; system a is the segment [xoff[a], xoff[a] + len[a]) of the
// operator's vectors [nrhs][N] (one (right-hand side, surface) pair), with
// its own Arnoldi basis (CGS2) and Givens rotations, all FP64 on the device
// (launch_gm_*).  One iteration (gather of the current basis vectors, the
// operator on all systems at once (zero segments for the stopped ones),
// CGS2, the Givens step, the next basis vector) is captured once as a HIP
// graph and replayed; the host reads one integer per iteration, the number
// of systems still iterating.
// A(in [nrhs][N], out [nrhs][N], nrhs, stream): kernel launches only.
// ---------------------------------------------------------------------------
struct Systems {
  std::vector<int64_t> xoff, len;
};

// Euclidean norms of every system's segment of v [nrhs][N]
static std::vector<double> system_norms(lb_ctx* ctx, const Systems& sy, const double* v, hipStream_t st) {
  const int ns = (int)sy.xoff.size();
  ctx->msys2.alloc(sizeof(int64_t) * 2 * ns + sizeof(double) * (ns * 33 + 8));
  int64_t* d = dptr<int64_t>(ctx->msys2);
  double* part = reinterpret_cast<double*>(d + 2 * ns);
  double* out = part + (size_t)ns * 32;
  std::vector<int64_t> t(2 * ns);
  for (int a = 0; a < ns; ++a) { t[a] = sy.xoff[a]; t[ns + a] = sy.len[a]; }
  HIPTRY(hipMemcpyAsync(d, t.data(), sizeof(int64_t) * 2 * ns, hipMemcpyHostToDevice, st));
  launch_msys_dots(ns, 1, d, d + ns, nullptr, nullptr, v, part, out, st);
  std::vector<double> h(ns);
  HIPTRY(hipMemcpyAsync(h.data(), out, sizeof(double) * ns, hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  for (double& x : h) x = std::sqrt(x);
  return h;
}

// the (right-hand side, surface) systems of nrhs densities
static Systems make_systems(const lb_ctx* ctx, int nrhs) {
  Systems sy;
  for (int q = 0; q < nrhs; ++q)
    for (int s = 0; s < ctx->n_surf; ++s) {
      sy.xoff.push_back((int64_t)q * ctx->N + ctx->node_off_h[s]);
      sy.len.push_back(ctx->node_off_h[s + 1] - ctx->node_off_h[s]);
    }
  return sy;
}

// device state of gmres_sys for ns systems and maxit iterations (one
// allocation, carved in 256-byte aligned pieces)
static GmresDev gmres_state(lb_ctx* ctx, const Systems& sy, int maxit, int64_t& vtot) {
  const int ns = (int)sy.xoff.size();
  const int km = maxit + 1;
  const size_t sz[] = {sizeof(int64_t) * ns * 3, sizeof(int) * ((size_t)ns * 2 + 2),
                       sizeof(double) * (size_t)ns * maxit * maxit, sizeof(double) * (size_t)ns * maxit * 2,
                       sizeof(double) * (size_t)ns * km * 3, sizeof(double) * (size_t)ns * 5,
                       sizeof(double) * (size_t)ns * km * 32, sizeof(double)};
  size_t off[9] = {0};
  for (int q = 0; q < 8; ++q) off[q + 1] = off[q] + (sz[q] + 255) / 256 * 256;
  ctx->gm_state.alloc(off[8]);
  ctx->gm_skip.alloc(sizeof(int) * (size_t)ns);
  if (!ctx->gm_host) HIPTRY(hipHostMalloc((void**)&ctx->gm_host, sizeof(int) * 4, hipHostMallocDefault));
  char* b = static_cast<char*>(ctx->gm_state.p);
  GmresDev gm;
  int64_t* i64 = reinterpret_cast<int64_t*>(b + off[0]);
  gm.xoff = i64; gm.len = i64 + ns; gm.vbase = i64 + 2 * ns;
  int* i32 = reinterpret_cast<int*>(b + off[1]);
  gm.active = i32; gm.kdone = i32 + ns; gm.iter = i32 + 2 * ns; gm.nactive = i32 + 2 * ns + 1;
  gm.R = reinterpret_cast<double*>(b + off[2]);
  gm.cs = reinterpret_cast<double*>(b + off[3]); gm.sn = gm.cs + (size_t)ns * maxit;
  gm.g = reinterpret_cast<double*>(b + off[4]); gm.h1 = gm.g + (size_t)ns * km; gm.h2 = gm.h1 + (size_t)ns * km;
  double* s5 = reinterpret_cast<double*>(b + off[5]);
  gm.beta = s5; gm.relres = s5 + ns; gm.sc = s5 + 2 * ns; gm.nr = s5 + 3 * ns;
  gm.part = reinterpret_cast<double*>(b + off[6]);
  gm.tol = reinterpret_cast<double*>(b + off[7]);
  gm.ns = ns; gm.maxit = maxit; gm.km = km;
  std::vector<int64_t> t(3 * (size_t)ns);
  vtot = 0;
  gm.maxlen = 1;
  for (int a = 0; a < ns; ++a) {
    t[a] = sy.xoff[a];
    t[ns + a] = sy.len[a];
    t[2 * ns + a] = vtot;
    vtot += (int64_t)km * sy.len[a];
    gm.maxlen = std::max(gm.maxlen, sy.len[a]);
  }
  HIPTRY(hipMemcpy(const_cast<int64_t*>(gm.xoff), t.data(), sizeof(int64_t) * t.size(), hipMemcpyHostToDevice));
  return gm;
}

template <typename ApplyFn>
static void gmres_sys(lb_ctx* ctx, ApplyFn A, OpGraph& G, int nrhs, const Systems& sy, const double* B, double* X,
                      double tol, int maxit, const std::vector<char>& skip, std::vector<double>& relres,
                      std::vector<int>& iters, hipStream_t st) {
  const int64_t N = ctx->N;
  const int ns = (int)sy.xoff.size();
  int64_t vtot = 0;
  const GmresDev gm = gmres_state(ctx, sy, maxit, vtot);
  ctx->V.alloc(sizeof(double) * (size_t)std::max<int64_t>(vtot, 1));
  ctx->wv.alloc(sizeof(double) * (size_t)N * nrhs * 2);
  double* Vall = dptr<double>(ctx->V);
  double* win = dptr<double>(ctx->wv);
  double* wout = win + (size_t)N * nrhs;
  {
    std::vector<int> sk(ns);
    for (int a = 0; a < ns; ++a) sk[a] = skip[a] ? 1 : 0;
    HIPTRY(hipMemcpyAsync(dptr<int>(ctx->gm_skip), sk.data(), sizeof(int) * ns, hipMemcpyHostToDevice, st));
    HIPTRY(hipMemcpyAsync(const_cast<double*>(gm.tol), &tol, sizeof(double), hipMemcpyHostToDevice, st));
    launch_gm_start(gm, B, dptr<int>(ctx->gm_skip), Vall, st);
    HIPTRY(hipMemcpyAsync(ctx->gm_host, gm.nactive, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));  // sk and tol are host locals; nactive read
  }
  auto body = [&](hipStream_t s) {
    launch_gm_gather(gm, Vall, win, s);
    A(win, wout, nrhs, s);
    launch_gm_arnoldi(gm, Vall, wout, s);
  };
  const bool use_graph = !(ctx->opts.flags & LB_NO_GRAPH);
  bool have = G.exec && G.in == win && G.out == wout && G.n == nrhs && G.aux0 == Vall && G.aux1 == ctx->gm_state.p &&
              G.aux2 == ((int64_t)ns << 32 | maxit);
  for (int j = 0; j < maxit && *ctx->gm_host > 0; ++j) {
    if (!use_graph) {
      body(st);
    } else if (have) {
      HIPTRY(hipGraphLaunch(G.exec, st));
    } else {
      // the first iteration runs eagerly (it makes the allocations the
      // operator needs); the following ones replay its graph
      G.reset();
      body(st);
      capture(ctx, G, body);
      G.in = win; G.out = wout; G.n = nrhs;
      G.aux0 = Vall; G.aux1 = ctx->gm_state.p; G.aux2 = (int64_t)ns << 32 | maxit;
      have = true;
    }
    HIPTRY(hipMemcpyAsync(ctx->gm_host, gm.nactive, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
  }
  launch_gm_finish(gm, Vall, X, st);
  std::vector<int> kd(ns);
  relres.assign(ns, 0.0);
  HIPTRY(hipMemcpyAsync(kd.data(), gm.kdone, sizeof(int) * ns, hipMemcpyDeviceToHost, st));
  HIPTRY(hipMemcpyAsync(relres.data(), gm.relres, sizeof(double) * ns, hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  iters.assign(kd.begin(), kd.end());
}

// ---------------------------------------------------------------------------
// Solve A sig = b for every system (b, sig [nrhs][N]; bnorm per system):
// LB_SOLVE_FP64: GMRES with the FP64 operator A64; LB_SOLVE_FP32_REFINE:
// iterative refinement, each correction from GMRES with the FP32 operator
// A32 on the FP64 residual.  A refinement step that leaves a system's FP64
// residual larger than before is taken back for that system; a system whose
// refinement stops contracting (residual above half the previous one) before
// reaching tol gets a last correction from GMRES with the FP64 operator.
// rel = final FP64 relative residuals per system.  A64 / A32: kernel
// launches only (in, out, nrhs, stream); G64 / G32 hold their GMRES
// iteration graphs, GR the residual apply's graph.  r, ut, dcorr: [nrhs][N]
// workspace.
// ---------------------------------------------------------------------------
template <typename Op64, typename Op32>
static void solve_system(lb_ctx* ctx, int nrhs, const Systems& sy, Op64& A64, Op32& A32, OpGraph& G64,
                         OpGraph& G32, OpGraph& GR, const double* b, const std::vector<double>& bnorm, double* sig,
                         double* r, double* ut, double* dcorr, double tol, int mode, std::vector<double>& rel,
                         std::vector<int>& iters, std::vector<int>& outer, hipStream_t st) {
  const int64_t N = ctx->N;
  const size_t nN = (size_t)nrhs * N;
  const int maxit = ctx->opts.max_iter;
  const int ns = (int)sy.xoff.size();
  rel.assign(ns, 0.0);
  iters.assign(ns, 0);
  outer.assign(ns, 0);
  std::vector<double> inner;
  std::vector<int> it;
  std::vector<char> skip(ns, 0);
  auto residual = [&]() {  // r = b - A sig (FP64), rel = |r| / |b| per system
    graphed(ctx, GR, [&](hipStream_t s2) { A64(sig, ut, nrhs, s2); }, sig, ut, nrhs, st);
    launch_axpby(1.0, b, -1.0, ut, r, (int64_t)nN, st);
    std::vector<double> rn = system_norms(ctx, sy, r, st);
    for (int a = 0; a < ns; ++a) rel[a] = bnorm[a] > 0 ? rn[a] / bnorm[a] : 0.0;
  };
  if (mode == LB_SOLVE_FP64) {
    gmres_sys(ctx, A64, G64, nrhs, sy, b, sig, tol, maxit, skip, inner, it, st);
    for (int a = 0; a < ns; ++a) iters[a] = it[a];
    residual();
    return;
  }
  HIPTRY(hipMemsetAsync(sig, 0, sizeof(double) * nN, st));
  HIPTRY(hipMemcpyAsync(r, b, sizeof(double) * nN, hipMemcpyDeviceToDevice, st));
  for (int a = 0; a < ns; ++a) rel[a] = bnorm[a] > 0 ? 1.0 : 0.0;
  std::vector<double> prev(ns, 1e300);
  std::vector<char> stalled(ns, 0);
  const int max_outer = 12;
  for (int step = 0; step < max_outer; ++step) {
    bool any = false;
    for (int a = 0; a < ns; ++a) {
      if (rel[a] >= tol && rel[a] > 0.5 * prev[a]) stalled[a] = 1;  // refinement stopped contracting
      skip[a] = !(rel[a] >= tol) || stalled[a];
      any |= !skip[a];
    }
    if (!any) break;
    // inner FP32 solves: the FP32 operator is accurate to ~1e-6, so each
    // refinement step asks for no more than that
    double worst = 0;
    for (int a = 0; a < ns; ++a)
      if (!skip[a]) worst = std::max(worst, rel[a]);
    const double inner_tol = std::max(1e-6, 0.5 * tol / std::max(worst, 1e-300));
    gmres_sys(ctx, A32, G32, nrhs, sy, r, dcorr, inner_tol, maxit, skip, inner, it, st);
    for (int a = 0; a < ns; ++a) {
      if (skip[a]) continue;
      iters[a] += it[a];
      outer[a] += 1;
    }
    // skipped systems have a zero correction (gmres_sys writes zeros there)
    launch_axpby(1.0, sig, 1.0, dcorr, sig, (int64_t)nN, st);
    prev = rel;
    residual();
    bool undo = false;
    for (int a = 0; a < ns; ++a)
      if (!skip[a] && rel[a] > prev[a]) {  // the step made this system worse: take it back
        launch_axpby(1.0, sig + sy.xoff[a], -1.0, dcorr + sy.xoff[a], sig + sy.xoff[a], sy.len[a], st);
        stalled[a] = 1;
        undo = true;
      }
    if (undo) residual();
  }
  // FP64 correction for the systems whose refinement stalled above tol
  bool any = false;
  double worst = 0;
  for (int a = 0; a < ns; ++a) {
    skip[a] = !(stalled[a] && rel[a] >= tol);
    if (!skip[a]) {
      any = true;
      worst = std::max(worst, rel[a]);
    }
  }
  if (any) {
    gmres_sys(ctx, A64, G64, nrhs, sy, r, dcorr, std::min(0.5, 0.5 * tol / std::max(worst, 1e-300)), maxit, skip,
              inner, it, st);
    for (int a = 0; a < ns; ++a)
      if (!skip[a]) {
        iters[a] += it[a];
        outer[a] += 1;
      }
    launch_axpby(1.0, sig, 1.0, dcorr, sig, (int64_t)nN, st);
    residual();
  }
}

}  // namespace lb

namespace lb {
// Carve the gradient apply's workspace out of the static scratch (256-byte
// aligned pieces); throws LB_ENOMEM when it does not fit.
template <typename T>
static ApplyWs<T> scratch_ws(lb_ctx* ctx, Prec<T>& P, int nd) {
  size_t cnt[6];
  ws_counts<T>(ctx, P, std::min(nd, chunk_fwd<T>()), cnt);
  size_t off[7] = {0};
  for (int i = 0; i < 6; ++i) off[i + 1] = off[i] + (sizeof(T) * cnt[i] + 255) / 256 * 256;
  if (off[6] > NOALLOC_SCRATCH_BYTES)
    fail(LB_ENOMEM, "lb_apply_gradS_noalloc needs %zu bytes of scratch for %d densities, the static scratch holds %zu",
         off[6], nd, NOALLOC_SCRATCH_BYTES);
  unsigned char* base = static_cast<unsigned char*>(noalloc_scratch(ctx->device));
  ApplyWs<T> w;
  w.str = reinterpret_cast<T*>(base + off[0]);
  w.M = reinterpret_cast<T*>(base + off[1]);
  w.Lc = reinterpret_cast<T*>(base + off[2]);
  w.D = reinterpret_cast<T*>(base + off[3]);
  w.fmm = reinterpret_cast<T*>(base + off[4]);
  w.corr = reinterpret_cast<T*>(base + off[5]);
  return w;
}
}  // namespace lb


// ===========================================================================
// C ABI
// ===========================================================================
#define API_BEGIN try {
#define API_END                                  \
  }                                              \
  catch (const lb::Error& e) {                   \
    lb::set_last_error(e.what());                \
    return e.code;                               \
  }                                              \
  catch (const std::bad_alloc&) {                \
    lb::set_last_error("host allocation failed"); \
    return LB_ENOMEM;                            \
  }                                              \
  catch (const std::exception& e) {              \
    lb::set_last_error(e.what());                \
    return LB_EINVAL;                            \
  }                                              \
  return LB_OK;

extern "C" {

const char* lb_last_error(void) { return lb::g_last_error.c_str(); }

lb_status lb_default_opts(lb_opts* o) {
  API_BEGIN
  if (!o) fail(LB_EINVAL, "null opts");
  default_opts(o);
  API_END
}

lb_status lb_ref_nodes(int order, double* uv, double* w_ref) {
  API_BEGIN
  if (!uv) fail(LB_EINVAL, "null uv");
  std::vector<double> nodes = ref_nodes(order);
  std::memcpy(uv, nodes.data(), sizeof(double) * nodes.size());
  if (w_ref) {
    RefElem re(order, order + 2);
    std::memcpy(w_ref, re.w_ref.data(), sizeof(double) * re.n_p);
  }
  API_END
}

namespace lb {
// Corrections C = A - B of every (target, near patch) block on the device
// (self rule, adaptive near rule, far rule with and without the FP32 mask),
// left in the packed layouts of the combine kernels: v4 (S, Gx, Gy, Gz), v3
// (S, S', S''+D') and vD (D) per (block, node), FP64 and FP32.
struct DevCorrections {
  DBuf v4_64, v3_64, vD_64, v4_32, v3_32, vD_32;
};

static void corrections_device(const Surface& S, const RefElem& re, const QuadOpts& qo, const std::vector<float>& rm2,
                               DevCorrections& out) {
  const int n_p = S.n_p;
  const int64_t nb = S.near_ptr[S.N];
  std::vector<int64_t> row, blk, brow(nb), sblk(S.N, -1);
  std::vector<int32_t> pat;
  for (int64_t i = 0; i < S.N; ++i)
    for (int64_t b = S.near_ptr[i]; b < S.near_ptr[i + 1]; ++b) {
      brow[b] = i;
      if (S.near_patch[b] == (int32_t)(i / n_p)) {
        sblk[i] = b;
      } else {
        row.push_back(i);
        blk.push_back(b);
        pat.push_back(S.near_patch[b]);
      }
    }
  std::vector<double> ru, rw, g, gw, tg, tw, mg, mw;
  near_leaf_rule(qo.near_q, ru, rw);
  gauss_legendre01(qo.self_n, g, gw);
  gauss_legendre01(qo.self_nt, tg, tw);
  gauss_legendre01((re.k + 1) / 2, mg, mw);
  DBuf dX, dn, ddXu, ddXv, dJ, dcX, dcXu, dcXv, dja, djb, djc, dVinv, duv, dg, dgw, dtg, dtw, dru, drw;
  DBuf dcDu, dcDv, dmg, dmw;
  upload(dcDu, S.cDu); upload(dcDv, S.cDv); upload(dmg, mg); upload(dmw, mw);
  DBuf drow, dblk, dpat, dsblk, dbrow, dnp, ds, dnu, dwo, drm2, dP, dA;
  upload(dX, S.X); upload(dn, S.nrm); upload(ddXu, S.dXu); upload(ddXv, S.dXv); upload(dJ, S.J);
  upload(dcX, S.cX); upload(dcXu, S.cXu); upload(dcXv, S.cXv);
  upload(dja, re.ja); upload(djb, re.jb); upload(djc, re.jc); upload(dVinv, re.Vinv); upload(duv, re.uv);
  upload(dg, g); upload(dgw, gw); upload(dtg, tg); upload(dtw, tw); upload(dru, ru); upload(drw, rw);
  upload(drow, row); upload(dblk, blk); upload(dpat, pat); upload(dsblk, sblk); upload(dbrow, brow);
  upload(dnp, S.near_patch);
  upload(ds, S.s); upload(dnu, S.nu); upload(dwo, S.wo); upload(drm2, rm2); upload(dP, re.P);
  dA.alloc(sizeof(double) * (size_t)nb * n_p * NKER);
  SelfQuadArgs sq;
  sq.X = dptr<double>(dX); sq.nrm = dptr<double>(dn); sq.dXu = dptr<double>(ddXu); sq.dXv = dptr<double>(ddXv);
  sq.J = dptr<double>(dJ);
  sq.cX = dptr<double>(dcX); sq.cXu = dptr<double>(dcXu); sq.cXv = dptr<double>(dcXv);
  sq.ja = dptr<double>(dja); sq.jb = dptr<double>(djb); sq.jc = dptr<double>(djc);
  sq.Vinv = dptr<double>(dVinv); sq.uv = dptr<double>(duv);
  sq.g = dptr<double>(dg); sq.gw = dptr<double>(dgw); sq.tg = dptr<double>(dtg); sq.tw = dptr<double>(dtw);
  sq.sblk = dptr<int64_t>(dsblk); sq.A = dptr<double>(dA);
  sq.cDu = dptr<double>(dcDu); sq.cDv = dptr<double>(dcDv);
  sq.mg = dptr<double>(dmg); sq.mw = dptr<double>(dmw); sq.nm = (int)mg.size();
  sq.N = S.N; sq.k = re.k; sq.ns = qo.self_n; sq.nt = qo.self_nt; sq.panel = qo.self_panel;
  HIPTRY(launch_self_quad(sq, nullptr));
  NearQuadArgs nq;
  nq.X = sq.X; nq.nrm = sq.nrm; nq.cX = sq.cX; nq.cXu = sq.cXu; nq.cXv = sq.cXv;
  nq.ja = sq.ja; nq.jb = sq.jb; nq.jc = sq.jc; nq.Vinv = sq.Vinv;
  nq.ru = dptr<double>(dru); nq.rw = dptr<double>(drw);
  nq.row = dptr<int64_t>(drow); nq.blk = dptr<int64_t>(dblk); nq.patch = dptr<int32_t>(dpat);
  nq.A = sq.A; nq.nwork = (int64_t)row.size(); nq.k = re.k; nq.nq = qo.near_q * qo.near_q;
  nq.max_depth = qo.max_depth; nq.adm = qo.near_adm;
  HIPTRY(launch_near_quad(nq, nullptr));
  const size_t ne = (size_t)nb * n_p;
  out.v4_64.alloc(sizeof(double) * ne * 4);
  out.v3_64.alloc(sizeof(double) * ne * 3);
  out.vD_64.alloc(sizeof(double) * ne);
  out.v4_32.alloc(sizeof(float) * ne * 4);
  out.v3_32.alloc(sizeof(float) * ne * 3);
  out.vD_32.alloc(sizeof(float) * ne);
  // FP64 values from the primary far rule
  FarRuleArgs fr;
  fr.X = sq.X; fr.nrm = sq.nrm; fr.s = dptr<double>(ds); fr.nu = dptr<double>(dnu); fr.wo = dptr<double>(dwo);
  fr.rm2 = nullptr; fr.P = dptr<double>(dP);
  fr.brow = dptr<int64_t>(dbrow); fr.patch = dptr<int32_t>(dnp); fr.A = sq.A;
  fr.v4_64 = dptr<double>(out.v4_64); fr.v3_64 = dptr<double>(out.v3_64); fr.vD_64 = dptr<double>(out.vD_64);
  fr.v4_32 = nullptr; fr.v3_32 = nullptr; fr.vD_32 = nullptr;
  fr.nb = nb; fr.n_p = n_p; fr.n_o = S.n_o;
  HIPTRY(launch_far_rule(fr, nullptr));
  // FP32 values from the FP32 far rule, without the points its near-field
  // kernel skips
  DBuf ds32, dnu32, dwo32, dP32;
  upload(ds32, S.o32.s); upload(dnu32, S.o32.nu); upload(dwo32, S.o32.wo); upload(dP32, S.o32.re->P);
  fr.s = dptr<double>(ds32); fr.nu = dptr<double>(dnu32); fr.wo = dptr<double>(dwo32); fr.P = dptr<double>(dP32);
  fr.rm2 = dptr<float>(drm2);
  fr.v4_64 = nullptr; fr.v3_64 = nullptr; fr.vD_64 = nullptr;
  fr.v4_32 = dptr<float>(out.v4_32); fr.v3_32 = dptr<float>(out.v3_32); fr.vD_32 = dptr<float>(out.vD_32);
  fr.n_o = S.o32.n_o;
  HIPTRY(launch_far_rule(fr, nullptr));
  HIPTRY(hipDeviceSynchronize());
}

// Setup of n_surf surfaces (surface q: pps[q] patches, in order).
// given (nullable): corrections taken over instead of generated (an
// imported setup), already on the device in the packed layouts.
static void setup_impl(lb_ctx* ctx, int n_surf, const int32_t* pps, int order, const double* X, const double* Xu,
                       const double* Xv, const lb_opts* opts, DevCorrections* given = nullptr) {
  if (!X || !Xu || !Xv || !pps) fail(LB_EINVAL, "null argument");
  if (n_surf < 1) fail(LB_EINVAL, "n_surf must be >= 1");
  ctx->surf_patch.assign(n_surf + 1, 0);
  for (int q = 0; q < n_surf; ++q) {
    if (pps[q] < 1) fail(LB_EINVAL, "surface %d has %d patches", q, pps[q]);
    ctx->surf_patch[q + 1] = ctx->surf_patch[q] + pps[q];
  }
  const int n_patches = ctx->surf_patch[n_surf];
  if (order < 1 || order > 7) fail(LB_EINVAL, "order %d out of range 1..7", order);
  if (opts) ctx->opts = *opts; else default_opts(&ctx->opts);
  lb_opts& o = ctx->opts;
  if (o.over_q <= 0) o.over_q = order + 6;
  if (o.over_q32 <= 0) o.over_q32 = std::max(order + 2, 6);
  if (o.over_q > 40 || o.over_q32 > 40) fail(LB_EINVAL, "over_q / over_q32 must be <= 40");
  if (o.eta_near <= 1.0) fail(LB_EINVAL, "eta_near must be > 1");
  if (o.p_f32 < 2 || o.p_f32 > 31 || o.p_f64 < 2 || o.p_f64 > 31) fail(LB_EINVAL, "expansion order out of range 2..31");
  if (o.max_iter < 1) fail(LB_EINVAL, "max_iter must be >= 1");
  if (o.self_n < 4 || o.near_q < 2 || o.near_adm <= 0) fail(LB_EINVAL, "bad quadrature options");
  if (!(o.m2l_trunc32 >= 0 && o.m2l_trunc32 < 1e6) || !(o.m2l_trunc64 >= 0 && o.m2l_trunc64 < 1e6))
    fail(LB_EINVAL, "m2l_trunc32 / m2l_trunc64 must be finite and >= 0");
  ctx->host_only = (o.flags & LB_HOST_ONLY) != 0;
  ctx->k = order;
  ctx->n_surf = n_surf;
  ctx->re.reset(new RefElem(order, o.over_q));
  ctx->re32.reset(new RefElem(order, o.over_q32));
  Surface& S = ctx->S;
  S.build(*ctx->re, n_patches, X, Xu, Xv, o.eta_near);
  S.build_over(*ctx->re32, S.o32);
  S.surf_of_patch.resize(n_patches);
  for (int q = 0; q < n_surf; ++q)
    for (int pt = ctx->surf_patch[q]; pt < ctx->surf_patch[q + 1]; ++pt) S.surf_of_patch[pt] = q;
  S.build_near_lists();
  ctx->NP = n_patches;
  ctx->n_p = S.n_p;
  ctx->n_o = S.n_o;
  ctx->N = S.N;
  ctx->No = S.No;
  ctx->node_off_h.assign(n_surf + 1, 0);
  ctx->surf_area.assign(n_surf, 0.0);
  std::vector<int> nsurf_of(S.N);
  std::vector<double> inv(n_surf);
  for (int q = 0; q < n_surf; ++q) {
    ctx->node_off_h[q + 1] = (int64_t)ctx->surf_patch[q + 1] * S.n_p;
    for (int64_t i = ctx->node_off_h[q]; i < ctx->node_off_h[q + 1]; ++i) {
      ctx->surf_area[q] += S.w[i];
      nsurf_of[i] = q;
    }
    inv[q] = 1.0 / ctx->surf_area[q];
  }
  QuadOpts qo;
  qo.self_n = o.self_n;
  qo.near_q = o.near_q;
  qo.near_adm = o.near_adm;
  // the device rules: at most 3 max_depth + 1 triangles on the near rule's
  // stack, at most 256 (node, kernel) outputs per block
  const bool dev_quad = given || (!ctx->host_only && !(o.flags & LB_HOST_QUAD) && 3 * qo.max_depth + 1 <= 72 &&
                                  NKER * S.n_p <= 256);
  std::vector<double> A, B;
  if (!dev_quad) {
    near_integrals(S, qo, A);
    std::vector<float> none;
    far_rule_blocks(S, none, none, none, false, B);
    ctx->C64.resize(A.size());
    for (size_t i = 0; i < A.size(); ++i) ctx->C64[i] = A[i] - B[i];
  }
  if (!ctx->host_only) {
    HIPTRY(hipGetDevice(&ctx->device));
    // device address of the static scratch of lb_apply_gradS_noalloc on
    // this device (looked up once per device, with the device current)
    (void)noalloc_scratch(ctx->device);
    // FP32 near-field mask: sources of patch l within kMaskFrac (eta-1) R_l
    // of a target are left to the corrections (such a patch is always in
    // Near(target), since |x - c_l| < (1 + (eta-1)) R_l)
    const double kMaskFrac = 0.5;
    std::vector<float> rm2(S.o32.No);
    double rmax = 0;
    for (int64_t m = 0; m < S.o32.No; ++m) {
      double rm = kMaskFrac * (o.eta_near - 1.0) * S.R[m / S.o32.n_o];
      rm2[m] = (float)(rm * rm);
      rmax = std::max(rmax, rm);
    }
    std::vector<double> C32;
    DevCorrections dc;
    if (given) {
      std::swap(dc.v4_64.p, given->v4_64.p); std::swap(dc.v4_64.bytes, given->v4_64.bytes);
      std::swap(dc.v3_64.p, given->v3_64.p); std::swap(dc.v3_64.bytes, given->v3_64.bytes);
      std::swap(dc.v4_32.p, given->v4_32.p); std::swap(dc.v4_32.bytes, given->v4_32.bytes);
      std::swap(dc.v3_32.p, given->v3_32.p); std::swap(dc.v3_32.bytes, given->v3_32.bytes);
      std::swap(dc.vD_64.p, given->vD_64.p); std::swap(dc.vD_64.bytes, given->vD_64.bytes);
      std::swap(dc.vD_32.p, given->vD_32.p); std::swap(dc.vD_32.bytes, given->vD_32.bytes);
    } else if (dev_quad) {
      corrections_device(S, *ctx->re, qo, rm2, dc);
    } else {
      std::vector<float> tx32(3 * S.N), sx32(3 * S.o32.No);
      for (int64_t i = 0; i < 3 * S.N; ++i) tx32[i] = (float)S.X[i];
      for (int64_t i = 0; i < 3 * S.o32.No; ++i) sx32[i] = (float)S.o32.s[i];
      std::vector<double> B32;
      far_rule_blocks(S, rm2, tx32, sx32, true, B32, &S.o32);
      C32.resize(A.size());
      for (size_t i = 0; i < A.size(); ++i) C32[i] = A[i] - B32[i];
    }
    A.clear(); A.shrink_to_fit();
    B.clear(); B.shrink_to_fit();
    upload(ctx->row_ptr, S.near_ptr);
    upload(ctx->patch, S.near_patch);
    upload(ctx->w, S.w);
    upload(ctx->node_off, ctx->node_off_h);
    upload(ctx->node_surf, nsurf_of);
    upload(ctx->inv_area, inv);
    const bool direct = (o.flags & LB_DIRECT) != 0;
    // the FP32 rule has fewer points per patch: the same leaf boxes as the
    // FP64 tree hold proportionally fewer of them
    const int leaf_src32 = std::max(16, (int)((int64_t)o.leaf_src * S.o32.n_o / S.n_o));
    build_prec<float>(ctx, ctx->f32, o.p_f32, C32, rm2, rmax * (1.0 + 1e-6), leaf_src32, direct, nullptr,
                      dev_quad ? &dc.v4_32 : nullptr, dev_quad ? &dc.v3_32 : nullptr, dev_quad ? &dc.vD_32 : nullptr);
    C32.clear(); C32.shrink_to_fit();
    ctx->rm2f = std::move(rm2);
    // the float positions used by the mask test must be exactly the ones on the device
    build_prec<double>(ctx, ctx->f64, o.p_f64, ctx->C64, std::vector<float>(), 0.0, o.leaf_src, direct, nullptr,
                       dev_quad ? &dc.v4_64 : nullptr, dev_quad ? &dc.v3_64 : nullptr, dev_quad ? &dc.vD_64 : nullptr);
    HIPTRY(hipDeviceSynchronize());
  }
}
}  // namespace lb

}  // extern "C" (templates below)

namespace lb {
// ---------------------------------------------------------------------------
// Saved setups.  The corrections dominate the setup (the paper generates them
// once and reuses them for every solve on the geometry, and across the two
// solves of a Hodge decomposition); a saved setup holds the chart samples,
// the options, the near lists, the packed corrections of both precisions and
// the tuning of each precision.  Loading rebuilds the geometry and the near
// lists (checked against the saved ones), takes the corrections over instead
// of generating them, and rebuilds the octrees and translation operators.
// Layout (native byte order): magic "LBSETUP", version, byte-order word,
// sizeof(lb_opts), n_surf, order, opts, patches per surface, N, nnz blocks,
// n_p, six tuning words per precision (FP32, FP64), X, Xu, Xv, near_ptr,
// near_patch, FP64 values k=4 and k=3, FP32 values k=4 and k=3, and an
// FNV-1a checksum of everything before it.
// ---------------------------------------------------------------------------
static const char kSetupMagic[8] = {'L', 'B', 'S', 'E', 'T', 'U', 'P', 0};
constexpr uint32_t kSetupVersion = 2;  // 2: the double-layer corrections

struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
  }
};

struct FileW {
  FILE* f = nullptr;
  Fnv sum;
  explicit FileW(const char* path) : f(std::fopen(path, "wb")) {
    if (!f) fail(LB_EINVAL, "cannot open %s for writing", path);
  }
  ~FileW() { if (f) std::fclose(f); }
  void put(const void* p, size_t n) {
    if (n && std::fwrite(p, 1, n, f) != n) fail(LB_EINVAL, "write failed");
    sum.add(p, n);
  }
  template <typename T> void put(const std::vector<T>& v) { put(v.data(), sizeof(T) * v.size()); }
  template <typename T> void val(const T& x) { put(&x, sizeof(T)); }
};

struct FileR {
  FILE* f = nullptr;
  Fnv sum;
  explicit FileR(const char* path) : f(std::fopen(path, "rb")) {
    if (!f) fail(LB_EINVAL, "cannot open %s", path);
  }
  ~FileR() { if (f) std::fclose(f); }
  void get(void* p, size_t n) {
    if (n && std::fread(p, 1, n, f) != n) fail(LB_EINVAL, "saved setup is truncated");
    sum.add(p, n);
  }
  template <typename T> void get(std::vector<T>& v, size_t n) {
    v.resize(n);
    get(v.data(), sizeof(T) * n);
  }
  template <typename T> T val() { T x; get(&x, sizeof(T)); return x; }
};

template <typename T>
static void tuning_words(const Prec<T>& P, int32_t* w) {
  w[0] = P.build_leaf_src; w[1] = P.leaf_fmax; w[2] = P.leaf_split;
  w[3] = P.fork_late; w[4] = P.near_grid; w[5] = P.corr_early;
}

template <typename T>
static std::vector<T> device_copy(const DBuf& b, size_t n) {
  std::vector<T> h(n);
  if (n) HIPTRY(hipMemcpy(h.data(), b.p, sizeof(T) * n, hipMemcpyDeviceToHost));
  return h;
}

static void export_setup(const lb_ctx* ctx, const char* path) {
  if (ctx->host_only) fail(LB_EINVAL, "a LB_HOST_ONLY context holds no device corrections to save");
  const Surface& S = ctx->S;
  const int64_t nnzb = S.near_ptr[S.N];
  const size_t ne = (size_t)nnzb * S.n_p;
  HIPTRY(hipDeviceSynchronize());
  FileW w(path);
  w.put(kSetupMagic, 8);
  w.val<uint32_t>(kSetupVersion);
  w.val<uint32_t>(0x01020304u);
  w.val<uint32_t>((uint32_t)sizeof(lb_opts));
  w.val<int32_t>(ctx->n_surf);
  w.val<int32_t>(ctx->k);
  w.put(&ctx->opts, sizeof(lb_opts));
  for (int q = 0; q < ctx->n_surf; ++q) w.val<int32_t>(ctx->surf_patch[q + 1] - ctx->surf_patch[q]);
  w.val<int64_t>(S.N);
  w.val<int64_t>(nnzb);
  w.val<int32_t>(S.n_p);
  int32_t tw[12];
  tuning_words(ctx->f32, tw);
  tuning_words(ctx->f64, tw + 6);
  w.put(tw, sizeof(tw));
  w.put(S.X); w.put(S.Xu); w.put(S.Xv);
  w.put(S.near_ptr); w.put(S.near_patch);
  w.put(device_copy<double>(ctx->f64.vals4, ne * 4));
  w.put(device_copy<double>(ctx->f64.vals3, ne * 3));
  w.put(device_copy<float>(ctx->f32.vals4, ne * 4));
  w.put(device_copy<float>(ctx->f32.vals3, ne * 3));
  w.put(device_copy<double>(ctx->f64.valsD, ne));
  w.put(device_copy<float>(ctx->f32.valsD, ne));
  const uint64_t h = w.sum.h;
  w.val<uint64_t>(h);
}

template <typename T>
static void apply_tuning_words(lb_ctx* ctx, Prec<T>& P, bool& adj_built, bool& z_built, const int32_t* w) {
  lb_tune_info c{};
  c.leaf_src = w[0]; c.leaf_fmax = w[1]; c.leaf_split = w[2];
  c.fork_late = w[3]; c.near_grid = w[4]; c.corr_early = w[5];
  if (P.direct) c.leaf_src = P.build_leaf_src;
  if (c.leaf_src < 16 || c.leaf_fmax < 1 || c.leaf_fmax > 64 || (c.leaf_fmax & (c.leaf_fmax - 1)) ||
      c.leaf_split < 0 || c.leaf_split > 3 || c.near_grid < 0)
    fail(LB_EINVAL, "saved setup holds an invalid tuning");
  set_tuning_t<T>(ctx, P, adj_built, z_built, c);
}

static void import_setup(lb_ctx* ctx, const char* path) {
  FileR r(path);
  char magic[8];
  r.get(magic, 8);
  if (std::memcmp(magic, kSetupMagic, 8) != 0) fail(LB_EINVAL, "%s is not a saved setup", path);
  if (r.val<uint32_t>() != kSetupVersion) fail(LB_EINVAL, "saved setup version differs");
  if (r.val<uint32_t>() != 0x01020304u) fail(LB_EINVAL, "saved setup has another byte order");
  if (r.val<uint32_t>() != (uint32_t)sizeof(lb_opts)) fail(LB_EINVAL, "saved setup options differ in size");
  const int32_t n_surf = r.val<int32_t>();
  const int32_t order = r.val<int32_t>();
  if (n_surf < 1 || n_surf > (1 << 24) || order < 1 || order > 7) fail(LB_EINVAL, "saved setup header is corrupt");
  lb_opts opts;
  r.get(&opts, sizeof(lb_opts));
  std::vector<int32_t> pps;
  r.get(pps, (size_t)n_surf);
  int64_t NP = 0;
  for (int32_t c : pps) {
    if (c < 1) fail(LB_EINVAL, "saved setup header is corrupt");
    NP += c;
  }
  const int64_t N = r.val<int64_t>(), nnzb = r.val<int64_t>();
  const int32_t n_p = r.val<int32_t>();
  if (n_p != (order + 1) * (order + 2) / 2 || N != NP * n_p || nnzb < N || nnzb > N * NP)
    fail(LB_EINVAL, "saved setup sizes are inconsistent");
  int32_t tw[12];
  r.get(tw, sizeof(tw));
  std::vector<double> X, Xu, Xv;
  r.get(X, 3 * (size_t)N); r.get(Xu, 3 * (size_t)N); r.get(Xv, 3 * (size_t)N);
  std::vector<int64_t> nptr;
  std::vector<int32_t> npat;
  r.get(nptr, (size_t)N + 1);
  r.get(npat, (size_t)nnzb);
  const size_t ne = (size_t)nnzb * n_p;
  std::vector<double> v4d, v3d, vDd;
  std::vector<float> v4f, v3f, vDf;
  r.get(v4d, ne * 4); r.get(v3d, ne * 3); r.get(v4f, ne * 4); r.get(v3f, ne * 3);
  r.get(vDd, ne); r.get(vDf, ne);
  const uint64_t h = r.sum.h;
  if (r.val<uint64_t>() != h) fail(LB_EINVAL, "saved setup checksum mismatch (corrupt file)");
  if (opts.flags & LB_HOST_ONLY) fail(LB_EINVAL, "saved setup asks for a host-only context");
  DevCorrections dc;
  upload(dc.v4_64, v4d); upload(dc.v3_64, v3d); upload(dc.v4_32, v4f); upload(dc.v3_32, v3f);
  upload(dc.vD_64, vDd); upload(dc.vD_32, vDf);
  v4d.clear(); v3d.clear(); v4f.clear(); v3f.clear(); vDd.clear(); vDf.clear();
  setup_impl(ctx, n_surf, pps.data(), order, X.data(), Xu.data(), Xv.data(), &opts, &dc);
  if (ctx->S.near_ptr != nptr || ctx->S.near_patch != npat)
    fail(LB_EINVAL, "the near lists rebuilt from the saved charts differ from the saved ones");
  apply_tuning_words<float>(ctx, ctx->f32, ctx->adj_built32, ctx->z_built32, tw);
  apply_tuning_words<double>(ctx, ctx->f64, ctx->adj_built64, ctx->z_built64, tw + 6);
}
}  // namespace lb

extern "C" {

lb_status lb_setup(lb_ctx** out, int n_patches, int order, const double* X, const double* Xu, const double* Xv,
                   const lb_opts* opts, void* stream) {
  API_BEGIN
  (void)stream;
  if (!out) fail(LB_EINVAL, "null argument");
  *out = nullptr;
  if (n_patches < 1) fail(LB_EINVAL, "n_patches must be >= 1");
  const double t0 = wall_seconds();
  auto ctx = std::make_unique<lb_ctx>();
  const int32_t np = n_patches;
  setup_impl(ctx.get(), 1, &np, order, X, Xu, Xv, opts);
  ctx->t_setup = wall_seconds() - t0;
  *out = ctx.release();
  API_END
}

lb_status lb_setup_batch(lb_ctx** out, int n_surf, const int32_t* patches_per_surf, int order, const double* X,
                         const double* Xu, const double* Xv, const lb_opts* opts, void* stream) {
  API_BEGIN
  (void)stream;
  if (!out) fail(LB_EINVAL, "null argument");
  *out = nullptr;
  const double t0 = wall_seconds();
  auto ctx = std::make_unique<lb_ctx>();
  setup_impl(ctx.get(), n_surf, patches_per_surf, order, X, Xu, Xv, opts);
  ctx->t_setup = wall_seconds() - t0;
  *out = ctx.release();
  API_END
}

lb_status lb_export_setup(const lb_ctx* ctx, const char* path) {
  API_BEGIN
  if (!ctx || !path) fail(LB_EINVAL, "null argument");
  export_setup(ctx, path);
  API_END
}

lb_status lb_import_setup(lb_ctx** out, const char* path, void* stream) {
  API_BEGIN
  (void)stream;
  if (!out || !path) fail(LB_EINVAL, "null argument");
  *out = nullptr;
  const double t0 = wall_seconds();
  auto ctx = std::make_unique<lb_ctx>();
  import_setup(ctx.get(), path);
  ctx->t_setup = wall_seconds() - t0;
  *out = ctx.release();
  API_END
}

lb_status lb_get_sizes(const lb_ctx* ctx, lb_sizes* s) {
  API_BEGIN
  if (!ctx || !s) fail(LB_EINVAL, "null argument");
  s->n_patches = ctx->NP;
  s->n_p = ctx->n_p;
  s->N = ctx->N;
  s->n_o = ctx->n_o;
  s->N_o = ctx->No;
  s->n_o32 = ctx->S.o32.n_o;
  s->N_o32 = ctx->S.o32.No;
  s->nnz_blocks = ctx->S.near_ptr.empty() ? 0 : ctx->S.near_ptr.back();
  s->fmm_levels = 0;
  if (!ctx->host_only)
    for (const Octree& t : ctx->f32.trees) s->fmm_levels = std::max<int64_t>(s->fmm_levels, t.depth);
  s->n_surf = ctx->n_surf;
  s->fmm_leaves = ctx->host_only ? 0 : ctx->f32.dt.n_leaf_tgt;
  s->p_f32 = ctx->opts.p_f32;
  s->p_f64 = ctx->opts.p_f64;
  s->p2p_pairs32 = s->m2l_pairs32 = s->p2p_pairs64 = s->m2l_pairs64 = 0;
  if (!ctx->host_only) {
    auto count = [](const std::vector<Octree>& trees, int64_t& pp, int64_t& mp) {
      pp = mp = 0;
      for (const Octree& t : trees) {
        const int nleaf = (int)t.tgt_beg.size();
        for (int b = 0; b < nleaf; ++b) {
          int64_t ns = 0;
          for (int u = t.ulist_ptr[b]; u < t.ulist_ptr[b + 1]; ++u) ns += t.src_end[t.ulist[u]] - t.src_beg[t.ulist[u]];
          pp += ns * (t.tgt_end[b] - t.tgt_beg[b]);
        }
        mp += t.vlist_ptr.empty() ? 0 : t.vlist_ptr.back();
      }
    };
    count(ctx->f32.trees, s->p2p_pairs32, s->m2l_pairs32);
    count(ctx->f64.trees, s->p2p_pairs64, s->m2l_pairs64);
  }
  s->m2l_flops32 = (int64_t)ctx->f32.m2l_flops;
  s->m2l_flops64 = (int64_t)ctx->f64.m2l_flops;
  API_END
}

lb_status lb_get_geometry(const lb_ctx* ctx, double* w, double* normals, double* H) {
  API_BEGIN
  if (!ctx) fail(LB_EINVAL, "null context");
  const Surface& S = ctx->S;
  if (w) std::memcpy(w, S.w.data(), sizeof(double) * S.N);
  if (normals) std::memcpy(normals, S.nrm.data(), sizeof(double) * 3 * S.N);
  if (H) std::memcpy(H, S.H.data(), sizeof(double) * S.N);
  API_END
}

lb_status lb_get_corrections(const lb_ctx* ctx, int64_t* row_ptr, int32_t* patch, double* vals) {
  API_BEGIN
  if (!ctx) fail(LB_EINVAL, "null context");
  const Surface& S = ctx->S;
  if (row_ptr) std::memcpy(row_ptr, S.near_ptr.data(), sizeof(int64_t) * (S.N + 1));
  if (patch) std::memcpy(patch, S.near_patch.data(), sizeof(int32_t) * S.near_patch.size());
  if (vals && !ctx->C64.empty()) {
    std::memcpy(vals, ctx->C64.data(), sizeof(double) * ctx->C64.size());
  } else if (vals) {
    // generated on the device: unpack the FP64 combine layouts
    const size_t ne = (size_t)S.near_ptr[S.N] * S.n_p;
    std::vector<double> v4(ne * 4), v3(ne * 3), vD(ne);
    HIPTRY(hipMemcpy(v4.data(), ctx->f64.vals4.p, sizeof(double) * v4.size(), hipMemcpyDeviceToHost));
    HIPTRY(hipMemcpy(v3.data(), ctx->f64.vals3.p, sizeof(double) * v3.size(), hipMemcpyDeviceToHost));
    HIPTRY(hipMemcpy(vD.data(), ctx->f64.valsD.p, sizeof(double) * vD.size(), hipMemcpyDeviceToHost));
    for (size_t e = 0; e < ne; ++e) {
      for (int t = 0; t < 4; ++t) vals[NKER * e + t] = v4[4 * e + t];
      vals[NKER * e + 4] = v3[3 * e + 1];
      vals[NKER * e + 5] = v3[3 * e + 2];
      vals[NKER * e + 6] = vD[e];
    }
  }
  API_END
}

static void check_apply(lb_ctx* ctx, int nd, int prec) {
  if (!ctx) fail(LB_EINVAL, "null context");
  if (ctx->host_only) fail(LB_EINVAL, "context was set up with LB_HOST_ONLY");
  if (nd < 1) fail(LB_EINVAL, "nd must be >= 1");
  if (prec != LB_PREC_FP32 && prec != LB_PREC_FP64) fail(LB_EINVAL, "prec must be 32 or 64");
  int dev = -1;
  HIPTRY(hipGetDevice(&dev));
  if (dev != ctx->device) fail(LB_EINVAL, "current device %d differs from the context's %d", dev, ctx->device);
}

lb_status lb_apply_gradS(lb_ctx* ctx, int nd, int prec, const void* sigma, void* pot, void* grad, void* dSdn,
                         void* surf_grad, void* stream) {
  API_BEGIN
  check_apply(ctx, nd, prec);
  if (!sigma || !grad) fail(LB_EINVAL, "null sigma or grad");
  hipStream_t st = (hipStream_t)stream;
  if (prec == LB_PREC_FP32)
    apply_gradS_t<float>(ctx, ctx->f32, nd, (const float*)sigma, (float*)pot, (float*)grad, (float*)dSdn,
                         (float*)surf_grad, st);
  else
    apply_gradS_t<double>(ctx, ctx->f64, nd, (const double*)sigma, (double*)pot, (double*)grad, (double*)dSdn,
                          (double*)surf_grad, st);
  HIPTRY(hipGetLastError());
  API_END
}


lb_status lb_apply_gradS_noalloc(lb_ctx* ctx, int nd, int prec, const void* sigma, void* pot, void* grad,
                                 void* dSdn, void* surf_grad, void* stream) {
  API_BEGIN
  check_apply(ctx, nd, prec);
  if (!sigma || !grad) fail(LB_EINVAL, "null sigma or grad");
  hipStream_t st = (hipStream_t)stream;
  if (prec == LB_PREC_FP32) {
    const ApplyWs<float> w = scratch_ws<float>(ctx, ctx->f32, nd);
    apply_gradS_t<float>(ctx, ctx->f32, nd, (const float*)sigma, (float*)pot, (float*)grad, (float*)dSdn,
                         (float*)surf_grad, st, nullptr, &w);
  } else {
    const ApplyWs<double> w = scratch_ws<double>(ctx, ctx->f64, nd);
    apply_gradS_t<double>(ctx, ctx->f64, nd, (const double*)sigma, (double*)pot, (double*)grad, (double*)dSdn,
                          (double*)surf_grad, st, nullptr, &w);
  }
  HIPTRY(hipGetLastError());
  API_END
}

lb_status lb_apply_A1(lb_ctx* ctx, int nd, int prec, const void* tau, void* out, void* stream) {
  API_BEGIN
  check_apply(ctx, nd, prec);
  if (!tau || !out) fail(LB_EINVAL, "null tau or out");
  hipStream_t st = (hipStream_t)stream;
  if (prec == LB_PREC_FP32)
    apply_A1_t<float>(ctx, ctx->f32, ctx->a1_phi0_32, nd, (const float*)tau, (float*)out, st);
  else
    apply_A1_t<double>(ctx, ctx->f64, ctx->a1_phi0_64, nd, (const double*)tau, (double*)out, st);
  HIPTRY(hipGetLastError());
  API_END
}

lb_status lb_apply_A2(lb_ctx* ctx, int nd, int prec, const void* tau, void* out, void* stream) {
  API_BEGIN
  check_apply(ctx, nd, prec);
  if (!tau || !out) fail(LB_EINVAL, "null tau or out");
  hipStream_t st = (hipStream_t)stream;
  if (prec == LB_PREC_FP32)
    apply_A2_t<float>(ctx, ctx->f32, nd, (const float*)tau, (float*)out, st);
  else
    apply_A2_t<double>(ctx, ctx->f64, nd, (const double*)tau, (double*)out, st);
  HIPTRY(hipGetLastError());
  API_END
}

lb_status lb_apply_gradS_adj(lb_ctx* ctx, int nd, int prec, const void* gpot, const void* ggrad,
                             const void* gdSdn, const void* gsurf, void* sigma_bar, void* stream) {
  API_BEGIN
  check_apply(ctx, nd, prec);
  if (!sigma_bar) fail(LB_EINVAL, "null sigma_bar");
  if (!gpot && !ggrad && !gdSdn && !gsurf) fail(LB_EINVAL, "all cotangents are null");
  hipStream_t st = (hipStream_t)stream;
  if (prec == LB_PREC_FP32)
    apply_adj_t<float>(ctx, ctx->f32, ctx->a32, ctx->adj_built32, nd, (const float*)gpot, (const float*)ggrad,
                       (const float*)gdSdn, (const float*)gsurf, (float*)sigma_bar, st);
  else
    apply_adj_t<double>(ctx, ctx->f64, ctx->a64, ctx->adj_built64, nd, (const double*)gpot, (const double*)ggrad,
                        (const double*)gdSdn, (const double*)gsurf, (double*)sigma_bar, st);
  HIPTRY(hipGetLastError());
  API_END
}

lb_status lb_apply_S_adj(lb_ctx* ctx, int nd, int prec, const void* gbar, void* sigma_bar, void* stream) {
  if (!gbar) {
    lb::set_last_error("null gbar");
    return LB_EINVAL;
  }
  return lb_apply_gradS_adj(ctx, nd, prec, gbar, nullptr, nullptr, nullptr, sigma_bar, stream);
}

lb_status lb_apply_S_adj_X(lb_ctx* ctx, int nd, int prec, const void* sigma, const void* gbar, void* X_bar,
                          void* stream) {
  API_BEGIN
  check_apply(ctx, nd, prec);
  if (!sigma || !gbar || !X_bar) fail(LB_EINVAL, "null sigma, gbar or X_bar");
  hipStream_t st = (hipStream_t)stream;
  if (prec == LB_PREC_FP32)
    apply_S_xbar_t<float>(ctx, ctx->f32, ctx->a32, ctx->adj_built32, nd, (const float*)sigma, (const float*)gbar,
                          (float*)X_bar, st);
  else
    apply_S_xbar_t<double>(ctx, ctx->f64, ctx->a64, ctx->adj_built64, nd, (const double*)sigma,
                           (const double*)gbar, (double*)X_bar, st);
  HIPTRY(hipGetLastError());
  API_END
}

lb_status lb_autotune(lb_ctx* ctx, int prec, int nd, lb_tune_info* info, void* stream) {
  API_BEGIN
  check_apply(ctx, nd, prec);
  if (nd > 64) fail(LB_EINVAL, "autotune takes at most 64 densities");
  hipStream_t st = (hipStream_t)stream;
  lb_tune_info r{};
  if (prec == LB_PREC_FP32)
    autotune_t<float>(ctx, ctx->f32, ctx->adj_built32, ctx->z_built32, nd, r, st);
  else
    autotune_t<double>(ctx, ctx->f64, ctx->adj_built64, ctx->z_built64, nd, r, st);
  if (info) *info = r;
  API_END
}

lb_status lb_set_tuning(lb_ctx* ctx, int prec, const lb_tune_info* config) {
  API_BEGIN
  check_apply(ctx, 1, prec);
  if (!config) fail(LB_EINVAL, "null config");
  const lb_tune_info& c = *config;
  if (c.leaf_src < 16 || c.leaf_src > (1 << 20)) fail(LB_EINVAL, "leaf_src %d out of range 16..2^20", c.leaf_src);
  if (c.leaf_fmax < 1 || c.leaf_fmax > 64 || (c.leaf_fmax & (c.leaf_fmax - 1)))
    fail(LB_EINVAL, "leaf_fmax must be a power of two in 1..64");
  if (c.leaf_split < 0 || c.leaf_split > 3) fail(LB_EINVAL, "leaf_split must be 0..3");
  if ((c.fork_late != 0 && c.fork_late != 1) || c.near_grid < 0 || (c.corr_early != 0 && c.corr_early != 1))
    fail(LB_EINVAL, "bad schedule");
  if (prec == LB_PREC_FP32)
    set_tuning_t<float>(ctx, ctx->f32, ctx->adj_built32, ctx->z_built32, c);
  else
    set_tuning_t<double>(ctx, ctx->f64, ctx->adj_built64, ctx->z_built64, c);
  API_END
}

lb_status lb_apply_A3_adj(lb_ctx* ctx, int nd, int prec, const void* v, void* out, void* stream) {
  API_BEGIN
  check_apply(ctx, nd, prec);
  if (!v || !out) fail(LB_EINVAL, "null v or out");
  hipStream_t st = (hipStream_t)stream;
  if (prec == LB_PREC_FP32)
    apply_A3T_t<float>(ctx, ctx->f32, ctx->a32, ctx->adj_built32, ctx->z32, ctx->z_built32, nd, (const float*)v,
                       (float*)out, st);
  else
    apply_A3T_t<double>(ctx, ctx->f64, ctx->a64, ctx->adj_built64, ctx->z64, ctx->z_built64, nd, (const double*)v,
                        (double*)out, st);
  HIPTRY(hipGetLastError());
  API_END
}

lb_status lb_apply_gradS_timed(lb_ctx* ctx, int nd, int prec, const void* sigma, void* pot, void* grad,
                               void* dSdn, void* surf_grad, double* phase_ms, void* stream) {
  API_BEGIN
  check_apply(ctx, nd, prec);
  if (!sigma || !grad || !phase_ms) fail(LB_EINVAL, "null sigma, grad or phase_ms");
  if (nd > CHUNK_GRAD) fail(LB_EINVAL, "timed apply takes at most %d densities", CHUNK_GRAD);
  hipStream_t st = (hipStream_t)stream;
  PhaseTimer tm;
  tm.on = true;
  for (int i = 0; i <= PH_N; ++i) HIPTRY(hipEventCreate(&tm.ev[i]));
  if (prec == LB_PREC_FP32)
    apply_gradS_t<float>(ctx, ctx->f32, nd, (const float*)sigma, (float*)pot, (float*)grad, (float*)dSdn,
                         (float*)surf_grad, st, &tm);
  else
    apply_gradS_t<double>(ctx, ctx->f64, nd, (const double*)sigma, (double*)pot, (double*)grad, (double*)dSdn,
                          (double*)surf_grad, st, &tm);
  HIPTRY(hipEventSynchronize(tm.ev[PH_N]));
  for (int i = 0; i < PH_N; ++i) {
    float ms = 0;
    HIPTRY(hipEventElapsedTime(&ms, tm.ev[i], tm.ev[i + 1]));
    phase_ms[i] = ms;
  }
  for (int i = 0; i <= PH_N; ++i) (void)hipEventDestroy(tm.ev[i]);
  API_END
}

namespace lb {
static void export_tree(const Octree& t, lb_tree_info* info, int64_t* tgt_perm, int64_t* src_perm,
                        int32_t* leaf_ranges, int32_t* ulist_ptr, int32_t* ulist, int32_t* vlist_ptr,
                        int32_t* vlist_src, int32_t* vlist_off, int32_t* boxes) {
  const int nb = t.nbox(), nleaf = t.lev_off[t.depth + 1] - t.lev_off[t.depth];
  if (info) {
    info->depth = t.depth;
    info->nbox = nb;
    info->nleaf = nleaf;
    info->nulist = (int32_t)t.ulist.size();
    info->nvlist = (int32_t)t.vlist_src.size();
    for (int d = 0; d < 3; ++d) info->lo[d] = t.lo[d];
    info->side = t.side;
  }
  if (tgt_perm) std::copy(t.tgt_perm.begin(), t.tgt_perm.end(), tgt_perm);
  if (src_perm) std::copy(t.src_perm.begin(), t.src_perm.end(), src_perm);
  if (leaf_ranges)
    for (int b = 0; b < nleaf; ++b) {
      leaf_ranges[4 * b] = t.tgt_beg[b];
      leaf_ranges[4 * b + 1] = t.tgt_end[b];
      leaf_ranges[4 * b + 2] = t.src_beg[b];
      leaf_ranges[4 * b + 3] = t.src_end[b];
    }
  if (ulist_ptr) std::copy(t.ulist_ptr.begin(), t.ulist_ptr.end(), ulist_ptr);
  if (ulist) std::copy(t.ulist.begin(), t.ulist.end(), ulist);
  if (vlist_ptr) std::copy(t.vlist_ptr.begin(), t.vlist_ptr.end(), vlist_ptr);
  if (vlist_src) std::copy(t.vlist_src.begin(), t.vlist_src.end(), vlist_src);
  if (vlist_off) std::copy(t.vlist_off.begin(), t.vlist_off.end(), vlist_off);
  if (boxes)
    for (int l = 0; l <= t.depth; ++l)
      for (int g = t.lev_off[l]; g < t.lev_off[l + 1]; ++g) {
        boxes[5 * g] = l;
        boxes[5 * g + 1] = t.bx[g];
        boxes[5 * g + 2] = t.by[g];
        boxes[5 * g + 3] = t.bz[g];
        boxes[5 * g + 4] = (t.has_tgt[g] ? 1 : 0) | (t.has_src[g] ? 2 : 0);
      }
}
}  // namespace lb

struct lb_tree {
  Octree t;
};

lb_status lb_tree_build(lb_tree** out, const double* tgt, int64_t nt, const double* src, int64_t ns, int leaf_src,
                        double min_leaf_side, int depth, int on_device) {
  API_BEGIN
  if (!out || !tgt || !src) fail(LB_EINVAL, "null argument");
  *out = nullptr;
  if (nt < 1 || ns < 1) fail(LB_EINVAL, "empty point set");
  if (depth > 20) fail(LB_EINVAL, "depth must be <= 20");
  if (depth < 0 && leaf_src < 1) fail(LB_EINVAL, "leaf_src must be >= 1");
  for (int64_t i = 0; i < 3 * nt; ++i)
    if (!std::isfinite(tgt[i])) fail(LB_EINVAL, "non-finite target coordinate");
  for (int64_t i = 0; i < 3 * ns; ++i)
    if (!std::isfinite(src[i])) fail(LB_EINVAL, "non-finite source coordinate");
  auto t = std::make_unique<lb_tree>();
  if (on_device)
    t->t.build_device(tgt, nt, src, ns, leaf_src, min_leaf_side, depth);
  else
    t->t.build(tgt, nt, src, ns, leaf_src, min_leaf_side, depth);
  *out = t.release();
  API_END
}

lb_status lb_tree_get(const lb_tree* tree, lb_tree_info* info, int64_t* tgt_perm, int64_t* src_perm,
                      int32_t* leaf_ranges, int32_t* ulist_ptr, int32_t* ulist, int32_t* vlist_ptr,
                      int32_t* vlist_src, int32_t* vlist_off, int32_t* boxes) {
  API_BEGIN
  if (!tree) fail(LB_EINVAL, "null tree");
  export_tree(tree->t, info, tgt_perm, src_perm, leaf_ranges, ulist_ptr, ulist, vlist_ptr, vlist_src, vlist_off,
              boxes);
  API_END
}

void lb_tree_destroy(lb_tree* tree) { delete tree; }

lb_status lb_get_tree(const lb_ctx* ctx, int prec, int transposed, int surf, lb_tree_info* info, int64_t* tgt_perm,
                      int64_t* src_perm, int32_t* leaf_ranges, int32_t* ulist_ptr, int32_t* ulist,
                      int32_t* vlist_ptr, int32_t* vlist_src, int32_t* vlist_off, int32_t* boxes) {
  API_BEGIN
  if (!ctx) fail(LB_EINVAL, "null context");
  if (ctx->host_only) fail(LB_EINVAL, "context was set up with LB_HOST_ONLY (no tree)");
  if (prec != LB_PREC_FP32 && prec != LB_PREC_FP64) fail(LB_EINVAL, "prec must be 32 or 64");
  const bool built = prec == LB_PREC_FP32 ? ctx->adj_built32 : ctx->adj_built64;
  if (transposed && !built) fail(LB_EINVAL, "the transposed tree is built by the first adjoint apply");
  if (surf < 0 || surf >= ctx->n_surf) fail(LB_EINVAL, "surface %d out of range", surf);
  const Octree& t = prec == LB_PREC_FP32 ? (transposed ? ctx->a32.trees[surf] : ctx->f32.trees[surf])
                                         : (transposed ? ctx->a64.trees[surf] : ctx->f64.trees[surf]);
  export_tree(t, info, tgt_perm, src_perm, leaf_ranges, ulist_ptr, ulist, vlist_ptr, vlist_src, vlist_off, boxes);
  API_END
}

lb_status lb_apply_S(lb_ctx* ctx, int nd, int prec, const void* sigma, void* pot, void* stream) {
  API_BEGIN
  check_apply(ctx, nd, prec);
  if (!sigma || !pot) fail(LB_EINVAL, "null sigma or pot");
  hipStream_t st = (hipStream_t)stream;
  if (prec == LB_PREC_FP32)
    apply_S_t<float>(ctx, ctx->f32, nd, (const float*)sigma, (float*)pot, st);
  else
    apply_S_t<double>(ctx, ctx->f64, nd, (const double*)sigma, (double*)pot, st);
  HIPTRY(hipGetLastError());
  API_END
}

lb_status lb_apply_A3(lb_ctx* ctx, int nd, int prec, const void* tau, void* out, void* stream) {
  API_BEGIN
  check_apply(ctx, nd, prec);
  if (!tau || !out) fail(LB_EINVAL, "null tau or out");
  hipStream_t st = (hipStream_t)stream;
  if (prec == LB_PREC_FP32)
    apply_A3_t<float>(ctx, ctx->f32, nd, (const float*)tau, (float*)out, st);
  else
    apply_A3_t<double>(ctx, ctx->f64, nd, (const double*)tau, (double*)out, st);
  HIPTRY(hipGetLastError());
  API_END
}

lb_status lb_solve(lb_ctx* ctx, int nrhs, const double* f, double* u, double tol, int mode, lb_solve_info* info,
                   void* stream) {
  API_BEGIN
  const double t_start = wall_seconds();
  check_apply(ctx, nrhs, LB_PREC_FP64);
  if (!f || !u) fail(LB_EINVAL, "null f or u");
  if (!(tol > 0)) fail(LB_EINVAL, "tol must be > 0");
  // formulation: A3 (eq. ie-dis2, u = S S sigma) or, with LB_SOLVE_A2, A2
  // (eq. ie-dis1: A2 sigma = S f, u = S sigma)
  const bool a2 = (mode & LB_SOLVE_A2) != 0;
  mode &= ~LB_SOLVE_A2;
  if (mode != LB_SOLVE_FP64 && mode != LB_SOLVE_FP32_REFINE) fail(LB_EINVAL, "unknown mode");
  hipStream_t st = (hipStream_t)stream;
  const int64_t N = ctx->N;
  const int nsf = ctx->n_surf;
  ensure_ws(ctx, ctx->f64, CHUNK_GRAD);
  ensure_ws(ctx, ctx->f32, CHUNK_GRAD);
  if (a2) {
    a2_ws<double>(ctx, ctx->f64);
    a2_ws<float>(ctx, ctx->f32);
  }
  const size_t nN = (size_t)nrhs * N;
  ctx->r.alloc(sizeof(double) * nN);
  ctx->sig.alloc(sizeof(double) * nN);
  ctx->ftmp.alloc(sizeof(double) * nN);
  ctx->utmp.alloc(sizeof(double) * nN * 2);
  ctx->f32.tmp_in.alloc(sizeof(float) * nN);
  ctx->f32.tmp_out.alloc(sizeof(float) * nN);
  double* r = dptr<double>(ctx->r);
  double* sig = dptr<double>(ctx->sig);
  double* fz = dptr<double>(ctx->ftmp);
  double* ut = dptr<double>(ctx->utmp);
  double* dcorr = ut + nN;
  auto A64 = [&](const double* v, double* w, int na, hipStream_t s2) {
    if (a2)
      apply_A2_t<double>(ctx, ctx->f64, na, v, w, s2);
    else
      apply_A3_t<double>(ctx, ctx->f64, na, v, w, s2);
  };
  auto A32 = [&](const double* v, double* w, int na, hipStream_t s2) {
    float* vi = dptr<float>(ctx->f32.tmp_in);
    float* vo = dptr<float>(ctx->f32.tmp_out);
    launch_convert<double, float>(v, vi, (int64_t)na * N, s2);
    if (a2)
      apply_A2_t<float>(ctx, ctx->f32, na, vi, vo, s2);
    else
      apply_A3_t<float>(ctx, ctx->f32, na, vi, vo, s2);
    launch_convert<float, double>(vo, w, (int64_t)na * N, s2);
  };
  // mean projection per surface (Lemma 1): fz = f - (sum_q w f / area_q) on surface q
  DBuf means;
  means.alloc(sizeof(double) * (size_t)nrhs * nsf);
  launch_seg_dot<double>(nrhs, nsf, N, dptr<int64_t>(ctx->node_off), f, dptr<double>(ctx->w),
                         dptr<double>(ctx->inv_area), dptr<double>(means), st);
  launch_seg_axpy<double>(nrhs, nsf, N, dptr<int>(ctx->node_surf), f, -1.0, nullptr, dptr<double>(means), fz, st);
  std::vector<double> mean((size_t)nrhs * nsf);
  HIPTRY(hipMemcpyAsync(mean.data(), means.p, sizeof(double) * mean.size(), hipMemcpyDeviceToHost, st));
  const Systems sy = make_systems(ctx, nrhs);
  const std::vector<double> fn = system_norms(ctx, sy, f, st);
  if (ctx->opts.flags & LB_STRICT_MEAN) {
    for (size_t a = 0; a < fn.size(); ++a)
      if (std::fabs(mean[a]) > 1e-12 * fn[a])
        fail(LB_ENOTMEANZERO, "right-hand side %d (surface %d) has weighted mean %g", (int)(a / nsf), (int)(a % nsf),
             mean[a]);
  }
  std::vector<double> fnorm = system_norms(ctx, sy, fz, st);
  // a right-hand side that is constant up to rounding leaves only rounding
  // noise after the projection: it is the zero right-hand side (u = 0)
  for (size_t a = 0; a < fnorm.size(); ++a)
    if (fnorm[a] > 0 && fnorm[a] <= 1e-13 * fn[a]) {
      HIPTRY(hipMemsetAsync(fz + sy.xoff[a], 0, sizeof(double) * (size_t)sy.len[a], st));
      fnorm[a] = 0.0;
    }
  std::vector<double> rel;
  std::vector<int> iters, outer;
  if (a2) {
    // the right-hand side S f of eq. ie-dis1, its norms for the residual test
    ctx->a2b.alloc(sizeof(double) * nN);
    double* b = dptr<double>(ctx->a2b);
    apply_S_t<double>(ctx, ctx->f64, nrhs, fz, b, st);
    std::vector<double> bnorm = system_norms(ctx, sy, b, st);
    for (size_t a = 0; a < bnorm.size(); ++a)
      if (fnorm[a] == 0.0) bnorm[a] = 0.0;
    solve_system(ctx, nrhs, sy, A64, A32, ctx->gI64a2, ctx->gI32a2, ctx->gR64a2, b, bnorm, sig, r, ut, dcorr, tol,
                 mode, rel, iters, outer, st);
    // u = S[sigma] in FP64
    apply_S_t<double>(ctx, ctx->f64, nrhs, sig, u, st);
  } else {
    solve_system(ctx, nrhs, sy, A64, A32, ctx->gI64, ctx->gI32, ctx->gR64, fz, fnorm, sig, r, ut, dcorr, tol, mode,
                 rel, iters, outer, st);
    // u = S[S[sigma]] in FP64
    apply_S_t<double>(ctx, ctx->f64, nrhs, sig, ut, st);
    apply_S_t<double>(ctx, ctx->f64, nrhs, ut, u, st);
  }
  HIPTRY(hipStreamSynchronize(st));
  const double t_solve = wall_seconds() - t_start;
  lb_status ret = LB_OK;
  for (size_t a = 0; a < rel.size(); ++a) {
    if (!(rel[a] < tol)) ret = LB_ENOCONV;
    if (info) {
      info[a].iters = iters[a];
      info[a].outer_steps = mode == LB_SOLVE_FP64 ? 0 : std::max(outer[a] - 1, 0);
      info[a].rel_resid = rel[a];
      info[a].removed_mean = mean[a];
      info[a].t_setup = ctx->t_setup;
      info[a].t_solve = t_solve;
    }
  }
  if (ret != LB_OK) {
    lb::set_last_error("GMRES did not reach the tolerance for some right-hand side");
    return ret;
  }
  API_END
}

namespace lb {
static SurfCalcArgs calc_args(lb_ctx* ctx) {
  if (!ctx->calc_built) {
    upload(ctx->c_Du, ctx->re->Du);
    upload(ctx->c_Dv, ctx->re->Dv);
    upload(ctx->c_Xu, ctx->S.Xu);
    upload(ctx->c_Xv, ctx->S.Xv);
    upload(ctx->c_nrm, ctx->S.nrm);
    ctx->calc_built = true;
  }
  SurfCalcArgs q;
  q.Du = dptr<double>(ctx->c_Du);
  q.Dv = dptr<double>(ctx->c_Dv);
  q.Xu = dptr<double>(ctx->c_Xu);
  q.Xv = dptr<double>(ctx->c_Xv);
  q.nrm = dptr<double>(ctx->c_nrm);
  q.N = ctx->N;
  q.n_p = ctx->n_p;
  return q;
}
}  // namespace lb

lb_status lb_surface_grad(lb_ctx* ctx, int nd, const double* psi, double* grad, void* stream) {
  API_BEGIN
  check_apply(ctx, nd, LB_PREC_FP64);
  if (!psi || !grad) fail(LB_EINVAL, "null psi or grad");
  HIPTRY(launch_surf_grad(calc_args(ctx), nd, psi, grad, (hipStream_t)stream));
  API_END
}

lb_status lb_surface_div(lb_ctx* ctx, int nd, const double* V, int cross_n, double* div, void* stream) {
  API_BEGIN
  check_apply(ctx, nd, LB_PREC_FP64);
  if (!V || !div) fail(LB_EINVAL, "null V or div");
  if (cross_n != 0 && cross_n != 1) fail(LB_EINVAL, "cross_n must be 0 or 1");
  HIPTRY(launch_surf_div(calc_args(ctx), nd, V, cross_n, 1.0, div, (hipStream_t)stream));
  API_END
}

lb_status lb_hodge(lb_ctx* ctx, int nf, const double* F, double* alpha, double* beta, double* H, double tol,
                   int mode, lb_solve_info* info, void* stream) {
  API_BEGIN
  check_apply(ctx, nf, LB_PREC_FP64);
  if (!F || !H) fail(LB_EINVAL, "null F or H");
  hipStream_t st = (hipStream_t)stream;
  const SurfCalcArgs q = calc_args(ctx);
  const size_t nN = (size_t)nf * ctx->N;
  DBuf rhs, u;
  rhs.alloc(sizeof(double) * nN * 2);
  u.alloc(sizeof(double) * nN * 2);
  double* r = dptr<double>(rhs);
  double* uu = dptr<double>(u);
  // Delta alpha = div F (rows 0..nf-1), Delta beta = -div(n x F) (rows nf..2nf-1)
  HIPTRY(launch_surf_div(q, nf, F, 0, 1.0, r, st));
  HIPTRY(launch_surf_div(q, nf, F, 1, -1.0, r + nN, st));
  const lb_status status = lb_solve(ctx, 2 * nf, r, uu, tol, mode, info, stream);
  if (status < 0) return status;
  HIPTRY(launch_hodge_h(q, nf, F, uu, uu + nN, H, st));
  if (alpha) HIPTRY(hipMemcpyAsync(alpha, uu, sizeof(double) * nN, hipMemcpyDeviceToDevice, st));
  if (beta) HIPTRY(hipMemcpyAsync(beta, uu + nN, sizeof(double) * nN, hipMemcpyDeviceToDevice, st));
  HIPTRY(hipStreamSynchronize(st));
  if (status != LB_OK) return status;
  API_END
}

lb_status lb_solve_adj(lb_ctx* ctx, int nrhs, const double* ubar, double* fbar, double tol, int mode,
                       lb_solve_info* info, void* stream) {
  API_BEGIN
  const double t_start = wall_seconds();
  check_apply(ctx, nrhs, LB_PREC_FP64);
  if (!ubar || !fbar) fail(LB_EINVAL, "null ubar or fbar");
  if (!(tol > 0)) fail(LB_EINVAL, "tol must be > 0");
  if (mode != LB_SOLVE_FP64 && mode != LB_SOLVE_FP32_REFINE) fail(LB_EINVAL, "unknown mode");
  hipStream_t st = (hipStream_t)stream;
  const int64_t N = ctx->N;
  const int nsf = ctx->n_surf;
  ensure_ws(ctx, ctx->f64, CHUNK_GRAD);
  ensure_ws(ctx, ctx->f32, CHUNK_GRAD);
  const size_t nN = (size_t)nrhs * N;
  ctx->r.alloc(sizeof(double) * nN);
  ctx->sig.alloc(sizeof(double) * nN);
  ctx->ftmp.alloc(sizeof(double) * nN);
  ctx->utmp.alloc(sizeof(double) * nN * 2);
  ctx->f32.tmp_in.alloc(sizeof(float) * nN);
  ctx->f32.tmp_out.alloc(sizeof(float) * nN);
  double* r = dptr<double>(ctx->r);
  double* y = dptr<double>(ctx->sig);
  double* rhs = dptr<double>(ctx->ftmp);
  double* ut = dptr<double>(ctx->utmp);
  double* dcorr = ut + nN;
  auto A64 = [&](const double* v, double* w, int na, hipStream_t s2) {
    apply_A3T_t<double>(ctx, ctx->f64, ctx->a64, ctx->adj_built64, ctx->z64, ctx->z_built64, na, v, w, s2);
  };
  auto A32 = [&](const double* v, double* w, int na, hipStream_t s2) {
    float* vi = dptr<float>(ctx->f32.tmp_in);
    float* vo = dptr<float>(ctx->f32.tmp_out);
    launch_convert<double, float>(v, vi, (int64_t)na * N, s2);
    apply_A3T_t<float>(ctx, ctx->f32, ctx->a32, ctx->adj_built32, ctx->z32, ctx->z_built32, na, vi, vo, s2);
    launch_convert<float, double>(vo, w, (int64_t)na * N, s2);
  };
  // rhs = S^T S^T ubar (adjoint of u = S[S[sigma]])
  apply_adj_t<double>(ctx, ctx->f64, ctx->a64, ctx->adj_built64, nrhs, ubar, nullptr, nullptr, nullptr, ut, st);
  apply_adj_t<double>(ctx, ctx->f64, ctx->a64, ctx->adj_built64, nrhs, ut, nullptr, nullptr, nullptr, rhs, st);
  const Systems sy = make_systems(ctx, nrhs);
  const std::vector<double> bnorm = system_norms(ctx, sy, rhs, st);
  std::vector<double> rel;
  std::vector<int> iters, outer;
  solve_system(ctx, nrhs, sy, A64, A32, ctx->gIT64, ctx->gIT32, ctx->gRT64, rhs, bnorm, y, r, ut, dcorr, tol, mode,
               rel, iters, outer, st);
  // fbar = (I - w 1^T / area_q) y on each surface q: the transposed mean projection
  DBuf sc;
  sc.alloc(sizeof(double) * (size_t)nrhs * nsf);
  launch_seg_dot<double>(nrhs, nsf, N, dptr<int64_t>(ctx->node_off), y, nullptr, dptr<double>(ctx->inv_area),
                         dptr<double>(sc), st);
  launch_seg_axpy<double>(nrhs, nsf, N, dptr<int>(ctx->node_surf), y, -1.0, dptr<double>(ctx->w), dptr<double>(sc),
                          fbar, st);
  std::vector<double> removed((size_t)nrhs * nsf);
  HIPTRY(hipMemcpyAsync(removed.data(), sc.p, sizeof(double) * removed.size(), hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  const double t_solve = wall_seconds() - t_start;
  lb_status ret = LB_OK;
  for (size_t a = 0; a < rel.size(); ++a) {
    if (!(rel[a] < tol)) ret = LB_ENOCONV;
    if (info) {
      info[a].iters = iters[a];
      info[a].outer_steps = mode == LB_SOLVE_FP64 ? 0 : std::max(outer[a] - 1, 0);
      info[a].rel_resid = rel[a];
      info[a].removed_mean = removed[a];
      info[a].t_setup = ctx->t_setup;
      info[a].t_solve = t_solve;
    }
  }
  if (ret != LB_OK) {
    lb::set_last_error("GMRES did not reach the tolerance for some right-hand side");
    return ret;
  }
  API_END
}

void lb_destroy(lb_ctx* ctx) {
  if (!ctx) return;
  try {
    if (!ctx->host_only) (void)hipSetDevice(ctx->device);
    delete ctx;
  } catch (...) {
  }
}

}  // extern "C"
