// Launch wrappers of the HIP kernels (plain pointers, stream ordered).
#pragma once
#include <cstdint>
#include <hip/hip_runtime.h>

#include "nker.hpp"

namespace lb {

// FMM output sets at the targets (tree order), per right-hand side:
//   FMM_POT : phi
//   FMM_GRAD: phi, d/dx phi, d/dy phi, d/dz phi
//   FMM_A3B : n.grad phi_1, phi_2, n.grad phi_2, n.gradgrad phi_2.n + n.grad phi_3
//             (expansions per rhs: charge mu1, charge mu2, dipole mu2 * nu)
//   FMM_ADJ : psi = sum_j q_j / r + d_j . (x - y_j) / r^3 (sources with a
//             charge q_j and a dipole vector d_j: strengths q, dx, dy, dz;
//             the mask radius belongs to the target on the transposed tree,
//             see DevTree::trm2, and to the source on the forward tree)
//   FMM_ADJ3: the far part of the first step of the transposed A3, at
//             targets x with normal nu from sources y_j with normal n_j and
//             strengths v_j, w_j (d = x - y_j, m = n_j - nu):
//               psi_a = sum_j v_j (n_j . d) / r^3                 (S'^T)
//               psi_b = sum_j v_j (3 (n_j . d)(m . d) / r^5 - (n_j . m) / r^3)
//                     + w_j (n_j . d) / r^3                       ((S''+D')^T, S'^T)
//             through a dipole expansion (v n; potential and gradient) and
//             a quadrupole + dipole expansion (v n n^T, w n; potential):
//             psi_b = phi_2 + nu . grad phi_1
// phi = sum_j c_j / |x - y_j| (no 1/(4 pi)).
enum FmmMode { FMM_POT = 0, FMM_GRAD = 1, FMM_A3B = 2, FMM_ADJ = 3, FMM_ADJ3 = 4 };
__host__ __device__ inline int fmm_nout(int mode) {
  return mode == FMM_POT || mode == FMM_ADJ ? 1 : (mode == FMM_ADJ3 ? 2 : 4);
}
__host__ __device__ inline int fmm_nexp(int mode) { return mode == FMM_A3B ? 3 : (mode == FMM_ADJ3 ? 2 : 1); }
__host__ __device__ inline int fmm_nstr(int mode) {
  return mode == FMM_A3B || mode == FMM_ADJ3 ? 2 : (mode == FMM_ADJ ? 4 : 1);
}

// Batched translation plan: (matrix id, source box, target box) triples
// sorted by (matrix, target).  Each matrix group is one GEMM
// Y[:, c] = T_mat X[src(c)] over columns c = (triple, expansion); then every
// target box sums its columns (scaled by its level factor when `scaled`)
// into (or onto, when `accumulate`) its coefficient vector.  Column tiles are
// 64 wide; work[ne] lists (group, first column) for ne expansions per box.
// Output tile of the grouped translation GEMM: rows x columns per block.
constexpr int GEMM_TILE_ROWS = 128, GEMM_TILE_COLS = 64;
// Number of XCDs of the device: consecutive workgroups go to the XCDs in
// turn, each XCD with its own L2.
constexpr int GEMM_NXCD = 8;

// Most expansions one FMM traversal may carry (FP32; the FP64 plans stop at
// 8): sixteen densities of a gradient apply or of the second A3 pass (three
// expansions each).
constexpr int GEMM_NE_MAX = 48;

struct GemmPlan {
  int ngrp = 0, npair = 0, nbox = 0;
  const int *grp_mat = nullptr, *grp_beg = nullptr;  // [ngrp], [ngrp+1] (triple index)
  const int *pair_src = nullptr;                      // [npair] source box
  // active size of each group's translation (nullable: L): the leading
  // grp_lo[g] coefficients in and out (a lower expansion order); pair_lo
  // [npair] the same per pair, for the column reduction
  const int *grp_lo = nullptr, *pair_lo = nullptr;
  const int* boxes = nullptr;                         // [nbox] target boxes
  const double* box_scale = nullptr;                  // [nbox] factor of each target box (scaled plans)
  const int *tptr = nullptr, *tpairs = nullptr;       // [nbox+1], [npair]
  // per expansion count ne (1..ne_max; built for the counts the applies use,
  // null for the others): work items (group, first column, first row, first
  // k), ordered group -> row tile -> column tile -> k slice
  const int* work[GEMM_NE_MAX + 1] = {nullptr};
  int nwork[GEMM_NE_MAX + 1] = {0};
  int ne_max = 0;
  // k split: slices of kslice coefficients (0: the whole sum in one block);
  // slice s of column c goes to Y[s][c], and the column reduction adds the
  // nslice slices
  int kslice = 0, nslice = 1;
  bool scaled = false, accumulate = false;
};

template <typename T>
struct DevTree {
  // geometry in tree order
  const T *tx, *ty, *tz, *tnx, *tny, *tnz;       // targets
  const T *sx, *sy, *sz, *snx, *sny, *snz;       // sources
  const T *rm2;                                  // squared mask radius per source
  const T *trm2;                                 // squared mask radius per target (FMM_ADJ)
  const T *bcx, *bcy, *bcz;                      // box centres [nbox]
  const int *tgt_beg, *tgt_end, *src_beg, *src_end;  // per leaf
  const int *ulist_ptr, *ulist;
  const int *vlist_ptr, *vlist_src, *vlist_off;
  const int *parent;
  const int *child;                              // [nbox][8]
  const int *child_src;                          // [nbox][8], -1 unless the child holds sources
  const int *leaf_tgt_list;  int n_leaf_tgt;     // leaves holding targets
  const int4 *leaf_work;  int n_leaf_work;       // leaf-kernel blocks: (leaf, tbeg, tend, lanes per target)
  const int *leaf_src_list;  int n_leaf_src;     // leaves holding sources
  const int *lev_box_src;  const int *lev_box_src_ptr;  // per level: boxes with sources
  const int *lev_box_tgt;  const int *lev_box_tgt_ptr;  // per level: boxes with targets
  // leaves, numbered over all trees of the forest (one tree per surface)
  const int *leaf_box;                           // [leaves] global box id
  const int *leaf_lvl;                           // [leaves] level (= depth of its tree)
  const T *leaf_h;                               // [leaves] side
  int depth, nbox;                               // deepest level of any tree, boxes
  int p, L;                  // expansion order, (p+1)^2
  const T *m2m, *l2l, *m2l;  // transposed [..][in][out]
  const T *dgradT, *dhessT;  // transposed [t][in][out]
  const GemmPlan* m2l_plan;   // host structs with device pointers (nullable):
  const GemmPlan* m2m_plan;   //   M2L over all levels in m2l_parts parts run in turn (the
  const GemmPlan* l2l_plan;   //   first writes, the others add); M2M and L2L indexed by level
  int m2l_parts;
  void* Y;                    // column scratch [max columns of one plan * ne_max][L]
  const T *p2m_H, *p2m_D;     // per-source P2M tables [No][L] in tree order (nullable)
  int leaf_fmax;              // most lanes per target in the leaf kernel (power of two, 1..64)
  // host handles (nullable side): a non-blocking stream for the near-field
  // sums and the events that fork it from and join it to the caller's stream
  hipStream_t side;
  hipEvent_t fork_ev, join_ev;
  // schedule of the overlapped apply: the near-field kernel forked after
  // the strengths (fork_late = 0) or after P2M (1), with at most near_grid
  // blocks (0: one per work item); corr_early: the gradient apply's
  // correction sums run on the side stream before the near field
  int fork_late, near_grid, corr_early;
};

// strengths c[e][tree pos of m] = wo[m] * (P tau_e)[m] for ne densities
template <typename T>
void launch_strengths(const T* tau, int ne, int64_t N, int NP, int n_p, int n_o, const T* P,
                      const T* wo, const int* src_pos, int64_t No, T* str, hipStream_t st);

// Adjoint applies.  Node strengths of the transposed far sum from the
// cotangents (each nullable, density-major, user order):
//   q_i = gpot_i,  d_i = ggrad_i + n_i gdSdn_i + (gsurf_i - n_i (n_i . gsurf_i))
// written as str [nd][4][N] at the tree positions src_pos of the transposed
// tree, and in user order as g4 [nd][N][4] for the transposed corrections.
template <typename T>
void launch_adj_strengths(int nd, int64_t N, const T* gpot, const T* ggrad, const T* gdSdn, const T* gsurf,
                          const T* nrm, const int* src_pos, T* str, T* g4, hipStream_t st);
// sigma_bar [nd][N] = P^T (w^over psi / (4 pi)) per patch + C4^T g4, with psi
// [nd][No] at the target positions tgt_pos of the transposed tree, and the
// transposed block-CSR (per patch: entries (row, block), cptr [NP+1]).
template <typename T>
void launch_adj_combine(int nd, int NP, int n_p, int n_o, int64_t N, int64_t No, const T* P, const T* wo,
                        const T* psi, const int* tgt_pos, const int64_t* cptr, const int* crow,
                        const int64_t* cblk, const T* vals4, const T* g4, T* sigma_bar, hipStream_t st);

// Kernel-position derivative of S (node positions X; the far-rule points
// s = P X move with them; weights, oversampled density and corrections fixed):
//   X_bar_j += sum_d [gbar_dj grad phi_d(x_j) + sum_{m in patch(j)} P_mk c_dm grad psi_d(s_m)] / (4 pi)
// with grad phi [nd][4][N] (FMM_GRAD output of the forward tree, strengths
// c = str [nd][No]) and grad psi [nd][4][No] (FMM_GRAD output of the
// transposed tree for charges gbar at the nodes).
// scatter: out[d][pos[i]] = in[d][i], d < nd, i < n.
template <typename T>
void launch_scatter_perm(int nd, int64_t n, const T* in, const int* pos, T* out, hipStream_t st);
template <typename T>
void launch_xbar_S(int nd, int NP, int n_p, int n_o, int64_t N, int64_t No, const T* P, const T* str,
                   const int* src_pos, const T* gphi, const int* tgt_pos, const T* gbar, const T* gpsi,
                   const int* atgt_pos, T* xbar, hipStream_t st);

// Transposed A3 (adjoint of lb_apply_A3), on the transposed tree:
//   step 1 strengths from v [nd][N]: (v, 2 H v) -> str [nd][2][N] at src_pos
//     and g2 [nd][N][2] (user order)
//   step 1 combine: a = S'^T v, b = (S''+D')^T v + S'^T (2 H v) from psi
//     [nd][2][No] (psi_a, psi_b) and the transposed corrections (vals3)
//   step 2 strengths: charge -b, dipole a n -> str [nd][4][N] (FMM_ADJ),
//     g2 = (a, b)
//   step 2 combine: out = -v/4 + (far) + C_S'^T a - C_S^T b + cs z,
//     cs = sum over the node's surface of v / its area (scal [nd][nsurf],
//     node_surf [N]), z = S^T S^T w
template <typename T>
void launch_adj3_str1(int nd, int64_t N, const T* v, const T* H, const int* src_pos, T* str, T* g2,
                      hipStream_t st);
template <typename T>
void launch_adj3_str2(int nd, int64_t N, const T* a, const T* b, const T* nrm, const int* src_pos, T* str, T* g2,
                      hipStream_t st);
template <typename T>
void launch_adj3_comb1(int nd, int NP, int n_p, int n_o, int64_t N, int64_t No, const T* P, const T* wo,
                       const T* psi, const int* tgt_pos, const int64_t* cptr, const int* crow, const int64_t* cblk,
                       const T* vals3, const T* g2, T* a, T* b, hipStream_t st);
template <typename T>
void launch_adj3_comb2(int nd, int NP, int n_p, int n_o, int64_t N, int64_t No, const T* P, const T* wo,
                       const T* psi, const int* tgt_pos, const int64_t* cptr, const int* crow, const int64_t* cblk,
                       const T* vals3, const T* g2, const T* v, const T* z, const double* scal, int nsurf,
                       const int* node_surf, T* out, hipStream_t st);
// Several GMRES systems at once (FP64): system a owns the segment
// [xoff[a], xoff[a] + len[a]) of the operator's vectors and the basis
// vectors V + vbase[a] + j len[a].  gather: win = V_j(a) (0 where active[a]
// is 0); dots: out[a k + jj] = V_jj(a) . W(a) (vbase null: W(a) . W(a), k = 1;
// partial: [nsys k 32]); gemv: W(a) += sign sum_jj h[a k + jj] V_jj(a);
// scale_copy: V_j(a) = sc[a] W(a).  maxlen = max len (grid size).
void launch_msys_gather(int nsys, int64_t maxlen, const int64_t* xoff, const int64_t* len, const int64_t* vbase,
                        const int* active, int j, const double* V, double* win, hipStream_t st);
void launch_msys_dots(int nsys, int k, const int64_t* xoff, const int64_t* len, const int64_t* vbase,
                      const double* V, const double* W, double* partial, double* out, hipStream_t st);
void launch_msys_gemv(int nsys, int64_t maxlen, int k, const int64_t* xoff, const int64_t* len, const int64_t* vbase,
                      const double* V, const double* h, double sign, double* W, hipStream_t st);
void launch_msys_scale_copy(int nsys, int64_t maxlen, int j, const int64_t* xoff, const int64_t* len,
                            const int64_t* vbase, const double* sc, const double* W, double* V, hipStream_t st);
// GMRES (Section 6) driven on the device for ns independent systems (FP64):
// system a owns the segment [xoff[a], xoff[a] + len[a]) of the operator's
// vectors and the basis vectors V + vbase[a] + j len[a], j = 0..maxit.  The
// iteration number lives in *iter, so the launches of one iteration are the
// same for every j (one captured graph replays them all).  R [ns][maxit]
// [maxit] holds the rotated Hessenberg matrix (R[r][c]), cs, sn [ns][maxit]
// the rotations, g [ns][km] the rotated right-hand side (km = maxit + 1),
// h1, h2 [ns][km] the two Gram-Schmidt passes' coefficients (h1 later y),
// nr [ns] squared norms, part [ns][km][32] partial sums.
struct GmresDev {
  const int64_t *xoff = nullptr, *len = nullptr, *vbase = nullptr;
  int *active = nullptr, *kdone = nullptr, *iter = nullptr, *nactive = nullptr;
  double *R = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *beta = nullptr, *relres = nullptr;
  double *sc = nullptr, *h1 = nullptr, *h2 = nullptr, *nr = nullptr, *part = nullptr;
  const double* tol = nullptr;  // [1] relative residual target
  int ns = 0, maxit = 0, km = 0;
  int64_t maxlen = 1;           // largest segment (grid size)
};
// norms of b, beta, g_0, the active flags (skip[a] = 1: not solved), the
// first basis vectors V_0 = b / beta, iter = 0, nactive
void launch_gm_start(const GmresDev& gm, const double* B, const int* skip, double* V, hipStream_t st);
// win = V_j of the active systems (0 elsewhere)
void launch_gm_gather(const GmresDev& gm, const double* V, double* win, hipStream_t st);
// after the operator has written W = A V_j: CGS2 against V_0..V_j, the
// Givens step, V_{j+1} = W / |W|, iter = j + 1, nactive
void launch_gm_arnoldi(const GmresDev& gm, double* V, double* W, hipStream_t st);
// x(a) = V y(a) with R y = g over the iterations each system ran
void launch_gm_finish(const GmresDev& gm, const double* V, double* X, hipStream_t st);

// Per-surface reductions (surface q owns rows [off[q], off[q+1])):
// seg_dot: out[d][q] = scale[q] sum_{i in q} x[d][i] (w ? w[i] : 1);
// seg_axpy: y[d][i] = x[d][i] + alpha (w ? w[i] : 1) c[d][surf[i]].
template <typename T>
void launch_seg_dot(int nd, int nsurf, int64_t N, const int64_t* off, const T* x, const double* w,
                    const double* scale, double* out, hipStream_t st);
template <typename T>
void launch_seg_axpy(int nd, int nsurf, int64_t N, const int* surf, const T* x, double alpha, const double* w,
                     const double* c, T* y, hipStream_t st);

// P2M tables of every source about its leaf centre (setup): H, Dp [No][L]
// in tree order; see k_p2m_build
template <typename T>
void launch_p2m_tables(const DevTree<T>& t, T* H, T* Dp, hipStream_t st);
// A2 (Section 4.2).  Strengths of the first pass from c = w^over P tau
// [nd][No] (tree order): s3 [nd][2][No] for FMM_A3B (charges 0 and c) and sd
// [nd][4][No] for FMM_ADJ (dipole vector c nu, nu the tree's source normals)
template <typename T>
void launch_a2_str1(int nd, int64_t No, const T* c, const T* nx, const T* ny, const T* nz, T* s3, T* sd,
                    hipStream_t st);
// second pass: sd [nd][4][No] = (c2, c1 nu) from c1, c2 [nd][No]
template <typename T>
void launch_a2_str2(int nd, int64_t No, const T* c1, const T* c2, const T* nx, const T* ny, const T* nz, T* sd,
                    hipStream_t st);
// mu1 = D tau, mu2 = -(S''+D') tau - 2 H S' tau and y = S tau [nd][N] from the
// FMM_A3B output f3 [nd][4][N], the FMM_ADJ output fd [nd][N] and the
// corrections vals3 (S, S', S''+D'), valsD (D)
template <typename T>
void launch_combine_a2a(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch, const T* vals3,
                        const T* valsD, const T* tau, const T* f3, const T* fd, const int* tgt_pos, const T* H,
                        T* mu1, T* mu2, T* y, hipStream_t st);
// out = -tau/4 + S mu2 + D mu1 from the FMM_ADJ output fb [nd][N] (charge
// mu2, dipole vector mu1 nu) and the corrections
template <typename T>
void launch_combine_a2b(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch, const T* vals3,
                        const T* valsD, const T* tau, const T* mu1, const T* mu2, const T* fb, const int* tgt_pos,
                        T* out, hipStream_t st);

// values per (leaf work item, density) of the workspace D that the leaf
// kernels of `mode` use at expansion order p (0: none)
template <typename T>
int64_t leaf_d_stride(int mode, int p);

// full FMM (or direct sums when depth < 2): str [nrhs*nstr][No] -> out [nrhs*nout][N]
// Optional phase timer: events recorded on the launch stream at the phase
// boundaries of one apply (strengths | P2M | M2M | M2L | L2L | leaf | combine).
enum Phase { PH_STR = 0, PH_P2M, PH_M2M, PH_M2L, PH_L2L, PH_LEAF, PH_COMB, PH_N };
struct PhaseTimer {
  hipEvent_t ev[PH_N + 1];
  bool on = false;
  void mark(int i, hipStream_t st) { if (on) (void)hipEventRecord(ev[i], st); }
};

// nrhs * fmm_nexp(mode) <= the plans' ne_max.  D: scratch [n_leaf_work][nrhs][leaf_d_stride(mode, p)]
template <typename T>
void launch_fmm(const DevTree<T>& t, int mode, int nrhs, const T* str, T* M, T* Lc, T* D, T* out,
                int64_t N, int64_t No, hipStream_t st, PhaseTimer* tm = nullptr);

// corrections + combine (user order)
// gradS: sigma [nd][N] -> pot/grad/dSdn/surf (each nullable except grad)
template <typename T>
void launch_combine_grad(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch,
                         const T* vals4, const T* sigma, const T* fmm, const int* tgt_pos,
                         const T* nrm, T* pot, T* grad, T* dSdn, T* surf, hipStream_t st);
// the same in two steps: the corrections alone (corr [nd][N][4], no FMM
// output needed, so they can run beside the FMM), then the final sums
template <typename T>
void launch_corr_grad(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch, const T* vals4,
                      const T* sigma, T* corr, hipStream_t st);
template <typename T>
void launch_combine_grad_fin(int nd, int64_t N, const T* fmm, const T* corr, const int* tgt_pos, const T* nrm,
                             T* pot, T* grad, T* dSdn, T* surf, hipStream_t st);
// S only: pot = S sigma from the FMM_POT output and the S corrections
template <typename T>
void launch_combine_pot(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch, const T* vals3,
                        const T* sigma, const T* fmm, const int* tgt_pos, T* pot, hipStream_t st);
// A3 step 1: tau -> mu1 = S' tau, mu2 = S tau  (density d of mu1/mu2 at offset d*ldmu)
template <typename T>
void launch_combine_a3a(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch,
                        const T* vals3, const T* tau, const T* fmm, const int* tgt_pos,
                        const T* nrm, T* mu1, T* mu2, int64_t ldmu, hipStream_t st);
// A3 step 2: out = -tau/4 + S'mu1 - (S''+D')mu2 - 2H S'mu2 + W S mu2, the
// last term per surface (surface q: rows [node_off[q], node_off[q+1]),
// inv_area[q]; node_surf [N]); y2buf [nd][N] and scal [nd][nsurf] scratch
template <typename T>
void launch_combine_a3b(int nd, int64_t N, int n_p, const int64_t* row_ptr, const int* patch,
                        const T* vals3, const T* tau, const T* mu1, const T* mu2, int64_t ldmu, const T* fmm,
                        const int* tgt_pos, const T* H, const double* w, int nsurf, const int64_t* node_off,
                        const int* node_surf, const double* inv_area, T* out, T* y2buf, double* scal,
                        hipStream_t st);

// FP64 helpers for GMRES
void launch_dots(const double* V, int64_t ldv, int k, const double* w, int64_t N, double* out,
                 double* partial, hipStream_t st);                 // out[j] = V_j . w, j < k
void launch_gemv_sub(const double* V, int64_t ldv, int k, const double* h, double* w, int64_t N,
                     hipStream_t st);                              // w -= V h
void launch_gemv_add(const double* V, int64_t ldv, int k, const double* y, double* x, int64_t N,
                     hipStream_t st);                              // x += V y
void launch_scale_copy(const double* w, double a, double* v, int64_t N, hipStream_t st);  // v = a w
void launch_axpby(double a, const double* x, double b, const double* y, double* z, int64_t N,
                  hipStream_t st);                                 // z = a x + b y
template <typename A, typename B>
void launch_convert(const A* x, B* y, int64_t n, hipStream_t st);
void launch_wmean(const double* f, const double* w, int64_t N, double* partial, double* out,
                  hipStream_t st);                                 // out = sum w f
void launch_sub_scalar(double* f, const double* s, double scale, int64_t N, hipStream_t st);  // f -= scale*s[0]

// Accurate integrals A of the corrections for (target, near patch) pairs
// with the patch not the target's own (Section 4, eq. nys-lcq2), by the
// adaptive subdivision rule: work item w is target row[w] against patch
// patch[w], written to block blk[w] of A: A[blk][b][t] (n_p values b,
// kernels t = S, Gx, Gy, Gz, S', S''+D').
struct NearQuadArgs {
  const double* X = nullptr;    // [N][3] targets
  const double* nrm = nullptr;  // [N][3] target normals
  const double* cX = nullptr;   // [NP][n_p][3] modal coefficients of X, X_u, X_v
  const double* cXu = nullptr;
  const double* cXv = nullptr;
  const double* ja = nullptr;   // [(k+1)^2] Jacobi recurrence of the modal basis
  const double* jb = nullptr;
  const double* jc = nullptr;
  const double* Vinv = nullptr; // [n_p][n_p]
  const double* ru = nullptr;   // [nq][2] leaf rule on the unit triangle
  const double* rw = nullptr;   // [nq]
  const int64_t* row = nullptr; // [nwork]
  const int64_t* blk = nullptr; // [nwork]
  const int32_t* patch = nullptr;
  double* A = nullptr;          // [nnz_blocks][n_p][6]
  int64_t nwork = 0;
  int k = 0, nq = 0, max_depth = 0;
  double adm = 2.0;
};
hipError_t launch_near_quad(const NearQuadArgs& q, hipStream_t st);

// Accurate integrals A of the self blocks (Section 4: Duffy triangles at the
// node, sinh-graded edge variable, principal value of the gradient kernels):
// target i writes block sblk[i] of A (no block when sblk[i] < 0).
struct SelfQuadArgs {
  const double* X = nullptr;    // [N][3]
  const double* nrm = nullptr;  // [N][3]
  const double* dXu = nullptr;  // [N][3] derivatives of the interpolated chart at the nodes
  const double* dXv = nullptr;
  const double* J = nullptr;    // [N]
  const double* cX = nullptr;   // [NP][n_p][3]
  const double* cXu = nullptr;
  const double* cXv = nullptr;
  const double* ja = nullptr;   // [(k+1)^2]
  const double* jb = nullptr;
  const double* jc = nullptr;
  const double* Vinv = nullptr; // [n_p][n_p]
  const double* uv = nullptr;   // [n_p][2] reference nodes
  const double* g = nullptr;    // [ns] Gauss-Legendre rule on [0, 1] along the rays
  const double* gw = nullptr;
  const double* tg = nullptr;   // [nt] the same per panel of the edge variable
  const double* tw = nullptr;
  const int64_t* sblk = nullptr;  // [N]
  double* A = nullptr;          // [nnz_blocks][n_p][6]
  // the displacement x_i - X(u0 + s e) as -s sum_j mw_j X'(u0 + mg_j s e) e:
  // modal coefficients of the derivatives of the interpolated X
  // [NP][n_p][3] and an nm-point Gauss rule on [0, 1] (nm = ceil(k / 2))
  const double* cDu = nullptr;
  const double* cDv = nullptr;
  const double* mg = nullptr;
  const double* mw = nullptr;
  int nm = 0;
  int64_t N = 0;
  int k = 0, ns = 0, nt = 0;
  double panel = 2.0;
};
hipError_t launch_self_quad(const SelfQuadArgs& q, hipStream_t st);

// C = A - B of every block (eq. nys-lcq) in the packed layouts of the
// combine kernels, for FP64 (B over every oversampled point of the patch)
// and FP32 (B without the points that the float32 near-field kernel skips:
// float r^2 below rm2 of the point).  Either pair of outputs may be null
// (the FP32 values then need no rm2), so that the two precisions can use
// far rules of their own (two launches).
struct FarRuleArgs {
  const double* X = nullptr;    // [N][3]
  const double* nrm = nullptr;  // [N][3]
  const double* s = nullptr;    // [No][3] oversampled points
  const double* nu = nullptr;   // [No][3]
  const double* wo = nullptr;   // [No]
  const float* rm2 = nullptr;   // [No]
  const double* P = nullptr;    // [n_o][n_p]
  const int64_t* brow = nullptr;  // [nb] target of each block
  const int32_t* patch = nullptr; // [nb]
  const double* A = nullptr;    // [nb][n_p][NKER]
  double* v4_64 = nullptr;      // [nb * n_p][4]: S, Gx, Gy, Gz
  double* v3_64 = nullptr;      // [nb * n_p][3]: S, S', S''+D'
  double* vD_64 = nullptr;      // [nb * n_p]: D
  float* v4_32 = nullptr;
  float* v3_32 = nullptr;
  float* vD_32 = nullptr;
  int64_t nb = 0;
  int n_p = 0, n_o = 0;
};
hipError_t launch_far_rule(const FarRuleArgs& q, hipStream_t st);

// Surface calculus of node values (Section 2): the order-k interpolant on
// each patch differentiated in the chart (Du, Dv [n_p][n_p] nodal
// differentiation, Xu, Xv [N][3] the chart derivatives given at the nodes).
struct SurfCalcArgs {
  const double* Du = nullptr;
  const double* Dv = nullptr;
  const double* Xu = nullptr;
  const double* Xv = nullptr;
  const double* nrm = nullptr;  // [N][3]
  int64_t N = 0;
  int n_p = 0;
};
// grad [nd][N][3] = surface gradient of psi [nd][N]
hipError_t launch_surf_grad(const SurfCalcArgs& q, int nd, const double* psi, double* grad, hipStream_t st);
// div [nd][N] = sign * surface divergence of the tangential part of V (or of
// n x V when cross_n), V [nd][N][3]
hipError_t launch_surf_div(const SurfCalcArgs& q, int nd, const double* V, int cross_n, double sign, double* div,
                           hipStream_t st);
// H [nf][N][3] = F - grad alpha - n x grad beta (alpha, beta [nf][N])
hipError_t launch_hodge_h(const SurfCalcArgs& q, int nf, const double* F, const double* alpha, const double* beta,
                          double* H, hipStream_t st);

// A1 (Section 4.1): mu [3 nd][N] from grad_Gamma S tau [nd][N][3], and
// out [nd][N] = sum_l (d_l S)[mu_l] + eta[d][surface] S[1] from the gradient
// apply of mu (g [3 nd][N][3]), eta [nd][nsurf] and phi0 = S[1] [N]
template <typename T>
hipError_t launch_a1_split(int64_t N, int nd, const T* surf, T* mu, hipStream_t st);
template <typename T>
hipError_t launch_a1_finish(int64_t N, int nd, int nsurf, const int* surf_of, const T* g, const double* eta,
                            const T* phi0, T* out, hipStream_t st);

}  // namespace lb
