/*
 * lb.h -- C ABI of the MI355X Laplace-Beltrami layer-potential library.
 *
 * The library applies the Laplace single layer S and its gradient on the
 * Nystrom nodes of high-order curved triangular patches, with a fast
 * multipole method for the far field and stored locally corrected quadrature
 * for the near field, and solves the Laplace-Beltrami problem with the
 * second-kind formulation A3 = -I/4 + S'^2 - (S''+D'+2HS')S + WS^2
 * (Agarwal, O'Neil, Rachh, arXiv 2111.10743: Section 3 for the operators and
 * Lemma 1 for the mean-zero setting, Section 4 for the discretization and
 * eq. (nys-lcq2), Section 4.3 for the A3 apply, Section 6 for GMRES).  It
 * also applies the non-second-kind A1 (Section 4.1) and computes Hodge
 * decompositions of tangential fields (the harmonic-vector-field section).
 *
 * Conventions shared by every entry point:
 *  - Every function returns an lb_status.  0 is success, negative values are
 *    errors (nothing useful was written), LB_ENOCONV (> 0) is a warning.
 *    lb_last_error() returns a thread-local message for the last failure.
 *  - Patches: n_patches charts X: T0 -> Gamma, T0 = {u,v >= 0, u+v <= 1},
 *    sampled at the n_p = (k+1)(k+2)/2 nodes of lb_ref_nodes(k).  Node data
 *    is patch-major: index i = patch * n_p + local node.  N = n_patches * n_p.
 *  - Buffers passed to lb_setup and lb_ref_nodes are HOST pointers; they are
 *    copied, the context keeps no caller pointer.
 *  - Density and output buffers of the apply/solve calls are DEVICE pointers
 *    owned by the caller, contiguous, in the dtype selected by `prec`
 *    (32: float, 64: double).  Densities are [nd][N] (density-major).
 *  - All device work is enqueued on `stream` (a hipStream_t, NULL = the
 *    default stream) and is stream ordered; calls return without waiting
 *    unless stated.  Use one context from one stream at a time.
 *  - The caller's current HIP device must be the one the context was
 *    created on.
 */
#ifndef LB_H
#define LB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int lb_status;
#define LB_OK            0
#define LB_ENOCONV       1   /* warning: GMRES stopped at max_iter; best iterate written */
#define LB_EINVAL       -1   /* bad argument (order, sizes, NaN/Inf input, null pointer) */
#define LB_ENOMEM       -2   /* host or device allocation failed */
#define LB_EHIP         -3   /* a HIP runtime call failed */
#define LB_ENOTMEANZERO -4   /* strict-mean mode and f is not mean zero */
#define LB_EGEOM        -5   /* degenerate patch (zero Jacobian) */

/* precisions of the apply calls */
#define LB_PREC_FP32 32
#define LB_PREC_FP64 64

/* lb_solve modes */
#define LB_SOLVE_FP64        0   /* FP64 FMM, FP64 corrections, FP64 GMRES */
#define LB_SOLVE_FP32_REFINE 1   /* FP32 inner GMRES operator, FP64 residual refinement */
#define LB_SOLVE_A2          4   /* or-ed into either mode: the A2 formulation (eq. ie-dis1) */

/* lb_opts.flags */
#define LB_STRICT_MEAN 1   /* lb_solve rejects f with |mean| > 1e-12 ||f|| */
#define LB_HOST_ONLY   2   /* lb_setup does the host work only (no HIP call) */
#define LB_DIRECT      4   /* far field by all-pairs sums instead of the FMM */
#define LB_HOST_OCTREE 16  /* build the FMM octrees on the host instead of the device (same tree) */
#define LB_NO_GRAPH    32  /* GMRES applies its operator by plain launches instead of replaying
                              a captured HIP graph of one application */
#define LB_NO_OVERLAP  64  /* run the near-field sums after the far-field passes on the caller's
                              stream instead of concurrently on a second (non-blocking) stream */
#define LB_HOST_QUAD   128 /* lb_setup computes the quadrature corrections on the host (OpenMP)
                              instead of on the device */
#define LB_NO_P2M_TABLES 8 /* compute the leaf harmonics of P2M on the fly instead of keeping
                              per-source tables (2 (p+1)^2 values per oversampled point and
                              precision, kept when they fit in a quarter of free device memory
                              and under 64 GiB) */

typedef struct lb_ctx lb_ctx;   /* opaque: owns host and device state */

typedef struct {
  double eta_near;  /* Near(x_i) = { l : |x_i - c_l| < eta_near * R_l }      (default 2)  */
  int over_q;       /* oversampled far rule of the FP64 path: q x q conical Gauss points
                       (default k+6)                                                   */
  int p_f32;        /* FMM expansion order of the FP32 path                   (default 14) */
  int p_f64;        /* FMM expansion order of the FP64 path                   (default 28) */
  int leaf_src;     /* target mean number of sources per FMM leaf box of the FP64 tree
                       (default 1024); the FP32 tree starts from leaf_src n_o32 / n_o,
                       the same boxes for its coarser far rule                        */
  int max_iter;     /* GMRES iteration cap per (inner) solve                  (default 100)*/
  int flags;        /* LB_STRICT_MEAN | LB_HOST_ONLY | LB_DIRECT | LB_NO_P2M_TABLES |
                       LB_HOST_OCTREE | LB_NO_GRAPH | LB_NO_OVERLAP | LB_HOST_QUAD     */
  int self_n;       /* self-patch rule: Gauss points along each Duffy ray    (default 16) */
  int near_q;       /* adaptive near rule: near_q x near_q points per leaf    (default 8)  */
  double near_adm;  /* adaptive near rule admissibility dist >= adm * diam    (default 2)  */
  double m2l_trunc32; /* M2L order by offset, FP32 tree: an offset at centre distance d
                         (box widths) translates the first (p_d+1)^2 coefficients,
                         p_d = min(p, ceil(s p ln rho(2) / ln rho(d))), rho(d) = a/(d-a),
                         a = sqrt(3)/2, s this factor; 0: order p for every offset
                         (default 2.5) */
  double m2l_trunc64; /* the same for the FP64 tree (default 2.0) */
  int over_q32;     /* far rule of the FP32 path: q x q conical Gauss points (default
                       max(k+2, 6): it changes the operator by 7.5e-9 (k = 6) .. 1.4e-7
                       (k = 4) against the k+6 rule, at or below FP32 rounding) */
} lb_opts;

typedef struct {
  int iters;            /* total GMRES iterations (inner, summed over refinement steps) */
  int outer_steps;      /* FP64 residual evaluations after the first (0 in LB_SOLVE_FP64) */
  double rel_resid;     /* ||f - A3 sigma||_2 / ||f||_2 of the returned sigma, FP64 operator */
  double removed_mean;  /* weighted mean sum w f / sum w that was removed from f */
  double t_setup;       /* wall-clock seconds the context's setup took (lb_setup, lb_setup_batch
                           or lb_import_setup): the paper's quadrature time t_q plus the tree
                           and translation setup */
  double t_solve;       /* wall-clock seconds of this lb_solve / lb_solve_adj call, from entry
                           to the synchronized result (the paper's t_s without t_q) */
} lb_solve_info;

typedef struct {
  int64_t n_patches, n_p, N;      /* patches, nodes per patch, nodes            */
  int64_t n_o, N_o;               /* oversampled points per patch, in total     */
  int64_t nnz_blocks;             /* (target, near patch) pairs of the corrections */
  int64_t fmm_levels, fmm_leaves; /* octree depth and number of nonempty leaves */
  int64_t p_f32, p_f64;           /* expansion orders in use                     */
  int64_t p2p_pairs32, m2l_pairs32; /* near-field (target, source) pairs and V-list
                                       (target box, source box) pairs, FP32 tree */
  int64_t p2p_pairs64, m2l_pairs64; /* the same for the FP64 tree               */
  int64_t n_surf;                   /* surfaces of the context (lb_setup_batch)  */
  int64_t m2l_flops32, m2l_flops64; /* algorithmic M2L flops per density: 2 L_o^2 per
                                       V-list pair, L_o the active size of its offset */
  int64_t n_o32, N_o32;             /* oversampled points per patch, in total, of the
                                       FP32 far rule (n_o, N_o: the FP64 one)      */
} lb_sizes;

/* Fill *opts with the defaults listed above. */
lb_status lb_default_opts(lb_opts *opts);

/* Reference nodes of order k (1 <= k <= 7) on T0, where callers sample their
 * charts (Section 4: the order-k interpolation nodes; this library's node
 * family is the Blyth-Pozrikidis construction on Gauss-Legendre points).
 * uv: host [n_p][2] (u, v); w_ref: host [n_p] interpolatory weights, nullable. */
lb_status lb_ref_nodes(int order, double *uv, double *w_ref);

/* Build geometry, near lists, quadrature corrections (Section 4, eqs. nys-lcq
 * and nys-lcq2), the octree and the translation operators, and upload them.
 * X, Xu, Xv: host [n_patches][n_p][3] chart samples and first derivatives at
 * lb_ref_nodes(order).  opts: nullable (defaults).  The corrections are
 * computed on the current device (one wavefront per target for the self
 * blocks, per (target, patch) pair for the others and the far rule), on the
 * host with LB_HOST_QUAD or LB_HOST_ONLY: the same rules, equal up to
 * rounding order.  On success *ctx owns all
 * state; release it with lb_destroy.  Errors: LB_EINVAL (order out of range,
 * NaN/Inf input), LB_EGEOM (zero Jacobian), LB_ENOMEM, LB_EHIP. */
lb_status lb_setup(lb_ctx **ctx, int n_patches, int order, const double *X,
                   const double *Xu, const double *Xv, const lb_opts *opts,
                   void *stream);

/* Several independent surfaces in one context (for instance many small
 * surfaces whose applies and solves are batched): surface q has
 * patches_per_surf[q] patches, and X, Xu, Xv hold the patches of all surfaces
 * one surface after the other.  Every apply, the A3 operator and the solves
 * act on all surfaces at once (vectors [nd][N] with N the total number of
 * nodes, surfaces in order), but the surfaces never interact: each has its
 * own near lists, corrections, octree (one launch per FMM phase covers all
 * trees), mean projection and W term of A3, and each (right-hand side,
 * surface) pair is its own GMRES system with its own tolerance; info of
 * lb_solve / lb_solve_adj then has nrhs * n_surf entries (index
 * rhs * n_surf + surface).  Errors as lb_setup. */
lb_status lb_setup_batch(lb_ctx **ctx, int n_surf, const int32_t *patches_per_surf, int order,
                         const double *X, const double *Xu, const double *Xv,
                         const lb_opts *opts, void *stream);

/* Save a context's setup to the file `path` (the paper generates the
 * quadrature corrections once per geometry and reuses them: across the
 * iterations of a solve and across the two solves of a Hodge decomposition,
 * harmonic-vector-field section and Section 6): the chart samples, options,
 * near lists, the corrections of both precisions (eq. nys-lcq2) and the
 * tuning of each precision (lb_autotune / lb_set_tuning), with a checksum.
 * Host side (synchronizes the device); the file is in the native byte order.
 * Errors: LB_EINVAL (null argument, LB_HOST_ONLY context, file not
 * writable), LB_EHIP. */
lb_status lb_export_setup(const lb_ctx *ctx, const char *path);

/* Create a context from a file written by lb_export_setup, on the current
 * device, without generating the corrections: the geometry and near lists
 * are rebuilt from the saved charts and checked against the saved lists,
 * the saved corrections are uploaded, the octrees and translation operators
 * rebuilt with the saved tuning.  Applies and solves of the new context
 * equal those of the saved one bit for bit.  lb_solve_info.t_setup reports
 * the import time.  Errors: LB_EINVAL (missing, truncated, corrupt or
 * incompatible file: magic, version, byte order, option layout, checksum,
 * near lists), LB_ENOMEM, LB_EHIP. */
lb_status lb_import_setup(lb_ctx **ctx, const char *path, void *stream);

/* Sizes of the discretization held by ctx. */
lb_status lb_get_sizes(const lb_ctx *ctx, lb_sizes *out);

/* Host copies of the smooth weights w [N], unit normals [N][3] and mean
 * curvature H [N] (Section 2; H = +1 on the unit sphere).  Nullable outputs. */
lb_status lb_get_geometry(const lb_ctx *ctx, double *w, double *normals, double *H);

/* Host copy of the FP64 near corrections C = A - B (eq. nys-lcq2) in block
 * CSR form: row_ptr [N+1] (int64), patch [nnz_blocks] (int32) and
 * vals [nnz_blocks][n_p][7] for the kernels S, dS/dx1, dS/dx2, dS/dx3, S',
 * S''+D' and the double layer D = grad_y G . nu (Section 3), all including
 * the 1/(4 pi) of the Green's function.  Works on a LB_HOST_ONLY context.
 * Any output may be NULL. */
lb_status lb_get_corrections(const lb_ctx *ctx, int64_t *row_ptr, int32_t *patch,
                             double *vals);

/* The FMM octree of surface `surf` in one precision (transposed = 1: the
 * tree of the adjoint applies, after the first one).  Uniform depth; boxes numbered level by
 * level in Morton order (global id g); leaves = the boxes of level depth,
 * numbered from 0.  Outputs (host, nullable; sizes from *info, so a first
 * call may pass only info):
 *   tgt_perm [targets], src_perm [sources]: tree position -> input index
 *     (forward tree: targets = the N nodes, sources = the N_o oversampled
 *     points; transposed tree: the other way round), stable in the input
 *     order within a leaf;
 *   leaf_ranges [nleaf][4]: target begin/end, source begin/end positions;
 *   ulist_ptr [nleaf+1], ulist [nulist]: adjacent leaves holding sources of
 *     each leaf holding targets (leaf numbers);
 *   vlist_ptr [nbox+1], vlist_src [nvlist], vlist_off [nvlist]: for each box
 *     holding targets on levels >= 2, the children of its parent's neighbours
 *     that hold sources and are not adjacent (global ids), with the offset id
 *     ((ox+3)*7 + (oy+3))*7 + (oz+3) of target minus source in box units;
 *   boxes [nbox][5]: level, integer coordinates x, y, z on the level, and
 *     flags (1: holds targets, 2: holds sources).
 * The root cube is [lo, lo + side]^3. */
typedef struct {
  int32_t depth, nbox, nleaf, nulist, nvlist;
  double lo[3], side;
} lb_tree_info;
lb_status lb_get_tree(const lb_ctx *ctx, int prec, int transposed, int surf, lb_tree_info *info,
                      int64_t *tgt_perm, int64_t *src_perm, int32_t *leaf_ranges,
                      int32_t *ulist_ptr, int32_t *ulist, int32_t *vlist_ptr,
                      int32_t *vlist_src, int32_t *vlist_off, int32_t *boxes);

/* The same octree for arbitrary point sets (the FMM of Section 4 runs on
 * such a tree): tgt [nt][3], src [ns][3] host doubles; depth >= 0 fixes the
 * leaf level, depth < 0 picks the first level >= 2 whose mean number of
 * sources per non-empty leaf is <= leaf_src, coarsened while the leaf side is
 * <= min_leaf_side.  on_device = 1 builds with the HIP kernels on the current
 * device (synchronous), 0 on the host; both give the same tree.  Read it with
 * lb_tree_get (outputs as lb_get_tree), release it with lb_tree_destroy.
 * Errors: LB_EINVAL (empty or non-finite input, depth > 20), LB_EHIP. */
typedef struct lb_tree lb_tree;
lb_status lb_tree_build(lb_tree **tree, const double *tgt, int64_t nt, const double *src,
                        int64_t ns, int leaf_src, double min_leaf_side, int depth,
                        int on_device);
lb_status lb_tree_get(const lb_tree *tree, lb_tree_info *info, int64_t *tgt_perm,
                      int64_t *src_perm, int32_t *leaf_ranges, int32_t *ulist_ptr,
                      int32_t *ulist, int32_t *vlist_ptr, int32_t *vlist_src,
                      int32_t *vlist_off, int32_t *boxes);
void lb_tree_destroy(lb_tree *tree);

/* S[sigma] at the N nodes (Section 4.1 first sum, eq. nys-lcq2).
 * sigma: device [nd][N], pot: device [nd][N], dtype by prec. */
lb_status lb_apply_S(lb_ctx *ctx, int nd, int prec, const void *sigma, void *pot,
                     void *stream);

/* S[sigma] and its on-surface gradient (Section 4.1): grad = principal-value
 * gradient (the average of the two one-sided limits), dSdn = S' = n . grad,
 * surf_grad = grad - n (n . grad) = the tangential gradient of S on Gamma.
 * sigma: device [nd][N]; pot [nd][N], grad [nd][N][3], dSdn [nd][N],
 * surf_grad [nd][N][3]; every output except grad is nullable. */
lb_status lb_apply_gradS(lb_ctx *ctx, int nd, int prec, const void *sigma,
                         void *pot, void *grad, void *dSdn, void *surf_grad,
                         void *stream);

/* lb_apply_gradS for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results as lb_apply_gradS (bit for bit), but
 * the per-call workspace (strengths, multipole and local expansions, the
 * leaf kernel's derived expansions, FMM outputs, early correction sums) lives
 * in a static device array of 128 MiB that each device holds from library
 * load until the process ends; the call makes no hipMalloc or hipFree.  Every
 * call on a device shares that device's array, so calls that overlap in time
 * on one device (two streams, two contexts, two threads) race and must be
 * serialized by the caller; nothing in it needs to start at zero.  Limit:
 * the workspace of min(nd, 8) densities must fit in the 128 MiB (the FP32
 * apply of one density on a 5120-patch order-6 surface does); larger
 * requests return LB_ENOMEM without launching anything.  The context must
 * come from lb_setup / lb_setup_batch on the current device (which looked
 * up the array's device address). */
lb_status lb_apply_gradS_noalloc(lb_ctx *ctx, int nd, int prec, const void *sigma,
                                 void *pot, void *grad, void *dSdn, void *surf_grad,
                                 void *stream);

/* Adjoint of lb_apply_gradS with respect to the density: the exact transpose
 * of the discrete operators of the same precision (far sum over the
 * oversampled rule of Section 4 with its near mask, block corrections of
 * eq. nys-lcq2, oversampling tau~ = P tau):
 *   sigma_bar = S^T gpot + (grad S)^T ggrad + S'^T gdSdn + (grad_Gamma S)^T gsurf
 * with S' = n . grad S and grad_Gamma S = grad S - n (n . grad S) as in
 * lb_apply_gradS.  Cotangents: device gpot [nd][N], ggrad [nd][N][3],
 * gdSdn [nd][N], gsurf [nd][N][3], each nullable (not all); sigma_bar:
 * device [nd][N], overwritten.  The far part is an FMM with the N nodes as
 * sources (charge gpot, dipole vector formed from the other cotangents) and
 * the N_o oversampled points as targets.  The first call for a precision
 * builds the transposed octree and correction index on the host and
 * synchronizes the device; later calls are stream ordered on `stream`. */
lb_status lb_apply_gradS_adj(lb_ctx *ctx, int nd, int prec, const void *gpot,
                             const void *ggrad, const void *gdSdn, const void *gsurf,
                             void *sigma_bar, void *stream);

/* Adjoint of lb_apply_S: sigma_bar = S^T gbar (see lb_apply_gradS_adj).
 * gbar, sigma_bar: device [nd][N]. */
lb_status lb_apply_S_adj(lb_ctx *ctx, int nd, int prec, const void *gbar, void *sigma_bar,
                         void *stream);

/* Derivative of lb_apply_S with respect to the node positions X (the
 * gradient kernel): X_bar = d/dX sum_d <gbar_d, S sigma_d>, with the targets
 * x_i = X_i and the oversampled points s = P X of Section 4 moving with the
 * nodes, and the weights w^over, the oversampled density P sigma and the
 * near corrections held at their setup values (the kernel-position
 * derivative; a full shape derivative would also differentiate the
 * corrections).  With c = w^over P sigma:
 *   X_bar_j = sum_d [ gbar_dj grad phi_d(x_j)
 *                     + sum_{m in patch(j)} P_{m,k(j)} c_dm grad psi_d(s_m) ],
 *   phi_d(x) = sum_m c_dm G(x - s_m),  psi_d(y) = sum_i gbar_di G(x_i - y),
 * both sums over every pair but coincident points (no near mask), through
 * two gradient FMMs (forward and transposed trees).  sigma, gbar: device
 * [nd][N]; X_bar: device [N][3], overwritten; dtype by prec.  The first call
 * for a precision builds the transposed octree (as lb_apply_gradS_adj) and
 * synchronizes the device. */
lb_status lb_apply_S_adj_X(lb_ctx *ctx, int nd, int prec, const void *sigma, const void *gbar,
                           void *X_bar, void *stream);

/* lb_apply_gradS with per-phase timing (nd <= 8): HIP events recorded on
 * `stream` around each phase of the apply; synchronizes `stream`.
 * phase_ms: host [7], milliseconds of: density oversampling, P2M, M2M, M2L,
 * L2L, leaf evaluation (L2P + near-field sums), corrections + combination. */
lb_status lb_apply_gradS_timed(lb_ctx *ctx, int nd, int prec, const void *sigma,
                               void *pot, void *grad, void *dSdn, void *surf_grad,
                               double *phase_ms, void *stream);

/* Autotuner for the applies of one precision.  The octree is not fixed by
 * the method (Section 4 leaves it to the point FMM), and its depth trades
 * near-field pair sums against M2L translations; the leaf kernel's thread
 * shape trades lanes per target against targets per block.  lb_autotune
 * times lb_apply_gradS with nd densities (HIP events on `stream`, three
 * launches after one untimed) for every distinct forest obtained from
 * leaf_src in {1/4, 1/2, 1, 2, 4} x its current value (each tree's depth:
 * the first level whose mean number of oversampled points per leaf is at
 * most leaf_src, coarsened in FP32 so that the leaf side stays above the
 * near-mask radius) and leaf_fmax in {64, 32, 16} (most lanes per target,
 * one block per leaf: leaf_split 0), then, at the fastest of those,
 * leaf_split in {1, 2, 3} (a leaf cut into up to that many blocks), then
 * the schedule of the overlapped apply (near-field kernel forked after the
 * strengths or after P2M; on every work item or on 4 or 6 blocks per
 * compute unit: fork_late, near_grid = 0 or the block count; the gradient
 * apply's correction sums fused with the final combination or run first on
 * the side stream: corr_early), and keeps the fastest configuration.  Corrections and
 * node data are kept; captured GMRES graphs and transposed trees are dropped
 * and rebuilt on next use.  Results are the same operator up to the FMM
 * truncation error.  A direct context (LB_DIRECT) tunes leaf_fmax only.
 * Synchronizes the device; nd <= 64; info: host, nullable. */
#define LB_TUNE_MAX_TRIALS 32
typedef struct {
  int32_t leaf_src, leaf_fmax, leaf_split; /* chosen configuration */
  int32_t depth;                      /* deepest tree level of the chosen forest */
  int32_t n_trials;                   /* entries used in the trial arrays */
  double ms_best, ms_default;         /* apply time chosen / of the configuration on entry */
  int32_t trial_leaf_src[LB_TUNE_MAX_TRIALS], trial_fmax[LB_TUNE_MAX_TRIALS],
      trial_split[LB_TUNE_MAX_TRIALS], trial_depth[LB_TUNE_MAX_TRIALS];
  double trial_ms[LB_TUNE_MAX_TRIALS];
  int32_t fork_late, near_grid;       /* chosen schedule of the overlapped apply */
  int32_t trial_fork_late[LB_TUNE_MAX_TRIALS], trial_near_grid[LB_TUNE_MAX_TRIALS];
  int32_t corr_early;                 /* gradient apply: correction sums first on the side stream */
  int32_t trial_corr_early[LB_TUNE_MAX_TRIALS];
} lb_tune_info;
lb_status lb_autotune(lb_ctx *ctx, int prec, int nd, lb_tune_info *info, void *stream);

/* Apply a configuration of one precision without timing (for instance one
 * that lb_autotune chose earlier for the same geometry): config->leaf_src
 * (16 .. 2^20; a direct context keeps its own), leaf_fmax (power of two,
 * 1..64), leaf_split (0..3), fork_late (0 or 1), near_grid (>= 0) and
 * corr_early (0 or 1); the other fields are ignored.  Rebuilds the octrees when leaf_src differs;
 * captured graphs and transposed trees are dropped as by lb_autotune.
 * Synchronizes the device.  Errors: LB_EINVAL. */
lb_status lb_set_tuning(lb_ctx *ctx, int prec, const lb_tune_info *config);

/* The discretized A3 operator of eq. (ie-dis2), applied right to left as in
 * Section 4.3: out = -tau/4 + S'[S' tau] - (S''+D')[S tau] - 2H S'[S tau]
 * + W S[S tau].  tau, out: device [nd][N]. */
lb_status lb_apply_A3(lb_ctx *ctx, int nd, int prec, const void *tau, void *out,
                      void *stream);

/* Transpose of lb_apply_A3 (the same discrete operator of the same
 * precision): out = A3^T v = -v/4 + S'^T S'^T v - S^T (S''+D')^T v
 * - S^T S'^T (2 H v) + (sum_i v_i / area) S^T S^T w, through two FMMs on the
 * transposed tree (the first with dipole and quadrupole sources at the
 * nodes).  v, out: device [nd][N].  The first call for a precision builds the
 * transposed tree and S^T S^T w and synchronizes the device. */
lb_status lb_apply_A3_adj(lb_ctx *ctx, int nd, int prec, const void *v, void *out,
                          void *stream);

/* Solve Delta_Gamma u = f for the mean-zero u (Lemma 1), through
 * A3 sigma = f - mean(f) and u = S[S[sigma]] (eq. ie-dis2, Section 6 GMRES:
 * x0 = 0, no restart, relative Euclidean residual < tol, at most
 * opts.max_iter iterations per inner solve); with LB_SOLVE_A2 or-ed into
 * `mode`, through A2 sigma = S[f - mean(f)] and u = S[sigma] (eq. ie-dis1),
 * the residual relative to S[f - mean(f)].  f, u: device double [nrhs][N].
 * info: host [nrhs * n_surf], nullable.  Synchronizes `stream`.  Returns LB_ENOCONV
 * if some right-hand side did not reach tol (its best iterate is written),
 * LB_ENOTMEANZERO in strict-mean mode. */
lb_status lb_solve(lb_ctx *ctx, int nrhs, const double *f, double *u, double tol,
                   int mode, lb_solve_info *info, void *stream);

/* Adjoint of lb_solve with respect to f: with u = S S A3^{-1} (f - W f)
 * (W f = sum_i w_i f_i / area), fbar = (I - w 1^T / area) A3^{-T} S^T S^T ubar,
 * the A3^T system solved by GMRES (or FP32 inner / FP64 outer refinement) to
 * tol as in lb_solve.  ubar, fbar: device double [nrhs][N]; info: host
 * [nrhs * n_surf], nullable (removed_mean reports sum_i y_i / area of the solution y).
 * Synchronizes `stream`; LB_ENOCONV as lb_solve. */
lb_status lb_solve_adj(lb_ctx *ctx, int nrhs, const double *ubar, double *fbar, double tol,
                       int mode, lb_solve_info *info, void *stream);

/* A1 (Section 4.1, eq. ie-dis0): A1[tau] = div S[grad_Gamma S tau] + S W S tau,
 * the non-second-kind discretization of S (Delta + W) S, applied right to
 * left: S tau and mu = grad_Gamma S tau by one gradient apply, the three
 * Cartesian components of mu as densities of a second gradient apply,
 * div S[mu] = sum_l (d_l S)[mu_l], plus W(S tau) S[1] per surface (S[1]
 * computed on first use).  tau, out: device [nd][N] in the precision `prec`
 * (32 or 64).  Stream-ordered.  Errors as lb_apply_S. */
lb_status lb_apply_A1(lb_ctx *ctx, int nd, int prec, const void *tau, void *out, void *stream);

/* A2 (Section 4.2, eq. ie-dis1): A2[tau] = -tau/4 + D D tau
 * - S (S'' + D' + 2 H S') tau + S W S tau, the second-kind discretization of
 * S (Delta + W) S with the double layer D = grad_y G . nu (Section 3), applied
 * right to left: mu1 = D tau and mu2 = -(S''+D'+2HS') tau + W S tau from one
 * charge + dipole FMM (S, S', S''+D' of tau) and one dipole FMM (D tau), then
 * A2 tau = -tau/4 + S mu2 + D mu1 from one charge + dipole potential FMM, each
 * with its near corrections (the D column of lb_get_corrections included).
 * tau, out: device [nd][N] in the precision `prec` (32 or 64).  A2's
 * right-hand side is S[f] and its solution u = S sigma (eq. ie-dis1).
 * Stream-ordered.  Errors as lb_apply_S. */
lb_status lb_apply_A2(lb_ctx *ctx, int nd, int prec, const void *tau, void *out, void *stream);

/* Surface gradient of node values (Section 2): on each patch the order-k
 * interpolant of psi differentiated along the chart, with the metric of the
 * chart derivatives X_u, X_v given at the nodes: grad psi = g^{ij} (d_i psi) X_j.  psi: device double [nd][N]; grad:
 * device double [nd][N][3].  Stream-ordered on `stream`.  Errors: LB_EINVAL
 * (null pointer, nd < 1, host-only context), LB_EHIP. */
lb_status lb_surface_grad(lb_ctx *ctx, int nd, const double *psi, double *grad, void *stream);

/* Surface divergence (Section 2) of the tangential part of V (cross_n = 0)
 * or of n x V (cross_n = 1): |g|^{-1/2} d_i (|g|^{1/2} V^i) with V^i the
 * contravariant components, the derivatives as in lb_surface_grad.
 * V: device double [nd][N][3]; div: device double [nd][N].  Stream-ordered. */
lb_status lb_surface_div(lb_ctx *ctx, int nd, const double *V, int cross_n, double *div,
                         void *stream);

/* Hodge decomposition of nf tangential fields (harmonic vector field
 * section): F = grad alpha + n x grad beta + H with Delta alpha = div F,
 * Delta beta = -div(n x F) (both mean zero; one batched lb_solve of 2 nf
 * right-hand sides, alpha's first) and H = F - grad alpha - n x grad beta,
 * divergence free and with n x H divergence free (a harmonic field).
 * F: device double [nf][N][3] (its tangential part is used); H: device
 * double [nf][N][3]; alpha, beta: device double [nf][N], nullable.  tol,
 * mode and info [2 nf n_surf] as lb_solve.  Synchronizes `stream`; returns
 * LB_ENOCONV as lb_solve (H is still written). */
lb_status lb_hodge(lb_ctx *ctx, int nf, const double *F, double *alpha, double *beta, double *H,
                   double tol, int mode, lb_solve_info *info, void *stream);

/* Release all host and device state (NULL is ignored). */
void lb_destroy(lb_ctx *ctx);

/* Thread-local message describing the last failure of this thread. */
const char *lb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
