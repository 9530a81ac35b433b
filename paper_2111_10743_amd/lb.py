"""ctypes binding of liblb.so (include/lb.h): argument marshalling only.

Device buffers are torch tensors on the current HIP device; every call is
enqueued on torch's current stream.  The library must be built
(``python -m paper_2111_10743_amd.build``); importing this module without it
raises, there is no fallback.
"""
import ctypes
import functools
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblb.so")

LB_OK = 0
LB_ENOCONV = 1
LB_EINVAL = -1
LB_ENOMEM = -2
LB_EHIP = -3
LB_ENOTMEANZERO = -4
LB_EGEOM = -5
LB_PREC_FP32 = 32
LB_PREC_FP64 = 64
LB_SOLVE_FP64 = 0
LB_SOLVE_FP32_REFINE = 1
LB_SOLVE_A2 = 4  # or-ed into a mode: the A2 formulation (eq. ie-dis1)
LB_STRICT_MEAN = 1
LB_HOST_ONLY = 2
LB_DIRECT = 4
LB_NO_P2M_TABLES = 8
LB_HOST_OCTREE = 16
LB_HOST_QUAD = 128
LB_NO_GRAPH = 32
LB_NO_OVERLAP = 64

EXPORTED = ("lb_default_opts", "lb_ref_nodes", "lb_setup", "lb_setup_batch", "lb_get_sizes", "lb_get_geometry",
            "lb_get_corrections", "lb_get_tree", "lb_tree_build", "lb_tree_get", "lb_tree_destroy", "lb_apply_S", "lb_apply_gradS", "lb_apply_gradS_adj", "lb_apply_S_adj", "lb_apply_S_adj_X", "lb_autotune",
            "lb_apply_gradS_timed", "lb_apply_A3", "lb_apply_A3_adj", "lb_solve", "lb_solve_adj",
            "lb_surface_grad", "lb_surface_div", "lb_hodge", "lb_apply_A1", "lb_set_tuning", "lb_destroy",
            "lb_last_error", "lb_apply_gradS_noalloc", "lb_export_setup", "lb_import_setup", "lb_apply_A2")
PHASES = ("strengths", "p2m", "m2m", "m2l", "l2l", "leaf", "combine")


class Opts(ctypes.Structure):
    _fields_ = [("eta_near", ctypes.c_double), ("over_q", ctypes.c_int), ("p_f32", ctypes.c_int),
                ("p_f64", ctypes.c_int), ("leaf_src", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("flags", ctypes.c_int), ("self_n", ctypes.c_int), ("near_q", ctypes.c_int),
                ("near_adm", ctypes.c_double), ("m2l_trunc32", ctypes.c_double), ("m2l_trunc64", ctypes.c_double),
                ("over_q32", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_steps", ctypes.c_int), ("rel_resid", ctypes.c_double),
                ("removed_mean", ctypes.c_double), ("t_setup", ctypes.c_double), ("t_solve", ctypes.c_double)]


class Sizes(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("n_patches", "n_p", "N", "n_o", "N_o", "nnz_blocks",
                                               "fmm_levels", "fmm_leaves", "p_f32", "p_f64",
                                               "p2p_pairs32", "m2l_pairs32", "p2p_pairs64", "m2l_pairs64",
                                               "n_surf", "m2l_flops32", "m2l_flops64", "n_o32", "N_o32")]


class TreeInfo(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("nbox", ctypes.c_int32), ("nleaf", ctypes.c_int32),
                ("nulist", ctypes.c_int32), ("nvlist", ctypes.c_int32), ("lo", ctypes.c_double * 3),
                ("side", ctypes.c_double)]


TUNE_MAX = 32


class TuneInfo(ctypes.Structure):
    _fields_ = [("leaf_src", ctypes.c_int32), ("leaf_fmax", ctypes.c_int32), ("leaf_split", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("n_trials", ctypes.c_int32), ("ms_best", ctypes.c_double),
                ("ms_default", ctypes.c_double),
                ("trial_leaf_src", ctypes.c_int32 * TUNE_MAX), ("trial_fmax", ctypes.c_int32 * TUNE_MAX),
                ("trial_split", ctypes.c_int32 * TUNE_MAX), ("trial_depth", ctypes.c_int32 * TUNE_MAX),
                ("trial_ms", ctypes.c_double * TUNE_MAX),
                ("fork_late", ctypes.c_int32), ("near_grid", ctypes.c_int32),
                ("trial_fork_late", ctypes.c_int32 * TUNE_MAX), ("trial_near_grid", ctypes.c_int32 * TUNE_MAX),
                ("corr_early", ctypes.c_int32), ("trial_corr_early", ctypes.c_int32 * TUNE_MAX)]


class LBError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"lb error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2111_10743_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        L.lb_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.lb_ref_nodes.argtypes = [ip, dp, dp]
        L.lb_setup.argtypes = [ctypes.POINTER(vp), ip, ip, dp, dp, dp, ctypes.POINTER(Opts), vp]
        L.lb_setup_batch.argtypes = [ctypes.POINTER(vp), ip, ctypes.POINTER(ctypes.c_int32), ip, dp, dp, dp,
                                     ctypes.POINTER(Opts), vp]
        L.lb_get_sizes.argtypes = [vp, ctypes.POINTER(Sizes)]
        L.lb_export_setup.argtypes = [vp, ctypes.c_char_p]
        L.lb_import_setup.argtypes = [ctypes.POINTER(vp), ctypes.c_char_p, vp]
        L.lb_get_geometry.argtypes = [vp, dp, dp, dp]
        L.lb_get_corrections.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32), dp]
        L.lb_get_tree.argtypes = [vp, ip, ip, ip, ctypes.POINTER(TreeInfo)] + [vp] * 9
        L.lb_tree_build.argtypes = [ctypes.POINTER(vp), dp, ctypes.c_int64, dp, ctypes.c_int64, ip,
                                    ctypes.c_double, ip, ip]
        L.lb_tree_get.argtypes = [vp, ctypes.POINTER(TreeInfo)] + [vp] * 9
        L.lb_tree_destroy.argtypes = [vp]
        L.lb_apply_S.argtypes = [vp, ip, ip, vp, vp, vp]
        L.lb_apply_gradS.argtypes = [vp, ip, ip, vp, vp, vp, vp, vp, vp]
        L.lb_apply_gradS_noalloc.argtypes = [vp, ip, ip, vp, vp, vp, vp, vp, vp]
        L.lb_apply_gradS_adj.argtypes = [vp, ip, ip, vp, vp, vp, vp, vp, vp]
        L.lb_apply_S_adj.argtypes = [vp, ip, ip, vp, vp, vp]
        L.lb_apply_S_adj_X.argtypes = [vp, ip, ip, vp, vp, vp, vp]
        L.lb_autotune.argtypes = [vp, ip, ip, ctypes.POINTER(TuneInfo), vp]
        L.lb_apply_gradS_timed.argtypes = [vp, ip, ip, vp, vp, vp, vp, vp, dp, vp]
        L.lb_apply_A3.argtypes = [vp, ip, ip, vp, vp, vp]
        L.lb_solve.argtypes = [vp, ip, vp, vp, ctypes.c_double, ip, ctypes.POINTER(SolveInfo), vp]
        L.lb_solve_adj.argtypes = [vp, ip, vp, vp, ctypes.c_double, ip, ctypes.POINTER(SolveInfo), vp]
        L.lb_apply_A3_adj.argtypes = [vp, ip, ip, vp, vp, vp]
        L.lb_apply_A1.argtypes = [vp, ip, ip, vp, vp, vp]
        L.lb_apply_A2.argtypes = [vp, ip, ip, vp, vp, vp]
        L.lb_set_tuning.argtypes = [vp, ip, ctypes.POINTER(TuneInfo)]
        L.lb_surface_grad.argtypes = [vp, ip, vp, vp, vp]
        L.lb_surface_div.argtypes = [vp, ip, vp, ip, vp, vp]
        L.lb_hodge.argtypes = [vp, ip, vp, vp, vp, vp, ctypes.c_double, ip, ctypes.POINTER(SolveInfo), vp]
        L.lb_destroy.argtypes = [vp]
        L.lb_destroy.restype = None
        L.lb_tree_destroy.restype = None
        L.lb_last_error.restype = ctypes.c_char_p
        for n in EXPORTED:
            if n not in ("lb_destroy", "lb_last_error", "lb_tree_destroy"):
                getattr(L, n).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(code):
    if code < 0:
        raise LBError(code, lib().lb_last_error().decode())
    return code


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def default_opts():
    o = Opts()
    _check(lib().lb_default_opts(ctypes.byref(o)))
    return o


def ref_nodes(order):
    """(uv [n_p, 2], w_ref [n_p]) of the library's order-k node set."""
    n_p = (order + 1) * (order + 2) // 2
    uv = np.zeros((n_p, 2))
    w = np.zeros(n_p)
    _check(lib().lb_ref_nodes(order, _dp(uv), _dp(w)))
    return uv, w


def _tree_arrays(getter, nt, ns):
    info = TreeInfo()
    _check(getter(ctypes.byref(info), *([None] * 9)))
    out = {"depth": info.depth, "lo": np.array(info.lo[:]), "side": info.side,
           "tgt_perm": np.zeros(nt, np.int64), "src_perm": np.zeros(ns, np.int64),
           "leaf_ranges": np.zeros((info.nleaf, 4), np.int32),
           "ulist_ptr": np.zeros(info.nleaf + 1, np.int32), "ulist": np.zeros(info.nulist, np.int32),
           "vlist_ptr": np.zeros(info.nbox + 1, np.int32), "vlist_src": np.zeros(info.nvlist, np.int32),
           "vlist_off": np.zeros(info.nvlist, np.int32), "boxes": np.zeros((info.nbox, 5), np.int32)}
    ptr = [out[k].ctypes.data_as(ctypes.c_void_p) for k in ("tgt_perm", "src_perm", "leaf_ranges", "ulist_ptr",
                                                           "ulist", "vlist_ptr", "vlist_src", "vlist_off", "boxes")]
    _check(getter(ctypes.byref(info), *ptr))
    return out


def build_tree(tgt, src, leaf_src=1024, min_leaf_side=0.0, depth=-1, device=True):
    """The library's FMM octree of arbitrary points (lb_tree_build), as numpy arrays."""
    tgt = np.ascontiguousarray(tgt, dtype=np.float64)
    src = np.ascontiguousarray(src, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(lib().lb_tree_build(ctypes.byref(h), _dp(tgt), tgt.shape[0], _dp(src), src.shape[0], leaf_src,
                               min_leaf_side, depth, int(device)))
    try:
        return _tree_arrays(lambda *a: lib().lb_tree_get(h, *a), tgt.shape[0], src.shape[0])
    finally:
        lib().lb_tree_destroy(h)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Surface:
    """One discretized surface: lb_setup ... lb_destroy."""

    def __init__(self, X, Xu, Xv, order, opts=None, host_only=False, direct=False, p2m_tables=True,
                 host_octree=False, patches_per_surf=None, graphs=True, overlap=True, host_quad=False, **kw):
        """One surface, or with patches_per_surf several independent surfaces
        (their patches one after the other in X, Xu, Xv; lb_setup_batch)."""
        if X is None:  # Surface.load: the context comes from a saved setup (opts = its path)
            self.order = order
            self.host_only = False
            self._ctx = ctypes.c_void_p()
            _check(lib().lb_import_setup(ctypes.byref(self._ctx), os.fsencode(opts), _stream()))
            sz = self.sizes
            self.N = sz["N"]
            self.n_surf = sz["n_surf"]
            return
        X = np.ascontiguousarray(X, dtype=np.float64)
        Xu = np.ascontiguousarray(Xu, dtype=np.float64)
        Xv = np.ascontiguousarray(Xv, dtype=np.float64)
        o = opts if opts is not None else default_opts()
        for k, v in kw.items():
            setattr(o, k, v)
        if host_only:
            o.flags |= LB_HOST_ONLY
        if direct:
            o.flags |= LB_DIRECT
        if not p2m_tables:
            o.flags |= LB_NO_P2M_TABLES
        if host_octree:
            o.flags |= LB_HOST_OCTREE
        if not graphs:
            o.flags |= LB_NO_GRAPH
        if not overlap:
            o.flags |= LB_NO_OVERLAP
        if host_quad:
            o.flags |= LB_HOST_QUAD
        self.order = order
        self.host_only = host_only
        self._ctx = ctypes.c_void_p()
        stream = None if host_only else _stream()
        if patches_per_surf is None:
            _check(lib().lb_setup(ctypes.byref(self._ctx), X.shape[0], order, _dp(X), _dp(Xu), _dp(Xv),
                                  ctypes.byref(o), stream))
        else:
            pps = np.ascontiguousarray(patches_per_surf, dtype=np.int32)
            if int(pps.sum()) != X.shape[0]:
                raise ValueError("patches_per_surf must add up to the number of patches")
            _check(lib().lb_setup_batch(ctypes.byref(self._ctx), len(pps),
                                        pps.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), order, _dp(X), _dp(Xu),
                                        _dp(Xv), ctypes.byref(o), stream))
        sz = self.sizes
        self.N = sz["N"]
        self.n_surf = sz["n_surf"]

    @property
    def sizes(self):
        """lb_get_sizes (queried on each access: tuning rebuilds the trees)."""
        s = Sizes()
        _check(lib().lb_get_sizes(self._ctx, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in Sizes._fields_}

    def save(self, path):
        """lb_export_setup: write this context's setup (corrections, tuning) to path."""
        _check(lib().lb_export_setup(self._ctx, os.fsencode(path)))

    @classmethod
    def load(cls, path, order=None):
        """lb_import_setup: a context from a saved setup, without generating
        the corrections."""
        return cls(None, None, None, order, opts=path)

    def close(self):
        if self._ctx:
            lib().lb_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def geometry(self):
        w = np.zeros(self.N)
        n = np.zeros((self.N, 3))
        H = np.zeros(self.N)
        _check(lib().lb_get_geometry(self._ctx, _dp(w), _dp(n), _dp(H)))
        return w, n, H

    def corrections(self):
        nb = self.sizes["nnz_blocks"]
        ptr = np.zeros(self.N + 1, dtype=np.int64)
        patch = np.zeros(nb, dtype=np.int32)
        vals = np.zeros((nb, self.sizes["n_p"], 7))
        _check(lib().lb_get_corrections(self._ctx, ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        patch.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(vals)))
        return ptr, patch, vals

    def tree(self, prec=32, transposed=False, surf=0, counts=None):
        """The FMM octree of one surface (see lb_get_tree in include/lb.h) as
        numpy arrays; counts = (nodes, oversampled points of that precision's
        far rule) of that surface (default: the whole context, right for one
        surface)."""
        nn, no = counts if counts is not None else (self.N, self.sizes["N_o32" if prec == 32 else "N_o"])
        nt, ns = (no, nn) if transposed else (nn, no)
        return _tree_arrays(lambda *a: lib().lb_get_tree(self._ctx, prec, int(transposed), surf, *a), nt, ns)

    # -- device calls (torch tensors) --------------------------------------
    @staticmethod
    def _prec(t):
        import torch
        if t.dtype == torch.float32:
            return LB_PREC_FP32
        if t.dtype == torch.float64:
            return LB_PREC_FP64
        raise TypeError("density must be float32 or float64")

    def _nd(self, t):
        if not t.is_cuda or not t.is_contiguous() or t.numel() % self.N != 0:
            raise ValueError("density must be a contiguous device tensor with a multiple of N elements")
        return t.numel() // self.N

    def apply_S(self, sigma, out=None):
        import torch
        nd = self._nd(sigma)
        pot = out if out is not None else torch.empty_like(sigma)
        _check(lib().lb_apply_S(self._ctx, nd, self._prec(sigma), _ptr(sigma), _ptr(pot), _stream()))
        return pot

    def apply_gradS(self, sigma, want=("pot", "grad", "dSdn", "surf_grad")):
        import torch
        nd = self._nd(sigma)
        shape = sigma.shape
        o = {}
        o["grad"] = torch.empty(shape + (3,), dtype=sigma.dtype, device=sigma.device)
        for k in ("pot", "dSdn"):
            if k in want:
                o[k] = torch.empty_like(sigma)
        if "surf_grad" in want:
            o["surf_grad"] = torch.empty(shape + (3,), dtype=sigma.dtype, device=sigma.device)
        _check(lib().lb_apply_gradS(self._ctx, nd, self._prec(sigma), _ptr(sigma), _ptr(o.get("pot")),
                                    _ptr(o["grad"]), _ptr(o.get("dSdn")), _ptr(o.get("surf_grad")), _stream()))
        return o

    def apply_gradS_noalloc(self, sigma, out):
        """lb_apply_gradS_noalloc into caller-allocated outputs: out holds
        "grad" (shape sigma.shape + (3,)) and optionally "pot", "dSdn",
        "surf_grad"; the library allocates nothing."""
        _check(lib().lb_apply_gradS_noalloc(self._ctx, self._nd(sigma), self._prec(sigma), _ptr(sigma),
                                            _ptr(out.get("pot")), _ptr(out["grad"]), _ptr(out.get("dSdn")),
                                            _ptr(out.get("surf_grad")), _stream()))
        return out

    def apply_S_adj(self, gbar, out=None):
        """sigma_bar = S^T gbar (the transpose of the discrete S of this precision)."""
        import torch
        nd = self._nd(gbar)
        res = out if out is not None else torch.empty_like(gbar)
        _check(lib().lb_apply_S_adj(self._ctx, nd, self._prec(gbar), _ptr(gbar), _ptr(res), _stream()))
        return res

    def apply_S_adj_X(self, sigma, gbar):
        """X_bar [N, 3] = d/dX sum_d <gbar_d, S sigma_d>: the kernel-position
        derivative (nodes and far-rule points move with X; weights, P sigma and
        the near corrections fixed), summed over the densities."""
        import torch
        if sigma.shape != gbar.shape or sigma.dtype != gbar.dtype:
            raise ValueError("sigma and gbar must have the same shape and dtype")
        nd = self._nd(sigma)
        xbar = torch.empty((self.N, 3), dtype=sigma.dtype, device=sigma.device)
        _check(lib().lb_apply_S_adj_X(self._ctx, nd, self._prec(sigma), _ptr(sigma), _ptr(gbar), _ptr(xbar),
                                      _stream()))
        return xbar

    def apply_gradS_adj(self, gpot=None, ggrad=None, gdSdn=None, gsurf=None):
        """sigma_bar = S^T gpot + (grad S)^T ggrad + S'^T gdSdn + (grad_Gamma S)^T gsurf."""
        import torch
        ref = next(t for t in (gpot, gdSdn, ggrad, gsurf) if t is not None)
        if ref is gpot or ref is gdSdn:
            nd = self._nd(ref)
            shape = ref.shape
        else:
            nd = ref.numel() // (3 * self.N)
            shape = ref.shape[:-1]
        for t in (gpot, ggrad, gdSdn, gsurf):
            if t is not None and (not t.is_cuda or not t.is_contiguous() or t.dtype != ref.dtype):
                raise ValueError("cotangents must be contiguous device tensors of one dtype")
        res = torch.empty(shape, dtype=ref.dtype, device=ref.device)
        _check(lib().lb_apply_gradS_adj(self._ctx, nd, self._prec(ref), _ptr(gpot), _ptr(ggrad), _ptr(gdSdn),
                                        _ptr(gsurf), _ptr(res), _stream()))
        return res

    def autotune(self, prec=32, nd=1):
        """lb_autotune: time the gradient apply over octree depths (leaf_src)
        and leaf-kernel shapes (leaf_fmax), keep the fastest.  Returns the
        chosen configuration and every trial."""
        info = TuneInfo()
        _check(lib().lb_autotune(self._ctx, int(prec), int(nd), ctypes.byref(info), _stream()))
        n = info.n_trials
        return {"leaf_src": info.leaf_src, "leaf_fmax": info.leaf_fmax, "leaf_split": info.leaf_split,
                "depth": info.depth, "fork_late": info.fork_late, "near_grid": info.near_grid,
                "corr_early": info.corr_early,
                "ms_best": info.ms_best, "ms_default": info.ms_default,
                "trials": [{"leaf_src": info.trial_leaf_src[i], "leaf_fmax": info.trial_fmax[i],
                            "leaf_split": info.trial_split[i], "depth": info.trial_depth[i],
                            "fork_late": info.trial_fork_late[i], "near_grid": info.trial_near_grid[i],
                            "corr_early": info.trial_corr_early[i],
                            "ms": info.trial_ms[i]} for i in range(n)]}

    def set_tuning(self, prec, leaf_src, leaf_fmax, leaf_split=0, fork_late=0, near_grid=0, corr_early=0):
        """lb_set_tuning: apply a configuration (as returned by autotune)
        without timing."""
        c = TuneInfo()
        c.leaf_src, c.leaf_fmax, c.leaf_split = int(leaf_src), int(leaf_fmax), int(leaf_split)
        c.fork_late, c.near_grid, c.corr_early = int(fork_late), int(near_grid), int(corr_early)
        _check(lib().lb_set_tuning(self._ctx, int(prec), ctypes.byref(c)))

    def apply_gradS_timed(self, sigma):
        """apply_gradS plus per-phase milliseconds (HIP events on the stream)."""
        import torch
        nd = self._nd(sigma)
        shape = sigma.shape
        grad = torch.empty(shape + (3,), dtype=sigma.dtype, device=sigma.device)
        pot = torch.empty_like(sigma)
        ms = np.zeros(len(PHASES))
        _check(lib().lb_apply_gradS_timed(self._ctx, nd, self._prec(sigma), _ptr(sigma), _ptr(pot), _ptr(grad),
                                          None, None, _dp(ms), _stream()))
        return {"pot": pot, "grad": grad}, dict(zip(PHASES, ms))

    def apply_A3(self, tau, out=None):
        import torch
        nd = self._nd(tau)
        res = out if out is not None else torch.empty_like(tau)
        _check(lib().lb_apply_A3(self._ctx, nd, self._prec(tau), _ptr(tau), _ptr(res), _stream()))
        return res

    def apply_A1(self, tau, out=None):
        """lb_apply_A1: div S[grad_Gamma S tau] + S W S tau (Section 4.1)."""
        import torch
        nd = self._nd(tau)
        res = out if out is not None else torch.empty_like(tau)
        _check(lib().lb_apply_A1(self._ctx, nd, self._prec(tau), _ptr(tau), _ptr(res), _stream()))
        return res

    def apply_A2(self, tau, out=None):
        """lb_apply_A2: -tau/4 + D D tau - S (S''+D'+2HS') tau + S W S tau
        (Section 4.2, eq. ie-dis1)."""
        import torch
        nd = self._nd(tau)
        res = out if out is not None else torch.empty_like(tau)
        _check(lib().lb_apply_A2(self._ctx, nd, self._prec(tau), _ptr(tau), _ptr(res), _stream()))
        return res

    def apply_A3_adj(self, v, out=None):
        """A3^T v (the transpose of the discrete A3 of this precision)."""
        import torch
        nd = self._nd(v)
        res = out if out is not None else torch.empty_like(v)
        _check(lib().lb_apply_A3_adj(self._ctx, nd, self._prec(v), _ptr(v), _ptr(res), _stream()))
        return res

    def solve_adj(self, ubar, tol=1e-10, mode=LB_SOLVE_FP64):
        """fbar = (d u / d f)^T ubar for u = solve(f) (lb_solve_adj)."""
        import torch
        if ubar.dtype != torch.float64:
            raise TypeError("ubar must be float64")
        nrhs = self._nd(ubar)
        fbar = torch.empty_like(ubar)
        info = (SolveInfo * (nrhs * self.n_surf))()
        code = _check(lib().lb_solve_adj(self._ctx, nrhs, _ptr(ubar), _ptr(fbar), tol, mode, info, _stream()))
        infos = [{"iters": i.iters, "outer_steps": i.outer_steps, "rel_resid": i.rel_resid,
                  "removed_mean": i.removed_mean, "t_setup": i.t_setup, "t_solve": i.t_solve} for i in info]
        return fbar, infos, code

    def solve(self, f, tol=1e-10, mode=LB_SOLVE_FP64):
        import torch
        if f.dtype != torch.float64:
            raise TypeError("f must be float64")
        nrhs = self._nd(f)
        u = torch.empty_like(f)
        info = (SolveInfo * (nrhs * self.n_surf))()
        code = _check(lib().lb_solve(self._ctx, nrhs, _ptr(f), _ptr(u), tol, mode, info, _stream()))
        infos = [{"iters": i.iters, "outer_steps": i.outer_steps, "rel_resid": i.rel_resid,
                  "removed_mean": i.removed_mean, "t_setup": i.t_setup, "t_solve": i.t_solve} for i in info]
        return u, infos, code

    def _field(self, V):
        import torch
        if V.dtype != torch.float64 or not V.is_cuda or not V.is_contiguous() or V.shape[-1] != 3 \
                or V.numel() % (3 * self.N) != 0:
            raise ValueError("field must be a contiguous float64 device tensor [..., N, 3]")
        return V.numel() // (3 * self.N)

    def surface_grad(self, psi):
        """lb_surface_grad: surface gradient of node values psi [..., N] -> [..., N, 3] (FP64)."""
        import torch
        if psi.dtype != torch.float64:
            raise TypeError("psi must be float64")
        nd = self._nd(psi)
        g = torch.empty(psi.shape + (3,), dtype=psi.dtype, device=psi.device)
        _check(lib().lb_surface_grad(self._ctx, nd, _ptr(psi), _ptr(g), _stream()))
        return g

    def surface_div(self, V, cross_n=False):
        """lb_surface_div: surface divergence of the tangential part of V
        [..., N, 3] (of n x V with cross_n) -> [..., N] (FP64)."""
        import torch
        nd = self._field(V)
        d = torch.empty(V.shape[:-1], dtype=V.dtype, device=V.device)
        _check(lib().lb_surface_div(self._ctx, nd, _ptr(V), int(bool(cross_n)), _ptr(d), _stream()))
        return d

    def hodge(self, F, tol=1e-10, mode=LB_SOLVE_FP64):
        """lb_hodge: F = grad alpha + n x grad beta + H for fields F
        [..., N, 3]; returns (alpha, beta, H, info, code), info per solve
        (alpha's systems first)."""
        import torch
        nf = self._field(F)
        alpha = torch.empty(F.shape[:-1], dtype=F.dtype, device=F.device)
        beta = torch.empty_like(alpha)
        H = torch.empty_like(F)
        info = (SolveInfo * (2 * nf * self.n_surf))()
        code = _check(lib().lb_hodge(self._ctx, nf, _ptr(F), _ptr(alpha), _ptr(beta), _ptr(H), tol, mode, info,
                                     _stream()))
        infos = [{"iters": i.iters, "outer_steps": i.outer_steps, "rel_resid": i.rel_resid,
                  "removed_mean": i.removed_mean, "t_setup": i.t_setup, "t_solve": i.t_solve} for i in info]
        return alpha, beta, H, infos, code


@functools.lru_cache(maxsize=None)
def _autograd():
    import torch

    class ApplyS(torch.autograd.Function):
        """pot = S[sigma]; backward: sigma_bar = S^T pot_bar (lb_apply_S_adj)
        and, when the node positions X are an input, X_bar from
        lb_apply_S_adj_X (the kernel-position derivative)."""

        @staticmethod
        def forward(ctx, surf, sigma, X):
            ctx.surf = surf
            ctx.has_x = X is not None
            ctx.x_dtype = X.dtype if X is not None else None
            sigma = sigma.contiguous()
            if X is not None:
                ctx.save_for_backward(sigma)
            return surf.apply_S(sigma)

        @staticmethod
        def backward(ctx, gout):
            gout = gout.contiguous()
            gs = ctx.surf.apply_S_adj(gout) if ctx.needs_input_grad[1] else None
            gx = None
            if ctx.has_x and ctx.needs_input_grad[2]:
                (sigma,) = ctx.saved_tensors
                gx = ctx.surf.apply_S_adj_X(sigma, gout).to(ctx.x_dtype)
            return None, gs, gx

    class ApplyGradS(torch.autograd.Function):
        """(pot, grad, dSdn, surf_grad) = lb_apply_gradS(sigma); backward through
        lb_apply_gradS_adj with the four cotangents."""

        @staticmethod
        def forward(ctx, surf, sigma):
            ctx.surf = surf
            o = surf.apply_gradS(sigma.contiguous())
            return o["pot"], o["grad"], o["dSdn"], o["surf_grad"]

        @staticmethod
        def backward(ctx, gp, gg, gd, gs):
            c = [t.contiguous() if t is not None else None for t in (gp, gg, gd, gs)]
            if all(t is None for t in c):
                return None, None
            return None, ctx.surf.apply_gradS_adj(*c)

    class Solve(torch.autograd.Function):
        """u = lb_solve(f); backward: fbar = lb_solve_adj(ubar)."""

        @staticmethod
        def forward(ctx, surf, f, tol, mode):
            ctx.surf, ctx.tol, ctx.mode = surf, tol, mode
            u, info, code = surf.solve(f.contiguous(), tol=tol, mode=mode)
            if code != LB_OK:
                raise LBError(code, "solve did not converge")
            return u

        @staticmethod
        def backward(ctx, ubar):
            fbar, info, code = ctx.surf.solve_adj(ubar.contiguous(), tol=ctx.tol, mode=ctx.mode)
            if code != LB_OK:
                raise LBError(code, "adjoint solve did not converge")
            return None, fbar, None, None

    return ApplyS, ApplyGradS, Solve


def solve(surf, f, tol=1e-10, mode=LB_SOLVE_FP64):
    """Differentiable u = lb_solve(f) (torch.autograd; backward = lb_solve_adj)."""
    return _autograd()[2].apply(surf, f, tol, mode)


def apply_S(surf, sigma, X=None):
    """Differentiable S[sigma] (torch.autograd): the backward pass is the
    library's transposed apply.  X, optional: a [N, 3] tensor standing for
    the node positions the surface was set up with (its values are not read);
    when it requires grad, the backward pass returns the kernel-position
    derivative for it."""
    if X is not None and tuple(X.shape) != (surf.N, 3):
        raise ValueError(f"X must have shape ({surf.N}, 3)")
    return _autograd()[0].apply(surf, sigma, X)


def apply_gradS(surf, sigma):
    """Differentiable (S, grad S, S', grad_Gamma S)[sigma] (torch.autograd)."""
    return _autograd()[1].apply(surf, sigma)
