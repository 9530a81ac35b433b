"""MI355X Laplace-Beltrami layer potentials: FMM + locally corrected quadrature.

The compute path lives in ``liblb.so`` (HIP kernels for gfx950 and host C++,
C ABI in ``include/lb.h``); ``lb`` is its ctypes binding.
"""
from .lb import (Surface, ref_nodes, default_opts, LBError, LB_PREC_FP32, LB_PREC_FP64,  # noqa: F401
                 LB_SOLVE_FP64, LB_SOLVE_FP32_REFINE, LB_SOLVE_A2, LB_OK, LB_ENOCONV, LB_EINVAL, LB_ENOMEM, LB_EHIP,
                 LB_ENOTMEANZERO, LB_EGEOM, LB_STRICT_MEAN, LB_DIRECT, LB_NO_GRAPH, LB_NO_OVERLAP,
                 LB_NO_P2M_TABLES, LB_HOST_OCTREE, LB_HOST_QUAD, lib, apply_S, apply_gradS, build_tree, solve)
