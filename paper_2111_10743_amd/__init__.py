"""MI355X Laplace-Beltrami layer potentials: FMM + locally corrected quadrature.

The compute path lives in ``liblb.so`` (HIP kernels for gfx950 and host C++,
C ABI in ``include/lb.h``); ``lb`` is its ctypes binding.
"""
from .lb import (Surface, ref_nodes, default_opts, LBError, LB_PREC_FP32, LB_PREC_FP64,  # noqa: F401
                 LB_SOLVE_FP64, LB_SOLVE_FP32_REFINE, LB_OK, LB_ENOCONV, apply_S, apply_gradS, build_tree, solve)
