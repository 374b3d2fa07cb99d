"""MI355X-native #DNN-Verification counter with Symbolic Linear Relaxation.

The engine is the C-ABI library ``libslrcount.so`` (hand-written HIP for gfx950, declared in
``include/slrcount.h``); this package is its thin Python binding.  Build the library with
``python -m paper_2312_05890_amd.build``.
"""
from .slrcount import (EXPORTS, SAFE, SLR_BUDGET, SLR_OK, UNDECIDED, UNSAFE, Net, Property,  # noqa: F401
                       Batch, SlrError, alpha_kernel_variant, alpha_optimize, alpha_size, alpha_state_variant, alpha_tape_size, alpha_workspace_size,
                       bound_boxes, bound_boxes_alpha, bound_boxes_backward, bound_boxes_relax, bound_kernel_variant,
                       bound_tape_size, bound_tile_shape,
                       count_approx, count_exact, count_exact_batch, count_exact_noalloc,
                       count_exact_noalloc_max_bytes, count_exact_stack, stack_workspace_size, last_error, lib, load_net, load_property,
                       sample_violations, workspace_size)


def __getattr__(name):
    if name == "SLRBound":
        from . import slrcount
        return slrcount.SLRBound
    raise AttributeError(name)
