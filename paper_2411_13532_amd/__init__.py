"""MI355X (gfx950) mode-n tensor-times-matrix chain: Y = X x1 A x2 B x3 C, and the
periodic compact derivative scheme applied along one mode (X x_n A_c^-1 B_c).

The computation lives in libttm.so (hand-written HIP kernels behind the C
interface in include/ttm.h); this package is its PyTorch binding.
"""
from .ttm import (COMPACT6, BatchedPlan, TTMChain, chain, chain_backward, chain_backward_workspace_size,
                  chain_noalloc, chain_workspace_size, compact_apply, hosvd, reorder, set_slab_kernel, stream_copy,
                  timing_collect, timing_enable, ttm_chain)

__all__ = ["COMPACT6", "BatchedPlan", "TTMChain", "chain", "chain_backward", "chain_backward_workspace_size",
           "chain_noalloc", "chain_workspace_size", "compact_apply", "hosvd", "reorder", "set_slab_kernel", "stream_copy",
           "timing_collect",
           "timing_enable", "ttm_chain"]
