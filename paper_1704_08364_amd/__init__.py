"""BST backprojection on AMD MI355X: a HIP library (libbst.so, C ABI in
include/bst.h) and its thin ctypes binding.

    from paper_1704_08364_amd import Plan
    plan = Plan(n_det=2048, n_angles=2048, max_batch=64)
    img = plan.backproject(sino)            # sino: cuda float32 [B][V][n]
"""
from .binding import (  # noqa: F401
    Batch,
    BstError,
    BstNativeMissing,
    Event,
    Plan,
    LIB_PATH,
    lib,
    make_params,
    query_max_batch,
    query_workspace,
)
