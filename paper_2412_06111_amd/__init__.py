"""MI355X engine for the streaming sketch phase of the tree tensor network Nystrom
method (TTNN) and its sequential variant (STTNN): HIP kernels for gfx950 behind a
C ABI (include/ttnn.h), and a thin Python binding."""

from ._lib import (  # noqa: F401
    Plan, TTNNError, diff_norms, update_batched, tree_arrays, footprint_estimate, workspace_bytes, lib,
    order_cost, order_search, visit_places, visit_spec,
    F64, F32, BF16, TTNN, STTNN, KR, SK_R, SK_OMEGA, SK_PSI, TORCH_DTYPE, DTYPE_NAME,
)
