"""ProHD hot path on MI355X (gfx950): thin Python binding over libprohd.so.

The C ABI (include/prohd.h) does all the work in HIP kernels; this module only
marshals torch tensors (device memory, the current HIP stream) into pointers
and sizes.  It raises when the native library is missing -- there is no
fallback path.
"""

from ._lib import (  # noqa: F401
    ProhdError,
    Workspace,
    lib,
    library_path,
    workspace_size,
    prohd_project,
    prohd_select,
    prohd_hd,
    exact_hd,
    exact_hd_noalloc,
    NOALLOC_SCRATCH_BYTES,
    prohd,
    adaptive,
    decode_result,
    RESULT_BYTES,
    k_rule,
    alpha_k,
    default_m,
    prune_levels,
    mlp_param_count,
    mlp_workspace_size,
    mlp_init,
    mlp_score,
    mlp_grad,
    mlp_adamw,
    mlp_train_step,
    centroid,
    select_scored,
    prohd_top_keys,
    top_keys,
    TOPK_WS_BYTES,
    BatchPlan,
    certificate,
    profile_enable,
    profile_reset,
    profile_read,
    version,
    DIRS_GIVEN,
    INNER_FULL,
    SYNC,
    PRUNE,
    PREC_BF16,
    PREC_FP8,
)
