"""MI355X-native voxel-wise 3D structure tensor (fibre orientation, FA, HA, IA).

The compute path is the HIP library ``libst.so`` (hand-written gfx950
kernels behind a C ABI declared in ``include/st.h``); this package is its
thin Python binding.  Building: ``python -m paper_2508_07476_amd.csrc.build``.
"""

from ._binding import (  # noqa: F401
    ALL_OUTPUTS,
    ST_BATCH_GROUPED,
    ST_BATCH_MAX_LANES,
    ST_NOALLOC_SCRATCH_BYTES,
    ST_SURROGATE_WEIGHTS,
    SURROGATE_OUTPUTS,
    Batch,
    StChunk,
    LIB_PATH,
    ST_DTYPE_F32,
    ST_DTYPE_U16,
    ST_ERR_DEVICE,
    ST_ERR_INVALID_ARG,
    ST_ERR_OUT_OF_MEMORY,
    ST_ERR_UNSUPPORTED,
    ST_FLAG_DEGENERATE,
    ST_FLAG_ON_AXIS,
    ST_FLAG_OUTSIDE_MASK,
    ST_OK,
    SIGNATURES,
    StError,
    load_library,
    profile_enable,
    profile_read,
    profile_reset,
    st_angles,
    st_compute,
    st_compute_noalloc,
    st_filter_radius,
    st_surrogate_adam,
    st_surrogate_fallback_info,
    st_surrogate_grad,
    st_surrogate_grad_workspace_bytes,
    st_surrogate_infer,
    st_version,
    st_workspace_bytes,
)
