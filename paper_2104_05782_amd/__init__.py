"""lupp: LU factorization with partial pivoting on AMD MI355X (gfx950).

Thin ctypes binding over the C ABI in ``include/lupp.h``; every computation
runs in the HIP library ``liblupp.so`` built by ``paper_2104_05782_amd.build``.
PyTorch supplies device memory and the current stream only.  Importing this
package fails loudly when the library is missing: there is no CPU fallback.

Matrices are column-major: an m x n matrix is a tensor ``A`` of shape (m, n)
with ``A.stride(0) == 1`` (e.g. ``torch.empty(n, m).t()``).
"""
from ._binding import (  # noqa: F401
    LIB_PATH,
    IR_STATUS,
    PREC,
    IrOpts,
    IrReport,
    LuppError,
    BatchedSchedule,
    batched_shapes,
    Handle,
    colmajor,
    default_handle,
    lupp_dgetrf,
    lupp_dgetrs,
    lupp_sgetrf,
    lupp_sgetrs,
    getrf,
    geqrf,
    randutv,
    lupp_drandutv,
    lupp_dgeqrf,
    getrs,
    gesv_batched,
    gesv_mixed,
    lupp_xgesv_batched,
    lupp_dgesv_batched_noalloc,
    NOALLOC_MAX_BATCH,
    ir_opts,
    lupp_dgesv_mixed,
    status_string,
)
