"""MI355X-native kernel-compensated Maxwell eigensolver for anisotropic photonic crystals.

Thin Python binding of the C ABI in include/kcpc.h (libkcpc.so, built in-tree by
`paper_2511_17107_amd.build`).  The binding only marshals arguments: every step of the
operator application, the preconditioner and the eigensolver runs in the library's HIP
kernels.  PyTorch provides device memory and streams.  There is no fallback: if the
library is missing or fails to load, every call raises.
"""
from ._binding import (  # noqa: F401
    KC_EPS_CROSSDOF,
    KC_EPS_DIAGONAL,
    KC_EPS_TRIVIAL,
    KC_ERR_NO_CONVERGENCE,
    KC_START_PLANE_WAVES,
    KC_START_RANDOM,
    KC_FLAG_HPD_UNPROVEN,
    KC_KFLAG_K_OUTSIDE,
    KC_KFLAG_SPURIOUS_RISK,
    KC_PREC_FP32,
    KC_PREC_FP64,
    KC_PRECOND_DIAG,
    KC_PRECOND_LEARNED,
    KC_PRECOND_TRANSVERSE,
    KcError,
    Net,
    block_gram,
    block_gram_noalloc,
    block_update,
    block_work_bytes,
    Op,
    kc_create,
    kc_fft3d,
    kc_supported_n,
    lib,
    lib_path,
)

SCHEMES = {"diagonal": KC_EPS_DIAGONAL, "trivial": KC_EPS_TRIVIAL, "crossdof": KC_EPS_CROSSDOF}
