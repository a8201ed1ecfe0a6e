"""ctypes binding of libkcpc.so (include/kcpc.h): argument marshalling only."""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(HERE, "libkcpc.so")

KC_EPS_DIAGONAL, KC_EPS_TRIVIAL, KC_EPS_CROSSDOF = 0, 1, 2
KC_PREC_FP64, KC_PREC_FP32 = 0, 1
KC_OK, KC_ERR_NO_CONVERGENCE = 0, 6
KC_START_RANDOM, KC_START_PLANE_WAVES = 0, 1
KC_PRECOND_DIAG, KC_PRECOND_LEARNED, KC_PRECOND_TRANSVERSE = 0, 1, 2
KC_FLAG_HPD_UNPROVEN = 1
KC_KFLAG_K_OUTSIDE, KC_KFLAG_SPURIOUS_RISK = 1, 2

# caller allocator callbacks of kc_create (include/kcpc.h)
_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)


def _torch_alloc(ctx, nbytes):
    """Device memory for a handle's workspaces from PyTorch's caching allocator (current device
    and stream); NULL on failure (the library then reports KC_ERR_ALLOC)."""
    try:
        import torch

        return int(torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                      torch.cuda.current_stream()))
    except Exception:
        return None


def _torch_free(ctx, ptr, nbytes):
    try:
        import torch

        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


_torch_alloc_c = _ALLOC_FN(_torch_alloc)
_torch_free_c = _FREE_FN(_torch_free)
_live_ops = None  # weak set of live handles, destroyed at exit before torch shuts down

_lib = None


class KcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (msg, _status_name(status)))
        self.status = status


class KcSolveOpts(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int),
        ("guard", ctypes.c_int),
        ("tol", ctypes.c_double),
        ("maxit", ctypes.c_int),
        ("prec", ctypes.c_int),
        ("switch_tol", ctypes.c_double),
        ("batch_k", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("verbose", ctypes.c_int),
        ("precond", ctypes.c_int),
        ("graph", ctypes.c_int),
        ("x_init", ctypes.c_void_p),
        ("start", ctypes.c_int),
    ]


def lib():
    """The loaded library; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            raise KcError(-1, "libkcpc.so is not built (run python -m paper_2511_17107_amd.build)")
        # PyTorch ships its own HIP runtime with the same soname as the system one; loading torch
        # first makes the library bind to that single runtime, so device pointers and streams
        # from torch are valid in the library.
        import torch  # noqa: F401

        L = ctypes.CDLL(lib_path)
        vp, i32, dp = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
        L.kc_supported_n.argtypes = [i32]
        L.kc_create.argtypes = [i32, vp, i32, i32, vp, i32, vp, _ALLOC_FN, _FREE_FN, vp, vp, ctypes.POINTER(vp)]
        L.kc_op_flags.argtypes = [vp, vp]
        L.kc_set_kpoints.argtypes = [vp, i32, vp, vp]
        L.kc_get_gamma.argtypes = [vp, vp]
        L.kc_kpoint_flags.argtypes = [vp, vp]
        L.kc_spurious_bound.argtypes = [vp, vp]
        L.kc_to_real_space.argtypes = [vp, i32, vp, vp, vp]
        L.kc_to_kspace.argtypes = [vp, i32, vp, vp, vp]
        L.kc_apply.argtypes = [vp, i32, i32, i32, vp, vp, i32, vp]
        L.kc_precond.argtypes = [vp, i32, i32, i32, vp, vp, vp]
        L.kc_apply_timed.argtypes = [vp, i32, i32, i32, vp, vp, i32, vp, vp, vp]
        L.kc_fft3d.argtypes = [i32, i32, i32, i32, vp, vp, vp]
        L.kc_precond_transverse.argtypes = [vp, i32, i32, i32, vp, vp, vp, i32, vp]
        L.kc_tp_grad.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp]
        L.kc_solve_opts_default.argtypes = [ctypes.POINTER(KcSolveOpts)]
        L.kc_solve_opts_default.restype = None
        L.kc_solve.argtypes = [vp, i32, i32, ctypes.POINTER(KcSolveOpts), vp, vp, vp, vp, vp]
        L.kc_last_solve_stats.argtypes = [vp, vp]
        L.kc_last_residual_history.argtypes = [vp, i32, vp, vp, i32, vp]
        L.kc_tile_widths.argtypes = [vp, i32, vp]
        L.kc_release_workspaces.argtypes = [vp]
        L.kc_destroy.argtypes = [vp]
        L.kc_destroy.restype = None
        L.kc_net_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(vp)]
        L.kc_net_param_count.argtypes = []
        L.kc_net_param_count.restype = ctypes.c_size_t
        L.kc_net_get_params.argtypes = [vp, vp, ctypes.c_size_t]
        L.kc_net_set_params.argtypes = [vp, vp, ctypes.c_size_t]
        L.kc_net_forward.argtypes = [vp, i32, i32, vp, vp, vp]
        L.kc_net_gradients.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
        L.kc_net_backward.argtypes = [vp, i32, i32, vp, vp, vp, vp]
        L.kc_net_adam_step.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, vp]
        L.kc_net_destroy.argtypes = [vp]
        L.kc_net_destroy.restype = None
        L.kc_attach_net.argtypes = [vp, vp]
        L.kc_net_features.argtypes = [vp, i32, i32, vp, vp]
        L.kc_net_efield.argtypes = [vp, i32, i32, vp, vp]
        L.kc_precond_learned.argtypes = [vp, i32, i32, i32, vp, vp, i32, vp]
        L.kc_pcg.argtypes = [vp, i32, i32, vp, vp, ctypes.c_double, i32, ctypes.POINTER(i32), vp]
        L.kc_perturbed_residuals.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, vp]
        L.kc_net_loss_grad.argtypes = [vp, i32, i32, vp, vp, i32, ctypes.c_double, dp, vp, vp]
        L.kc_block_work_bytes.argtypes = [i32, ctypes.c_size_t, i32]
        L.kc_block_work_bytes.restype = ctypes.c_size_t
        L.kc_block_gram.argtypes = [i32, ctypes.c_size_t, i32, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.kc_block_gram_noalloc.argtypes = [i32, ctypes.c_size_t, i32, vp, vp, vp, vp, vp]
        L.kc_block_update.argtypes = [i32, ctypes.c_size_t, i32, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.kc_status_string.argtypes = [i32]
        L.kc_status_string.restype = ctypes.c_char_p
        L.kc_last_error.argtypes = []
        L.kc_last_error.restype = ctypes.c_char_p
        _ = dp
        _lib = L
        import atexit
        import weakref

        global _live_ops
        _live_ops = weakref.WeakSet()
        atexit.register(_destroy_live_ops)
    return _lib


def _destroy_live_ops():
    """Release every live handle while torch (whose allocator backs their memory) is still up."""
    for op in list(_live_ops or ()):
        op.close()


def _status_name(st: int) -> str:
    if _lib is None or st < 0:
        return "KC_ERR"
    return _lib.kc_status_string(st).decode()


def _check(st: int, what: str):
    if st != KC_OK:
        raise KcError(st, "%s failed: %s" % (what, lib().kc_last_error().decode()))


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _numel(t, n: int, what: str):
    """The library touches exactly n elements of t: anything else is refused here (the C ABI takes
    raw pointers and cannot check)."""
    if int(t.numel()) != int(n):
        raise ValueError("%s must hold %d elements, got %d (shape %s)" % (what, n, t.numel(), tuple(t.shape)))


def _dev_ptr(t, dtype_name: str, what: str):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) torch tensor" % what)
    if str(t.dtype) != dtype_name:
        raise TypeError("%s must have dtype %s, got %s" % (what, dtype_name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    return ctypes.c_void_p(t.data_ptr())


def kc_supported_n(N: int) -> bool:
    return bool(lib().kc_supported_n(int(N)))


def kc_fft3d(x, sign: int, prec: int = KC_PREC_FP64, out=None, stream=None):
    """Unnormalised 3D DFT of x (complex128 for FP64, complex64 for FP32), shape (nvec, N^3)
    or (nvec, N, N, N); out may be x."""
    import torch

    N = int(round(x.shape[-1] ** (1.0 / 3.0))) if x.dim() == 2 else int(x.shape[-1])
    nvec = int(x.shape[0])
    dt = "torch.complex128" if prec == KC_PREC_FP64 else "torch.complex64"
    _numel(x, nvec * N ** 3, "x")
    if out is None:
        out = torch.empty_like(x)
    _numel(out, nvec * N ** 3, "out")
    _check(lib().kc_fft3d(N, nvec, int(sign), int(prec), _dev_ptr(x, dt, "x"), _dev_ptr(out, dt, "out"),
                          _stream(stream)), "kc_fft3d")
    return out


def block_work_bytes(nb: int, n: int, nc: int) -> int:
    """Device workspace bytes of kc_block_gram / kc_block_update."""
    return int(lib().kc_block_work_bytes(int(nb), int(n), int(nc)))


def _block_shape(S, what: str):
    if S.dim() != 3:
        raise ValueError("%s must have shape (nb, nc, n)" % what)
    return int(S.shape[0]), int(S.shape[1]), int(S.shape[2])


def _work(nb, n, nc, work):
    import torch

    need = block_work_bytes(nb, n, nc)
    if work is None:
        work = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    elif work.numel() < need:
        raise ValueError("work holds %d bytes, %d needed" % (work.numel(), need))
    return work


def block_gram(S, AS, GA=None, GB=None, work=None, stream=None):
    """GA_b = S_b^H AS_b, GB_b = S_b^H S_b for blocks of shape (nb, nc, n), complex128."""
    import torch

    nb, nc, n = _block_shape(S, "S")
    if tuple(AS.shape) != (nb, nc, n):
        raise ValueError("AS must have the shape of S")
    if GA is None:
        GA = torch.empty((nb, nc, nc), dtype=torch.complex128, device=S.device)
    if GB is None:
        GB = torch.empty((nb, nc, nc), dtype=torch.complex128, device=S.device)
    work = _work(nb, n, nc, work)
    _check(lib().kc_block_gram(nb, n, nc, _dev_ptr(S, "torch.complex128", "S"),
                               _dev_ptr(AS, "torch.complex128", "AS"), _dev_ptr(GA, "torch.complex128", "GA"),
                               _dev_ptr(GB, "torch.complex128", "GB"), ctypes.c_void_p(work.data_ptr()),
                               work.numel(), _stream(stream)), "kc_block_gram")
    return GA, GB


def block_gram_noalloc(S, AS, GA, GB, stream=None):
    """kc_block_gram_noalloc: GA_b = S_b^H AS_b, GB_b = S_b^H S_b for blocks (nb, nc, n),
    complex128, into caller-provided GA, GB (nb, nc, nc); the library allocates nothing."""
    nb, nc, n = _block_shape(S, "S")
    if tuple(AS.shape) != (nb, nc, n):
        raise ValueError("AS must have the shape of S")
    _numel(GA, nb * nc * nc, "GA")
    _numel(GB, nb * nc * nc, "GB")
    _check(lib().kc_block_gram_noalloc(nb, n, nc, _dev_ptr(S, "torch.complex128", "S"),
                                       _dev_ptr(AS, "torch.complex128", "AS"), _dev_ptr(GA, "torch.complex128", "GA"),
                                       _dev_ptr(GB, "torch.complex128", "GB"), _stream(stream)),
           "kc_block_gram_noalloc")
    return GA, GB


def block_update(S, AS, C, theta, R=None, res=None, xnorm2=None, work=None, stream=None):
    """In place: [X P] <- S [C1 Cp], [AX AP] <- AS [C1 Cp] for blocks (nb, 3mb, n) and C (nb, 3mb,
    2mb); returns R (nb, mb, n) = AX - theta X, res = |R_j|/|X_j| and |X_j|^2 (nb, mb)."""
    import torch

    nb, nc, n = _block_shape(S, "S")
    if nc % 3 != 0:
        raise ValueError("S must hold 3mb columns per k-point")
    mb = nc // 3
    if tuple(AS.shape) != (nb, nc, n) or tuple(C.shape) != (nb, nc, 2 * mb) or tuple(theta.shape) != (nb, mb):
        raise ValueError("shapes: AS (nb, 3mb, n), C (nb, 3mb, 2mb), theta (nb, mb)")
    if R is None:
        R = torch.empty((nb, mb, n), dtype=torch.complex128, device=S.device)
    if res is None:
        res = torch.empty((nb, mb), dtype=torch.float64, device=S.device)
    if xnorm2 is None:
        xnorm2 = torch.empty((nb, mb), dtype=torch.float64, device=S.device)
    work = _work(nb, n, nc, work)
    _check(lib().kc_block_update(nb, n, mb, _dev_ptr(S, "torch.complex128", "S"),
                                 _dev_ptr(AS, "torch.complex128", "AS"), _dev_ptr(C, "torch.complex128", "C"),
                                 _dev_ptr(theta, "torch.float64", "theta"), _dev_ptr(R, "torch.complex128", "R"),
                                 _dev_ptr(res, "torch.float64", "res"), _dev_ptr(xnorm2, "torch.float64", "xnorm2"),
                                 ctypes.c_void_p(work.data_ptr()), work.numel(), _stream(stream)),
           "kc_block_update")
    return R, res, xnorm2


class Op:
    """Handle of one operator (grid, inverse-permittivity field, k-points).

    lattice: None (simple cubic) or (3, 3) primitive lattice vectors as rows (Section 2.2); ids and
    table then describe the unit-cube grid of fractional coordinates; stencil_m: order 2m of the
    curl/divergence stencils (1..5); allocator: "torch" (PyTorch's caching allocator backs the
    handle's device workspaces) or "hip" (the library's hipMalloc)."""

    def __init__(self, N: int, scheme: int, ids: np.ndarray, table: np.ndarray, lattice=None,
                 stencil_m: int = 1, allocator: str = "torch", stream=None):
        ids = np.ascontiguousarray(ids, dtype=np.uint8)
        if ids.shape != (4, N ** 3):
            raise ValueError("ids must have shape (4, N^3), got %s" % (ids.shape,))
        tab = np.ascontiguousarray(np.asarray(table, dtype=np.complex128))
        if tab.ndim != 3 or tab.shape[1:] != (3, 3):
            raise ValueError("table must have shape (n_mat, 3, 3)")
        tab_r = np.ascontiguousarray(tab.view(np.float64).reshape(tab.shape[0], 3, 3, 2))
        lat = None
        if lattice is not None:
            lat = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(3, 3))
        if allocator not in ("torch", "hip"):
            raise ValueError("allocator must be 'torch' or 'hip'")
        L = lib()
        al, fr = (_torch_alloc_c, _torch_free_c) if allocator == "torch" else (_ALLOC_FN(), _FREE_FN())
        h = ctypes.c_void_p()
        _check(L.kc_create(int(N), None if lat is None else lat.ctypes.data_as(ctypes.c_void_p), int(stencil_m),
                           int(scheme), ids.ctypes.data_as(ctypes.c_void_p), int(tab.shape[0]),
                           tab_r.ctypes.data_as(ctypes.c_void_p), al, fr, None,
                           None if stream is None else _stream(stream),
                           ctypes.byref(h)), "kc_create")
        self._h = h
        self.N = int(N)
        self.nk = 0
        self.stencil_m = int(stencil_m)
        _live_ops.add(self)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.kc_destroy(h)
        self._h = None

    def __del__(self):
        self.close()

    def release_workspaces(self):
        """Free the solver blocks and operator intermediates (allocated again when needed)."""
        _check(lib().kc_release_workspaces(self._h), "kc_release_workspaces")

    @property
    def n3(self) -> int:
        return self.N ** 3

    def flags(self) -> int:
        f = ctypes.c_int(0)
        _check(lib().kc_op_flags(self._h, ctypes.byref(f)), "kc_op_flags")
        return int(f.value)

    def kpoint_flags(self) -> np.ndarray:
        f = np.zeros(self.nk, dtype=np.int32)
        _check(lib().kc_kpoint_flags(self._h, f.ctypes.data_as(ctypes.c_void_p)), "kc_kpoint_flags")
        return f

    def spurious_bound(self) -> np.ndarray:
        b = np.zeros(self.nk)
        _check(lib().kc_spurious_bound(self._h, b.ctypes.data_as(ctypes.c_void_p)), "kc_spurious_bound")
        return b

    def _vpk(self, nvec: int, vecs_per_k: Optional[int]) -> int:
        vpk = nvec if vecs_per_k is None else int(vecs_per_k)
        return max(vpk, 1)

    def to_real_space(self, x, out=None, stream=None):
        """H = F3 x (face fields) for x complex128 (nvec, 3, N^3) on the GPU; out may be x."""
        import torch

        nvec = int(x.shape[0])
        _numel(x, nvec * 3 * self.n3, "x")
        if out is None:
            out = torch.empty_like(x)
        _numel(out, nvec * 3 * self.n3, "H")
        _check(lib().kc_to_real_space(self._h, nvec, _dev_ptr(x, "torch.complex128", "x"),
                                      _dev_ptr(out, "torch.complex128", "H"), _stream(stream)), "kc_to_real_space")
        return out

    def to_kspace(self, H, out=None, stream=None):
        """x = F3^H H for face fields H complex128 (nvec, 3, N^3) on the GPU; out may be H."""
        import torch

        nvec = int(H.shape[0])
        _numel(H, nvec * 3 * self.n3, "H")
        if out is None:
            out = torch.empty_like(H)
        _numel(out, nvec * 3 * self.n3, "x")
        _check(lib().kc_to_kspace(self._h, nvec, _dev_ptr(H, "torch.complex128", "H"),
                                  _dev_ptr(out, "torch.complex128", "x"), _stream(stream)), "kc_to_kspace")
        return out

    def set_kpoints(self, k: np.ndarray, gamma: Optional[np.ndarray] = None):
        k = np.ascontiguousarray(np.asarray(k, dtype=np.float64).reshape(-1, 3))
        g = None if gamma is None else np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(-1))
        _check(lib().kc_set_kpoints(self._h, int(k.shape[0]), k.ctypes.data_as(ctypes.c_void_p),
                                    None if g is None else g.ctypes.data_as(ctypes.c_void_p)), "kc_set_kpoints")
        self.nk = int(k.shape[0])

    def gamma(self) -> np.ndarray:
        g = np.zeros(self.nk)
        _check(lib().kc_get_gamma(self._h, g.ctypes.data_as(ctypes.c_void_p)), "kc_get_gamma")
        return g

    def apply(self, x, ik0: int = 0, vecs_per_k: Optional[int] = None, prec: int = KC_PREC_FP64,
              out=None, stream=None):
        """y = Op x; x complex128 (nvec, 3, N^3) on the GPU."""
        import torch

        nvec = int(x.shape[0])
        _numel(x, nvec * 3 * self.n3, "x")
        if out is None:
            out = torch.empty_like(x)
        _numel(out, nvec * 3 * self.n3, "y")
        vpk = self._vpk(nvec, vecs_per_k)
        _check(lib().kc_apply(self._h, int(ik0), int(nvec), max(vpk, 1), _dev_ptr(x, "torch.complex128", "x"),
                              _dev_ptr(out, "torch.complex128", "y"), int(prec), _stream(stream)), "kc_apply")
        return out

    def apply_timed(self, x, ik0: int = 0, vecs_per_k: Optional[int] = None, prec: int = KC_PREC_FP64,
                    out=None, stream=None):
        """kc_apply with per-pass HIP-event timings; returns (y, pass_ms)."""
        import torch

        nvec = int(x.shape[0])
        _numel(x, nvec * 3 * self.n3, "x")
        if out is None:
            out = torch.empty_like(x)
        _numel(out, nvec * 3 * self.n3, "y")
        vpk = self._vpk(nvec, vecs_per_k)
        ms = np.zeros(6)
        npass = ctypes.c_int(0)
        _check(lib().kc_apply_timed(self._h, int(ik0), int(nvec), max(vpk, 1),
                                    _dev_ptr(x, "torch.complex128", "x"), _dev_ptr(out, "torch.complex128", "y"),
                                    int(prec), _stream(stream), ms.ctypes.data_as(ctypes.c_void_p),
                                    ctypes.byref(npass)), "kc_apply_timed")
        return out, ms[: npass.value]

    def precond(self, r, ik0: int = 0, vecs_per_k: Optional[int] = None, out=None, stream=None):
        import torch

        nvec = int(r.shape[0])
        _numel(r, nvec * 3 * self.n3, "r")
        if out is None:
            out = torch.empty_like(r)
        _numel(out, nvec * 3 * self.n3, "z")
        vpk = self._vpk(nvec, vecs_per_k)
        _check(lib().kc_precond(self._h, int(ik0), int(nvec), max(vpk, 1), _dev_ptr(r, "torch.complex128", "r"),
                                _dev_ptr(out, "torch.complex128", "z"), _stream(stream)), "kc_precond")
        return out

    def precond_transverse(self, r, ik0: int = 0, vecs_per_k: Optional[int] = None, efield=None,
                           prec: int = KC_PREC_FP64, out=None, stream=None):
        """z = T_E r; efield None (E_c = 1/(eps^-1)_cc) or float32 [nk_used][3][N^3]."""
        import torch

        nvec = int(r.shape[0])
        _numel(r, nvec * 3 * self.n3, "r")
        if out is None:
            out = torch.empty_like(r)
        _numel(out, nvec * 3 * self.n3, "z")
        vpk = self._vpk(nvec, vecs_per_k)
        if efield is not None:
            _numel(efield, ((nvec - 1) // vpk + 1) * 3 * self.n3, "efield")
        ef = None if efield is None else _dev_ptr(efield, "torch.float32", "efield")
        _check(lib().kc_precond_transverse(self._h, int(ik0), int(nvec), max(vpk, 1),
                                           _dev_ptr(r, "torch.complex128", "r"), _dev_ptr(out, "torch.complex128", "z"),
                                           ef, int(prec), _stream(stream)), "kc_precond_transverse")
        return out

    def tp_grad(self, r, e, w, g, ik0: int = 0, vecs_per_k: Optional[int] = None, stream=None):
        """g (float32 [nvec/vpk][3][N^3]) += d/dE sum_j w_j Re<e_j, T_E r_j> (w float64 [nvec])."""
        nvec = int(r.shape[0])
        vpk = self._vpk(nvec, vecs_per_k)
        if nvec % vpk != 0:
            raise ValueError("nvec must be a multiple of vecs_per_k")
        _numel(r, nvec * 3 * self.n3, "r")
        _numel(e, nvec * 3 * self.n3, "e")
        _numel(w, nvec, "w")
        _numel(g, (nvec // vpk) * 3 * self.n3, "g")
        _check(lib().kc_tp_grad(self._h, int(ik0), int(nvec), max(vpk, 1), _dev_ptr(r, "torch.complex128", "r"),
                                _dev_ptr(e, "torch.complex128", "e"), _dev_ptr(w, "torch.float64", "w"),
                                _dev_ptr(g, "torch.float32", "g"), _stream(stream)), "kc_tp_grad")
        return g

    def solve(self, m: int, ik0: int = 0, nk: Optional[int] = None, tol: float = 1e-8, maxit: int = 500,
              prec: int = KC_PREC_FP64, switch_tol: float = 1e-3, batch_k: int = 1, guard: int = 0,
              seed: int = 1234, X_out=None, verbose: int = 0, stream=None, check: bool = True,
              precond: int = KC_PRECOND_DIAG, graph: bool = True, x_init=None, start: str = "random"):
        """Smallest positive eigenvalues for k-points ik0 .. ik0+nk-1 (x_init: optional start
        vectors, complex128 (nk, m, 3, N^3) on the device; otherwise start = "random" or
        "plane_waves").  Returns (eig (nk, m), res (nk, m), iters (nk,), status)."""
        nk = self.nk - ik0 if nk is None else int(nk)
        o = KcSolveOpts()
        lib().kc_solve_opts_default(ctypes.byref(o))
        o.m, o.guard, o.tol, o.maxit, o.prec = int(m), int(guard), float(tol), int(maxit), int(prec)
        o.switch_tol, o.batch_k, o.seed, o.verbose = float(switch_tol), int(batch_k), int(seed), int(verbose)
        o.precond = int(precond)
        o.graph = 1 if graph else 0
        if start not in ("random", "plane_waves"):
            raise ValueError("start: 'random' or 'plane_waves'")
        o.start = KC_START_PLANE_WAVES if start == "plane_waves" else KC_START_RANDOM
        if x_init is not None:
            if tuple(x_init.shape[:2]) != (nk, m):
                raise ValueError("x_init must hold (nk, m) start vectors")
            _numel(x_init, nk * m * 3 * self.n3, "x_init")
            o.x_init = _dev_ptr(x_init, "torch.complex128", "x_init")
        if X_out is not None:
            _numel(X_out, nk * m * 3 * self.n3, "X_out")
        eig = np.zeros((nk, m))
        res = np.zeros((nk, m))
        its = np.zeros(nk, dtype=np.int32)
        xo = None if X_out is None else _dev_ptr(X_out, "torch.complex128", "X_out")
        st = lib().kc_solve(self._h, int(ik0), nk, ctypes.byref(o), eig.ctypes.data_as(ctypes.c_void_p),
                            res.ctypes.data_as(ctypes.c_void_p), its.ctypes.data_as(ctypes.c_void_p), xo,
                            _stream(stream))
        if check and st not in (KC_OK, KC_ERR_NO_CONVERGENCE):
            _check(st, "kc_solve")
        return eig, res, its, st

    def tile_widths(self, prec: int = KC_PREC_FP32) -> np.ndarray:
        w = np.zeros(10, dtype=np.int32)
        _check(lib().kc_tile_widths(self._h, int(prec), w.ctypes.data_as(ctypes.c_void_p)), "kc_tile_widths")
        return w

    def residual_history(self, k: int = 0):
        """(max Res_j per iteration, precision per iteration) of k-point k of the last solve."""
        cnt = ctypes.c_int(0)
        _check(lib().kc_last_residual_history(self._h, int(k), None, None, 0, ctypes.byref(cnt)),
               "kc_last_residual_history")
        r = np.zeros(cnt.value)
        p = np.zeros(cnt.value, dtype=np.int32)
        _check(lib().kc_last_residual_history(self._h, int(k), r.ctypes.data_as(ctypes.c_void_p),
                                              p.ctypes.data_as(ctypes.c_void_p), cnt.value, ctypes.byref(cnt)),
               "kc_last_residual_history")
        return r, p

    def last_solve_stats(self) -> np.ndarray:
        s = np.zeros(8)
        _check(lib().kc_last_solve_stats(self._h, s.ctypes.data_as(ctypes.c_void_p)), "kc_last_solve_stats")
        return s


    def attach_net(self, net: Optional["Net"]):
        _check(lib().kc_attach_net(self._h, None if net is None else net._h), "kc_attach_net")
        self._net = net  # keep the network alive while attached

    def net_features(self, ik0: int = 0, nk: int = 1, out=None, stream=None):
        """Network input (bf16 [nk][N^3][32]) of k-points ik0 .. ik0+nk-1."""
        import torch

        if out is None:
            out = torch.empty((nk, self.N ** 3, 32), dtype=torch.bfloat16, device=torch.device("cuda"))
        _numel(out, nk * self.n3 * 32, "feat")
        _check(lib().kc_net_features(self._h, int(ik0), int(nk), _dev_ptr(out, "torch.bfloat16", "feat"),
                                     _stream(stream)), "kc_net_features")
        return out

    def net_efield(self, ik0: int = 0, nk: int = 1, out=None, stream=None):
        """Learned field (float32 [nk][3][N^3]) of k-points ik0 .. ik0+nk-1."""
        import torch

        if out is None:
            out = torch.empty((nk, 3, self.N ** 3), dtype=torch.float32, device=torch.device("cuda"))
        _numel(out, nk * 3 * self.n3, "efield")
        _check(lib().kc_net_efield(self._h, int(ik0), int(nk), _dev_ptr(out, "torch.float32", "efield"),
                                   _stream(stream)), "kc_net_efield")
        return out

    def pcg(self, r, ik: int = 0, tol: float = 1e-7, maxit: int = 400, out=None, stream=None):
        """kc_pcg: c = Op^{-1} r (block r complex128 [nvec][3][N^3] of k-point ik).  Returns
        (c, iterations, converged)."""
        import torch

        nvec = int(r.shape[0])
        _numel(r, nvec * 3 * self.n3, "r")
        if out is None:
            out = torch.empty_like(r)
        _numel(out, nvec * 3 * self.n3, "c")
        its = ctypes.c_int(0)
        st = lib().kc_pcg(self._h, int(ik), nvec, _dev_ptr(r, "torch.complex128", "r"),
                          _dev_ptr(out, "torch.complex128", "c"), float(tol), int(maxit), ctypes.byref(its),
                          _stream(stream))
        if st not in (KC_OK, KC_ERR_NO_CONVERGENCE):
            _check(st, "kc_pcg")
        return out, its.value, st == KC_OK

    def perturbed_residuals(self, X, noise, amp, ik: int = 0, x_out=None, r_out=None, stream=None):
        """kc_perturbed_residuals: (x, r) for orthonormal X and noise (complex128 [m][3][N^3])
        and amplitudes amp (m host values)."""
        import torch

        m = int(X.shape[0])
        _numel(X, m * 3 * self.n3, "X")
        _numel(noise, m * 3 * self.n3, "noise")
        a = np.ascontiguousarray(np.asarray(amp, dtype=np.float64).reshape(-1))
        if a.size != m:
            raise ValueError("amp needs one value per vector")
        x = torch.empty_like(X) if x_out is None else x_out
        r = torch.empty_like(X) if r_out is None else r_out
        _numel(x, m * 3 * self.n3, "x")
        _numel(r, m * 3 * self.n3, "r")
        _check(lib().kc_perturbed_residuals(self._h, int(ik), m, _dev_ptr(X, "torch.complex128", "X"),
                                            _dev_ptr(noise, "torch.complex128", "noise"),
                                            a.ctypes.data_as(ctypes.c_void_p), _dev_ptr(x, "torch.complex128", "x"),
                                            _dev_ptr(r, "torch.complex128", "r"), _stream(stream)),
               "kc_perturbed_residuals")
        return x, r

    def net_loss_grad(self, r, c, ik: int = 0, kind: str = "energy", grad: bool = False, scale: float = 1.0,
                      out=None, stream=None):
        """kc_net_loss_grad: mean misfit of T_E r (the attached network's field) against c; with
        grad, also scale * d(mean)/d(network output) (float32 [N^3][16]).  Returns (loss, gout)."""
        import torch

        nvec = int(r.shape[0])
        _numel(r, nvec * 3 * self.n3, "r")
        _numel(c, nvec * 3 * self.n3, "c")
        if kind not in ("energy", "euclidean"):
            raise ValueError("kind: 'energy' or 'euclidean'")
        gptr = None
        if grad:
            if out is None:
                out = torch.empty((self.n3, 16), dtype=torch.float32, device=r.device)
            _numel(out, self.n3 * 16, "gout")
            gptr = _dev_ptr(out, "torch.float32", "gout")
        loss = ctypes.c_double(0.0)
        _check(lib().kc_net_loss_grad(self._h, int(ik), nvec, _dev_ptr(r, "torch.complex128", "r"),
                                      _dev_ptr(c, "torch.complex128", "c"), 0 if kind == "energy" else 1,
                                      float(scale), ctypes.byref(loss), gptr, _stream(stream)), "kc_net_loss_grad")
        return loss.value, (out if grad else None)

    def precond_learned(self, r, ik0: int = 0, vecs_per_k: Optional[int] = None, prec: int = KC_PREC_FP64,
                        out=None, stream=None):
        import torch

        nvec = int(r.shape[0])
        _numel(r, nvec * 3 * self.n3, "r")
        if out is None:
            out = torch.empty_like(r)
        _numel(out, nvec * 3 * self.n3, "z")
        vpk = self._vpk(nvec, vecs_per_k)
        _check(lib().kc_precond_learned(self._h, int(ik0), int(nvec), max(vpk, 1),
                                        _dev_ptr(r, "torch.complex128", "r"), _dev_ptr(out, "torch.complex128", "z"),
                                        int(prec), _stream(stream)), "kc_precond_learned")
        return out


class Net:
    """Learned preconditioner network (kc_net)."""

    def __init__(self, seed: int = 0):
        h = ctypes.c_void_p()
        _check(lib().kc_net_create(ctypes.c_uint64(int(seed)), ctypes.byref(h)), "kc_net_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.kc_net_destroy(h)
            self._h = None

    @staticmethod
    def param_count() -> int:
        return int(lib().kc_net_param_count())

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.param_count(), dtype=np.float32)
        _check(lib().kc_net_get_params(self._h, p.ctypes.data_as(ctypes.c_void_p), p.size), "kc_net_get_params")
        return p

    def set_params(self, p: np.ndarray):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.param_count()
        _check(lib().kc_net_set_params(self._h, p.ctypes.data_as(ctypes.c_void_p), p.size), "kc_net_set_params")

    def forward(self, x, N: int, out=None, stream=None):
        """x: bf16 [batch][N^3][32] -> float32 [batch][N^3][16]."""
        import torch

        batch = int(x.shape[0])
        _numel(x, batch * N ** 3 * 32, "x")
        if out is None:
            out = torch.empty((batch, N ** 3, 16), dtype=torch.float32, device=x.device)
        _numel(out, batch * N ** 3 * 16, "out")
        _check(lib().kc_net_forward(self._h, int(N), int(batch), _dev_ptr(x, "torch.bfloat16", "x"),
                                    _dev_ptr(out, "torch.float32", "out"), _stream(stream)), "kc_net_forward")
        return out

    def gradients(self, x, target, N: int, host_grads: bool = True, stream=None):
        """MSE loss and parameter gradients (numpy float32, or None with host_grads=False)."""
        batch = int(x.shape[0])
        _numel(x, batch * N ** 3 * 32, "x")
        _numel(target, batch * N ** 3 * 16, "target")
        loss = ctypes.c_double(0.0)
        g = np.zeros(self.param_count(), dtype=np.float32) if host_grads else None
        _check(lib().kc_net_gradients(self._h, int(N), int(batch), _dev_ptr(x, "torch.bfloat16", "x"),
                                      _dev_ptr(target, "torch.float32", "target"), ctypes.byref(loss),
                                      None if g is None else g.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
               "kc_net_gradients")
        return loss.value, g

    def backward(self, x, gout, N: int, host_grads: bool = True, stream=None):
        """Parameter gradients for the output gradient gout (float32 [batch][N^3][16])."""
        batch = int(x.shape[0])
        _numel(x, batch * N ** 3 * 32, "x")
        _numel(gout, batch * N ** 3 * 16, "gout")
        g = np.zeros(self.param_count(), dtype=np.float32) if host_grads else None
        _check(lib().kc_net_backward(self._h, int(N), int(batch), _dev_ptr(x, "torch.bfloat16", "x"),
                                     _dev_ptr(gout, "torch.float32", "gout"),
                                     None if g is None else g.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
               "kc_net_backward")
        return g

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
        _check(lib().kc_net_adam_step(self._h, float(lr), float(beta1), float(beta2), float(eps), _stream(stream)),
               "kc_net_adam_step")


def kc_create(N: int, scheme: int, ids: np.ndarray, table: np.ndarray, **kw) -> Op:
    return Op(N, scheme, ids, table, **kw)
