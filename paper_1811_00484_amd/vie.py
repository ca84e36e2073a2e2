"""ctypes binding of libvie.so (argument marshalling only).

Every numerical step runs inside the HIP library; this module converts
torch tensors and numpy arrays to the plain pointers of the C ABI declared in
``include/vie.h`` and raises on negative status codes.  There is no fallback:
if the shared library is missing or fails to load, every call raises.

Tensor conventions: vectors are complex torch tensors of shape
(nrhs, 3, n3, n2, n1) (or (3, n3, n2, n1) for one right-hand side) on the
current HIP device, complex64 or complex128, contiguous; eps_c is
(n3, n2, n1) of the same dtype.  Work is enqueued on
``torch.cuda.current_stream()``.
"""
import ctypes
import os
import warnings

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# VIE_LIBRARY selects another build of the same library (e.g. one compiled
# with different launch shapes); the default is the in-tree build
LIB_PATH = os.environ.get("VIE_LIBRARY") or os.path.join(HERE, "libvie.so")

VIE_OK, VIE_NOT_CONVERGED = 0, 1
VIE_E_ARG, VIE_E_NOMEM, VIE_E_HIP, VIE_E_NONFINITE, VIE_E_UNSUPPORTED = -1, -2, -3, -4, -5
VIE_C64, VIE_C128 = 0, 1
VIE_RECON_AUTO, VIE_RECON_FP32, VIE_RECON_BF16, VIE_RECON_FP64 = 0, 1, 2, 3
VIE_OP_A, VIE_OP_N = 0, 1
VIE_NHAT_TUCKER, VIE_NHAT_DENSE = 0, 1

_RECON = {"auto": VIE_RECON_AUTO, "fp32": VIE_RECON_FP32, "bf16": VIE_RECON_BF16, "fp64": VIE_RECON_FP64}


class VieError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("vie status %d: %s" % (status, msg))
        self.status = status


class CompressOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("trunc_rule", ctypes.c_int), ("max_rank", ctypes.c_int)]


class CompressInfo(ctypes.Structure):
    _fields_ = [("ranks", (ctypes.c_int * 3) * 6), ("tail_bound", ctypes.c_double * 6),
                ("fro_norm", ctypes.c_double * 6), ("tucker_bytes_c64", ctypes.c_size_t),
                ("dense_bytes_c64", ctypes.c_size_t), ("device_bytes", ctypes.c_size_t),
                ("seconds", ctypes.c_double), ("cp", ctypes.c_int)]


class CrossOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("trunc_rule", ctypes.c_int), ("max_rank", ctypes.c_int),
                ("oversample", ctypes.c_int), ("max_sweeps", ctypes.c_int), ("n_sample", ctypes.c_int),
                ("seed", ctypes.c_ulonglong)]


class CrossInfo(ctypes.Structure):
    _fields_ = [("evals", ctypes.c_long * 6), ("evals_sample", ctypes.c_long * 6), ("sweeps", ctypes.c_int * 6),
                ("sample_rel_err", ctypes.c_double * 6), ("seconds", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_outer", ctypes.c_int),
                ("adjoint", ctypes.c_int), ("refine", ctypes.c_int), ("inner_recon", ctypes.c_int),
                ("inner_tol", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("matvecs", ctypes.c_int), ("matvecs_fp64", ctypes.c_int), ("restarts", ctypes.c_int),
                ("refine_steps", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("history", ctypes.POINTER(ctypes.c_double)),
                ("hist_cap", ctypes.c_int), ("hist_len", ctypes.c_int)]


class Instance(ctypes.Structure):
    _fields_ = [("op", ctypes.c_void_p), ("eps_c", ctypes.c_void_p), ("x", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("nrhs", ctypes.c_int)]


class SolveInstance(ctypes.Structure):
    _fields_ = [("op", ctypes.c_void_p), ("eps_c", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("nrhs", ctypes.c_int), ("info", ctypes.POINTER(SolveInfo))]


# exported symbols and their ctypes signatures (kept in step with include/vie.h)
_P = ctypes.c_void_p
_SIGS = {
    "vie_compress": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _P, ctypes.POINTER(CompressOpts),
                                    ctypes.POINTER(_P), ctypes.POINTER(CompressInfo)]),
    "vie_compress_cp": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _P, ctypes.POINTER(CompressOpts), ctypes.c_int,
                                       ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(CompressInfo), _P]),
    "vie_compress_k": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _P, ctypes.POINTER(CompressOpts),
                                      ctypes.POINTER(_P), ctypes.POINTER(CompressInfo)]),
    "vie_jm_workspace_bytes": (ctypes.c_size_t, [_P, _P, ctypes.c_int]),
    "vie_matvec_jm": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_double, _P, _P, _P, _P, _P,
                                     ctypes.c_size_t, _P]),
    "vie_solve_jm_workspace_bytes": (ctypes.c_size_t, [_P, _P, ctypes.c_int, ctypes.POINTER(SolveOpts)]),
    "vie_solve_jm": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_double, _P, _P, _P, _P,
                                    ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), _P, ctypes.c_size_t, _P]),
    "vie_jm_pwl_workspace_bytes": (ctypes.c_size_t, [_P, _P, ctypes.c_int]),
    "vie_matvec_jm_pwl": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_double, _P, _P, _P, _P, _P,
                                         ctypes.c_size_t, _P]),
    "vie_solve_jm_pwl_workspace_bytes": (ctypes.c_size_t, [_P, _P, ctypes.c_int, ctypes.POINTER(SolveOpts)]),
    "vie_solve_jm_pwl": (ctypes.c_int, [_P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_double, _P, _P, _P, _P,
                                        ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), _P, ctypes.c_size_t,
                                        _P]),
    "vie_magnetic_field": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_double, ctypes.c_double, _P, _P, _P]),
    "vie_compress_cross": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _P, _P, ctypes.POINTER(CrossOpts),
                                          ctypes.POINTER(_P), ctypes.POINTER(CompressInfo), ctypes.POINTER(CrossInfo)]),
    "vie_tucker_cross": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _P, _P, ctypes.c_int, ctypes.POINTER(CrossOpts),
                                        ctypes.POINTER(ctypes.c_int), _P, ctypes.c_size_t, _P, ctypes.c_size_t,
                                        ctypes.POINTER(CrossInfo)]),
    "vie_tucker_cross_pwl": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _P, _P, ctypes.c_int,
                                            ctypes.POINTER(CrossOpts), ctypes.POINTER(ctypes.c_int), _P, ctypes.c_size_t,
                                            _P, ctypes.c_size_t, ctypes.POINTER(CrossInfo)]),
    "vie_tucker_hadamard_ws_bytes": (ctypes.c_size_t, [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                                       ctypes.c_int, ctypes.c_int]),
    "vie_tucker_hadamard": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                           ctypes.c_int, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t, _P]),
    "vie_op_from_tucker": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int), _P, _P,
                                          ctypes.POINTER(_P), ctypes.POINTER(CompressInfo)]),
    "vie_compress_pwl": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _P, ctypes.POINTER(CompressOpts), ctypes.c_int,
                                        ctypes.c_int, ctypes.POINTER(_P), _P]),
    "vie_compress_pwl_k": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _P, ctypes.POINTER(CompressOpts),
                                          ctypes.POINTER(_P), _P]),
    "vie_pwl_op_destroy": (ctypes.c_int, [_P]),
    "vie_pwl_op_query": (ctypes.c_int, [_P, _P, _P]),
    "vie_pwl_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int, ctypes.c_int]),
    "vie_matvec_pwl": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P, ctypes.c_int, _P,
                                      ctypes.c_size_t, _P]),
    "vie_solve_pwl_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int, ctypes.POINTER(SolveOpts)]),
    "vie_solve_pwl": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, ctypes.POINTER(SolveOpts),
                                     ctypes.POINTER(SolveInfo), _P, ctypes.c_size_t, _P]),
    "vie_op_destroy": (ctypes.c_int, [_P]),
    "vie_op_query": (ctypes.c_int, [_P, _P, _P]),
    "vie_op_densify": (ctypes.c_int, [_P, ctypes.c_int]),
    "vie_op_set_nhat": (ctypes.c_int, [_P, ctypes.c_int]),
    "vie_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int, ctypes.c_int]),
    "vie_matvec": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P, ctypes.c_int, _P,
                                  ctypes.c_size_t, _P]),
    "vie_matvec_adjoint": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P, ctypes.c_int,
                                          _P, ctypes.c_size_t, _P]),
    "vie_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "vie_matvec_noalloc": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P,
                                          ctypes.c_int, _P]),
    "vie_solve_workspace_bytes": (ctypes.c_size_t, [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(SolveOpts)]),
    "vie_solve": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, ctypes.c_int, ctypes.POINTER(SolveOpts),
                                 ctypes.POINTER(SolveInfo), _P, ctypes.c_size_t, _P]),
    "vie_matvec_multi_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Instance), ctypes.c_int, ctypes.c_int]),
    "vie_matvec_multi": (ctypes.c_int, [ctypes.POINTER(Instance), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, _P, ctypes.c_size_t, _P]),
    "vie_solve_multi_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(SolveInstance), ctypes.c_int, ctypes.c_int,
                                                          ctypes.POINTER(SolveOpts)]),
    "vie_solve_multi": (ctypes.c_int, [ctypes.POINTER(SolveInstance), ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(SolveOpts), _P, ctypes.c_size_t, _P]),
    "vie_field_gradient": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_double, _P, _P, _P]),
    "vie_problem_setup": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, ctypes.c_double, _P, _P, _P]),
    "vie_total_field": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, ctypes.c_double, _P, _P]),
    "vie_adjoint_source": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P]),
    "vie_debug_nhat": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, ctypes.c_int, _P]),
    "vie_debug_pad": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int, _P]),
    "vie_debug_crop": (ctypes.c_int, [_P, ctypes.c_int, _P, _P, ctypes.c_int, _P]),
    "vie_debug_pass": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P,
                                      _P, _P, ctypes.c_int, _P]),
    "vie_debug_hosvd": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _P, ctypes.c_double, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int), _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "vie_debug_cp": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int), _P, ctypes.c_int, ctypes.c_int, _P,
                                    ctypes.POINTER(ctypes.c_double)]),
    "vie_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "vie_profile_collect": (ctypes.c_int, [_P, _P]),
    "vie_set_kernel_path": (ctypes.c_int, [ctypes.c_int]),
    "vie_set_batch_mode": (ctypes.c_int, [ctypes.c_int]),
    "vie_autotune": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, ctypes.c_size_t, _P, _P,
                                    ctypes.POINTER(ctypes.c_int)]),
    "vie_matvec_graph": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P, _P,
                                        ctypes.c_int, _P, ctypes.c_size_t, ctypes.POINTER(_P)]),
    "vie_graph_launch": (ctypes.c_int, [_P, _P]),
    "vie_graph_destroy": (ctypes.c_int, [_P]),
    "vie_last_error": (ctypes.c_char_p, []),
    "vie_version": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load libvie.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libvie.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status, what):
    if status < 0:
        msg = load().vie_last_error().decode(errors="replace")
        raise VieError(status, "%s: %s" % (what, msg))
    return status


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dt(t):
    if t.dtype == torch.complex64:
        return VIE_C64
    if t.dtype == torch.complex128:
        return VIE_C128
    raise TypeError("complex64 or complex128 expected, got %s" % t.dtype)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _require_like(t, ref, shape, name):
    """Check, before any library call, that ``t`` is a contiguous tensor of
    ``ref``'s dtype, on ``ref``'s device, of shape ``shape``: the kernels take
    the element size and extents from the vectors, so a mismatch would read
    or write outside the buffer."""
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor" % name)
    if t.dtype != ref.dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, ref.dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.device != ref.device:
        raise ValueError("%s must be on %s, got %s" % (name, ref.device, t.device))
    return t


def _require_device(t, name):
    if t.device.type != "cuda":
        raise ValueError("%s must be a device tensor (got %s)" % (name, t.device))
    return t


class Operator:
    """Device-resident Tucker-compressed Green's operator (owns a vie_op)."""

    def __init__(self, handle, n, info):
        self._h = handle
        self.n = tuple(n)
        self.ranks = [tuple(info.ranks[c][a] for a in range(3)) for c in range(6)]
        self.tail_bound = [info.tail_bound[c] for c in range(6)]
        self.fro_norm = [info.fro_norm[c] for c in range(6)]
        self.tucker_bytes_c64 = int(info.tucker_bytes_c64)
        self.dense_bytes_c64 = int(info.dense_bytes_c64)
        self.device_bytes = int(info.device_bytes)
        self.compress_seconds = float(info.seconds)
        self.cp = bool(info.cp)
        self._ws = {}

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("operator destroyed")
        return self._h

    def close(self):
        if self._h is not None:
            load().vie_op_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, nbytes, device):
        key = (device, nbytes)
        ws = self._ws.get(key)
        if ws is None:
            self._ws.clear()
            ws = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
            self._ws[key] = ws
        return ws


def compress(green, tol=1e-6, trunc_rule=0, max_rank=0):
    """HOSVD-compress the six defining tensors (numpy complex128,
    shape (6, n3, n2, n1)) and upload the operator to the current device."""
    lib = load()
    g = np.ascontiguousarray(green, dtype=np.complex128)
    if g.ndim != 4 or g.shape[0] != 6:
        raise ValueError("green must have shape (6, n3, n2, n1)")
    n = (ctypes.c_int * 3)(g.shape[3], g.shape[2], g.shape[1])
    opts = CompressOpts(float(tol), int(trunc_rule), int(max_rank))
    info = CompressInfo()
    h = ctypes.c_void_p()
    _check(lib.vie_compress(n, g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts), ctypes.byref(h),
                            ctypes.byref(info)), "vie_compress")
    return Operator(h, (g.shape[3], g.shape[2], g.shape[1]), info)


def compress_cp(green, tol=1e-6, cp_rank=0, cp_iters=0, trunc_rule=0, max_rank=0):
    """Tucker+CP compression (vie_compress_cp): HOSVD at ``tol``, then a CP of
    each core with ``cp_rank`` terms (0 = its smallest Tucker rank) by
    ``cp_iters`` ALS sweeps (0 = 1000).  The operator's ``cp_rel_err`` holds
    the six cores' relative CP fit errors."""
    lib = load()
    g = np.ascontiguousarray(green, dtype=np.complex128)
    if g.ndim != 4 or g.shape[0] != 6:
        raise ValueError("green must have shape (6, n3, n2, n1)")
    n = (ctypes.c_int * 3)(g.shape[3], g.shape[2], g.shape[1])
    opts = CompressOpts(float(tol), int(trunc_rule), int(max_rank))
    info = CompressInfo()
    err = np.zeros(6)
    h = ctypes.c_void_p()
    _check(lib.vie_compress_cp(n, g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts), int(cp_rank),
                               int(cp_iters), ctypes.byref(h), ctypes.byref(info), err.ctypes.data_as(ctypes.c_void_p)),
           "vie_compress_cp")
    op = Operator(h, (g.shape[3], g.shape[2], g.shape[1]), info)
    op.cp_rel_err = err
    return op


class PwlOperator:
    """Device-resident piecewise-linear operator (owns a vie_pwl_op): ten
    six-component Tucker (or Tucker+CP) blocks, one per basis pair (family
    'N'), or ten antisymmetric blocks of the magnetic operator (family 'K',
    ranks[:, 3:] the xy, xz, yz components)."""

    def __init__(self, handle, n, infos, family="N"):
        self._h = handle
        self.n = tuple(n)
        self.family = family
        self.ranks = np.array([[[info.ranks[c][a] for a in range(3)] for c in range(6)] for info in infos])
        self.tucker_bytes_c64 = int(sum(info.tucker_bytes_c64 for info in infos))
        self.device_bytes = int(sum(info.device_bytes for info in infos))
        self.compress_seconds = float(sum(info.seconds for info in infos))
        self._ws = {}

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("operator destroyed")
        return self._h

    def close(self):
        if self._h is not None:
            load().vie_pwl_op_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    workspace = Operator.workspace


def compress_pwl(green_pwl, tol=1e-6, cp_rank=-1, cp_iters=0, trunc_rule=0, max_rank=0):
    """Compress the sixty piecewise-linear defining tensors (numpy complex128,
    shape (10, 6, n3, n2, n1), pairs (0,0) (0,1) ... (3,3)) by HOSVD, or
    Tucker+CP when ``cp_rank`` >= 0, and upload them (vie_compress_pwl)."""
    lib = load()
    g = np.ascontiguousarray(green_pwl, dtype=np.complex128)
    if g.ndim != 5 or g.shape[:2] != (10, 6):
        raise ValueError("green_pwl must have shape (10, 6, n3, n2, n1)")
    n = (ctypes.c_int * 3)(g.shape[4], g.shape[3], g.shape[2])
    opts = CompressOpts(float(tol), int(trunc_rule), int(max_rank))
    infos = (CompressInfo * 10)()
    h = ctypes.c_void_p()
    _check(lib.vie_compress_pwl(n, g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts), int(cp_rank),
                                int(cp_iters), ctypes.byref(h), ctypes.cast(infos, ctypes.c_void_p)),
           "vie_compress_pwl")
    return PwlOperator(h, (g.shape[4], g.shape[3], g.shape[2]), list(infos))


def compress_pwl_k(green_pwl_k, tol=1e-6, trunc_rule=0, max_rank=0):
    """Compress the thirty piecewise-linear K tensors (numpy complex128, shape
    (10, 3, n3, n2, n1): pairs as compress_pwl, components xy, xz, yz) by
    HOSVD and upload them (vie_compress_pwl_k); apply with
    ``matvec_pwl(op, x, kind="N")``."""
    lib = load()
    g = np.ascontiguousarray(green_pwl_k, dtype=np.complex128)
    if g.ndim != 5 or g.shape[:2] != (10, 3):
        raise ValueError("green_pwl_k must have shape (10, 3, n3, n2, n1)")
    n = (ctypes.c_int * 3)(g.shape[4], g.shape[3], g.shape[2])
    opts = CompressOpts(float(tol), int(trunc_rule), int(max_rank))
    infos = (CompressInfo * 10)()
    h = ctypes.c_void_p()
    _check(lib.vie_compress_pwl_k(n, g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts), ctypes.byref(h),
                                  ctypes.cast(infos, ctypes.c_void_p)), "vie_compress_pwl_k")
    return PwlOperator(h, (g.shape[4], g.shape[3], g.shape[2]), list(infos), family="K")


def matvec_pwl(op, x, eps_c=None, kind="A", adjoint=False, out=None):
    """y = S A S x (kind 'A'), the bare sum S N S x (kind 'N'), or their
    adjoints, in the mass-normalised piecewise-linear basis (a K operator:
    S K S x, kind 'N' without adjoint only); x is
    (12, n3, n2, n1) = [l][q], or (nrhs, 12, n3, n2, n1) for several vectors
    with the same contrast, complex64 or complex128 on the device."""
    n1, n2, n3 = op.n
    dt = _dt(x)
    single = x.dim() == 4
    xb = x.unsqueeze(0) if single else x
    if xb.dim() != 5 or tuple(xb.shape[1:]) != (12, n3, n2, n1) or not xb.is_contiguous():
        raise ValueError("x must be a contiguous (12, %d, %d, %d) or (nrhs, 12, %d, %d, %d) tensor"
                         % (n3, n2, n1, n3, n2, n1))
    _require_device(xb, "x")
    k = VIE_OP_A if kind == "A" else VIE_OP_N
    if k == VIE_OP_A:
        if eps_c is None:
            raise ValueError("eps_c required for kind 'A'")
        _require_like(eps_c, xb, xb.shape[2:], "eps_c")
    y = torch.empty_like(xb) if out is None else _require_like(out, x, x.shape, "out")
    yb = y if out is None else (y.unsqueeze(0) if single else y)
    lib = load()
    nrhs = xb.shape[0]
    nbytes = lib.vie_pwl_workspace_bytes(op.handle, dt, nrhs)
    ws = op.workspace(nbytes, xb.device)
    _check(lib.vie_matvec_pwl(op.handle, k, 1 if adjoint else 0, dt, _ptr(eps_c) if k == VIE_OP_A else None,
                              _ptr(xb), _ptr(yb), nrhs, _ptr(ws), nbytes, _stream()), "vie_matvec_pwl")
    if out is not None:
        return out
    return y[0] if single else y


def solve_pwl(op, b, eps_c, tol=1e-6, restart=50, max_outer=200, adjoint=False, refine=False, inner_tol=1e-4,
              history=64):
    """GMRES for the piecewise-linear operator (vie_solve_pwl): b and the
    solution are (12, n3, n2, n1) in the mass-normalised basis.  ``refine``
    (complex128 only): FP32 products in the Arnoldi steps, FP64 restart
    residuals.  Returns (x, info dict, status)."""
    n1, n2, n3 = op.n
    if tuple(b.shape) != (12, n3, n2, n1) or not b.is_contiguous():
        raise ValueError("b must be contiguous (12, n3, n2, n1)")
    dt = _dt(b)
    _require_like(eps_c, b, (n3, n2, n1), "eps_c")
    _require_device(b, "b")
    lib = load()
    opts = SolveOpts(float(tol), int(restart), int(max_outer), int(bool(adjoint)), int(bool(refine)),
                     VIE_RECON_FP32, float(inner_tol))
    nbytes = lib.vie_solve_pwl_workspace_bytes(op.handle, dt, ctypes.byref(opts))
    if nbytes == 0:
        raise VieError(VIE_E_ARG, "vie_solve_pwl_workspace_bytes rejected the options")
    ws = _scratch(nbytes, b.device)
    x = torch.empty_like(b)
    hist = np.zeros(max(1, int(history)))
    info = SolveInfo()
    info.history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    info.hist_cap = int(history)
    st = lib.vie_solve_pwl(op.handle, dt, _ptr(eps_c), _ptr(b), _ptr(x), ctypes.byref(opts), ctypes.byref(info),
                           _ptr(ws), nbytes, _stream())
    _check(st, "vie_solve_pwl")
    d = {"matvecs": info.matvecs, "matvecs_fp64": info.matvecs_fp64, "restarts": info.restarts,
         "refine_steps": info.refine_steps, "converged": bool(info.converged),
         "rel_residual": info.rel_residual, "history": hist[:info.hist_len].tolist()}
    return x, d, st


def compress_k(green_k, tol=1e-6, trunc_rule=0, max_rank=0):
    """HOSVD-compress the three K defining tensors (numpy complex128, shape
    (3, n3, n2, n1), components xy, xz, yz) into a K operator on the current
    device (vie_compress_k).  ``op.k_ranks`` holds the Tucker ranks of xy,
    xz, yz.  Apply it with ``matvec(op, x, kind="N")``."""
    lib = load()
    g = np.ascontiguousarray(green_k, dtype=np.complex128)
    if g.ndim != 4 or g.shape[0] != 3:
        raise ValueError("green_k must have shape (3, n3, n2, n1)")
    n = (ctypes.c_int * 3)(g.shape[3], g.shape[2], g.shape[1])
    opts = CompressOpts(float(tol), int(trunc_rule), int(max_rank))
    info = CompressInfo()
    h = ctypes.c_void_p()
    _check(lib.vie_compress_k(n, g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts), ctypes.byref(h),
                              ctypes.byref(info)), "vie_compress_k")
    op = Operator(h, (g.shape[3], g.shape[2], g.shape[1]), info)
    op.k_ranks = op.ranks[3:]
    return op


def magnetic_field(op_k, j, h_inc, h):
    """H = h_inc + K j and |b1+| = mu0 |H_x + i H_y| (eq. 18) for a current
    ``j`` (3, n3, n2, n1) on the device; ``h`` is the voxel edge (m).  The K
    product runs in the library (vie_matvec, VIE_OP_N) and so does the field
    and b1+ kernel (vie_magnetic_field).  Returns (H, b1)."""
    _vec3(j, op_k, "j")
    _require_like(h_inc, j, j.shape, "h_inc")
    lib = load()
    kj = matvec(op_k, j, kind="N")
    H = torch.empty_like(kj)
    b1 = torch.empty(tuple(j.shape[1:]), dtype=torch.float64 if j.dtype == torch.complex128 else torch.float32,
                     device=j.device)
    _check(lib.vie_magnetic_field(op_k.handle, _dt(j), _ptr(h_inc), _ptr(kj), float(h), float(MU0), _ptr(H),
                                  _ptr(b1), _stream()), "vie_magnetic_field")
    return H, b1


def matvec_jm(op_n, op_k, x, eps_c, mu_c, h, freq_hz):
    """The full JMVIE operator of eq. 4 (vie_matvec_jm) on x = [J; M] of shape
    (2, 3, n3, n2, n1); eps_c, mu_c (n3, n2, n1) of the same dtype."""
    n1, n2, n3 = op_n.n
    if tuple(x.shape) != (2, 3, n3, n2, n1) or not x.is_contiguous():
        raise ValueError("x must be contiguous (2, 3, n3, n2, n1)")
    _dt(x)
    _require_like(eps_c, x, (n3, n2, n1), "eps_c")
    _require_like(mu_c, x, (n3, n2, n1), "mu_c")
    _require_device(x, "x")
    lib = load()
    dt = _dt(x)
    nbytes = lib.vie_jm_workspace_bytes(op_n.handle, op_k.handle, dt)
    ws = _scratch(nbytes, x.device)
    y = torch.empty_like(x)
    _check(lib.vie_matvec_jm(op_n.handle, op_k.handle, dt, float(h), 2.0 * np.pi * float(freq_hz), _ptr(eps_c),
                             _ptr(mu_c), _ptr(x), _ptr(y), _ptr(ws), nbytes, _stream()), "vie_matvec_jm")
    return y


def solve_jm(op_n, op_k, b, eps_c, mu_c, h, freq_hz, tol=1e-6, restart=50, max_outer=200, history=64,
             refine=False, inner_tol=1e-5):
    """GMRES for the full JMVIE system of eq. 4 (vie_solve_jm): b and the
    solution have shape (2, 3, n3, n2, n1) ([J; M]).  ``refine`` (complex128
    only): FP32 products in the Arnoldi steps, FP64 restart residuals.
    Returns (x, info dict, status)."""
    n1, n2, n3 = op_n.n
    if tuple(b.shape) != (2, 3, n3, n2, n1) or not b.is_contiguous():
        raise ValueError("b must be contiguous (2, 3, n3, n2, n1)")
    _dt(b)
    _require_like(eps_c, b, (n3, n2, n1), "eps_c")
    _require_like(mu_c, b, (n3, n2, n1), "mu_c")
    _require_device(b, "b")
    lib = load()
    dt = _dt(b)
    opts = SolveOpts(float(tol), int(restart), int(max_outer), 0, int(bool(refine)), VIE_RECON_FP32,
                     float(inner_tol))
    nbytes = lib.vie_solve_jm_workspace_bytes(op_n.handle, op_k.handle, dt, ctypes.byref(opts))
    if nbytes == 0:
        raise VieError(VIE_E_ARG, "vie_solve_jm_workspace_bytes rejected the options")
    ws = _scratch(nbytes, b.device)
    x = torch.empty_like(b)
    hist = np.zeros(max(1, int(history)))
    info = SolveInfo()
    info.history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    info.hist_cap = int(history)
    st = lib.vie_solve_jm(op_n.handle, op_k.handle, dt, float(h), 2.0 * np.pi * float(freq_hz), _ptr(eps_c),
                          _ptr(mu_c), _ptr(b), _ptr(x), ctypes.byref(opts), ctypes.byref(info), _ptr(ws), nbytes,
                          _stream())
    _check(st, "vie_solve_jm")
    d = {"matvecs": info.matvecs, "matvecs_fp64": info.matvecs_fp64, "restarts": info.restarts,
         "refine_steps": info.refine_steps, "converged": bool(info.converged),
         "rel_residual": info.rel_residual, "history": hist[:info.hist_len].tolist()}
    return x, d, st


def matvec_jm_pwl(op_n, op_k, x, eps_c, mu_c, h, freq_hz):
    """The JMVIE operator of eq. 4 in the mass-normalised piecewise-linear
    basis (vie_matvec_jm_pwl) on x = [J; M] of shape (2, 12, n3, n2, n1);
    op_n from compress_pwl, op_k from compress_pwl_k."""
    n1, n2, n3 = op_n.n
    if tuple(x.shape) != (2, 12, n3, n2, n1) or not x.is_contiguous():
        raise ValueError("x must be contiguous (2, 12, n3, n2, n1)")
    dt = _dt(x)
    _require_like(eps_c, x, (n3, n2, n1), "eps_c")
    _require_like(mu_c, x, (n3, n2, n1), "mu_c")
    _require_device(x, "x")
    lib = load()
    nbytes = lib.vie_jm_pwl_workspace_bytes(op_n.handle, op_k.handle, dt)
    ws = _scratch(nbytes, x.device)
    y = torch.empty_like(x)
    _check(lib.vie_matvec_jm_pwl(op_n.handle, op_k.handle, dt, float(h), 2.0 * np.pi * float(freq_hz),
                                 _ptr(eps_c), _ptr(mu_c), _ptr(x), _ptr(y), _ptr(ws), nbytes, _stream()),
           "vie_matvec_jm_pwl")
    return y


def solve_jm_pwl(op_n, op_k, b, eps_c, mu_c, h, freq_hz, tol=1e-6, restart=50, max_outer=200, history=64,
                 refine=False, inner_tol=1e-5):
    """GMRES for the JMVIE system in the piecewise-linear basis
    (vie_solve_jm_pwl): b and the solution (2, 12, n3, n2, n1), mass-normalised
    basis.  Returns (x, info dict, status)."""
    n1, n2, n3 = op_n.n
    if tuple(b.shape) != (2, 12, n3, n2, n1) or not b.is_contiguous():
        raise ValueError("b must be contiguous (2, 12, n3, n2, n1)")
    dt = _dt(b)
    _require_like(eps_c, b, (n3, n2, n1), "eps_c")
    _require_like(mu_c, b, (n3, n2, n1), "mu_c")
    _require_device(b, "b")
    lib = load()
    opts = SolveOpts(float(tol), int(restart), int(max_outer), 0, int(bool(refine)), VIE_RECON_FP32,
                     float(inner_tol))
    nbytes = lib.vie_solve_jm_pwl_workspace_bytes(op_n.handle, op_k.handle, dt, ctypes.byref(opts))
    if nbytes == 0:
        raise VieError(VIE_E_ARG, "vie_solve_jm_pwl_workspace_bytes rejected the options")
    ws = _scratch(nbytes, b.device)
    x = torch.empty_like(b)
    hist = np.zeros(max(1, int(history)))
    info = SolveInfo()
    info.history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    info.hist_cap = int(history)
    st = lib.vie_solve_jm_pwl(op_n.handle, op_k.handle, dt, float(h), 2.0 * np.pi * float(freq_hz), _ptr(eps_c),
                              _ptr(mu_c), _ptr(b), _ptr(x), ctypes.byref(opts), ctypes.byref(info), _ptr(ws), nbytes,
                              _stream())
    _check(st, "vie_solve_jm_pwl")
    d = {"matvecs": info.matvecs, "matvecs_fp64": info.matvecs_fp64, "restarts": info.restarts,
         "refine_steps": info.refine_steps, "converged": bool(info.converged),
         "rel_residual": info.rel_residual, "history": hist[:info.hist_len].tolist()}
    return x, d, st


def _cross_opts(tol, trunc_rule, max_rank, oversample, max_sweeps, n_sample, seed):
    return CrossOpts(float(tol), int(trunc_rule), int(max_rank), int(oversample), int(max_sweeps), int(n_sample),
                     int(seed))


def _cross_info_dict(xi, comps):
    return {"evals": [int(xi.evals[c]) for c in comps], "evals_sample": [int(xi.evals_sample[c]) for c in comps],
            "sweeps": [int(xi.sweeps[c]) for c in comps],
            "sample_rel_err": [float(xi.sample_rel_err[c]) for c in comps], "seconds": float(xi.seconds)}


def compress_cross(n, entry_fn, ctx, tol=1e-6, trunc_rule=0, max_rank=0, oversample=0, max_sweeps=0, n_sample=0,
                   seed=0):
    """Cross-Tucker compression (vie_compress_cross) from an entry callback:
    ``entry_fn`` a C function pointer (ctypes.c_void_p) of the vie_entry_fn
    shape and ``ctx`` its context pointer.  Returns (Operator, info dict)."""
    lib = load()
    nn = (ctypes.c_int * 3)(*[int(v) for v in n])
    opts = _cross_opts(tol, trunc_rule, max_rank, oversample, max_sweeps, n_sample, seed)
    info = CompressInfo()
    xi = CrossInfo()
    h = ctypes.c_void_p()
    _check(lib.vie_compress_cross(nn, entry_fn, ctx, ctypes.byref(opts), ctypes.byref(h), ctypes.byref(info),
                                  ctypes.byref(xi)), "vie_compress_cross")
    return Operator(h, tuple(int(v) for v in n), info), _cross_info_dict(xi, range(6))


def tucker_cross(n, entry_fn, ctx, comp, tol=1e-6, trunc_rule=0, max_rank=0, oversample=0, max_sweeps=0,
                 n_sample=0, seed=0, pwl=False):
    """Host-only cross-Tucker form of one component (vie_tucker_cross; with
    ``pwl`` a piecewise-linear component, vie_tucker_cross_pwl: comp 0..59
    the N components 6 P + c, 60..89 the K components 60 + 3 P + c).  Returns (core (r1, r2, r3), [U1, U2, U3], info
    dict), complex128."""
    lib = load()
    nn = (ctypes.c_int * 3)(*[int(v) for v in n])
    opts = _cross_opts(tol, trunc_rule, max_rank, oversample, max_sweeps, n_sample, seed)
    ranks = (ctypes.c_int * 3)()
    rcap = 64 + 16
    core = np.empty(2 * rcap ** 3, dtype=np.float64)
    fac = np.empty(2 * rcap * sum(int(v) for v in n), dtype=np.float64)
    xi = CrossInfo()
    fn = lib.vie_tucker_cross_pwl if pwl else lib.vie_tucker_cross
    _check(fn(nn, entry_fn, ctx, int(comp), ctypes.byref(opts), ranks, core.ctypes.data_as(ctypes.c_void_p),
              rcap ** 3, fac.ctypes.data_as(ctypes.c_void_p), rcap * sum(int(v) for v in n), ctypes.byref(xi)),
           "vie_tucker_cross_pwl" if pwl else "vie_tucker_cross")
    r = [int(ranks[a]) for a in range(3)]
    cz = core[:2 * r[0] * r[1] * r[2]].view(np.complex128).reshape(r)
    fz = fac.view(np.complex128)
    Us, o = [], 0
    for a in range(3):
        Us.append(fz[o:o + int(n[a]) * r[a]].reshape(int(n[a]), r[a]).copy())
        o += int(n[a]) * r[a]
    slot = int(comp) if not pwl else (int(comp) % 6 if comp < 60 else 3 + (int(comp) - 60) % 3)
    return cz.copy(), Us, _cross_info_dict(xi, [slot])


def tucker_hadamard(core, factors, x, cp=False, out=None):
    """y = D .* x for one component D = core x1 U1 x2 U2 x3 U3 (or, with
    ``cp``, the CP form with weights ``core`` of length R) on the grid of x
    (vie_tucker_hadamard).  ``core``, ``factors`` (U_a of shape (n_a, r_a))
    and ``x`` (shape (n3, n2, n1)) are device tensors of one complex dtype."""
    dt = _dt(x)
    n3, n2, n1 = x.shape
    _require_device(x, "x")
    for name, t in [("core", core)] + [("U%d" % (a + 1), f) for a, f in enumerate(factors)]:
        if t.dtype != x.dtype or t.device != x.device or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor on %s" % (name, x.dtype, x.device))
    r = [int(f.shape[1]) for f in factors]
    if [int(f.shape[0]) for f in factors] != [n1, n2, n3]:
        raise ValueError("factor rows must be (n1, n2, n3) = %s" % ((n1, n2, n3),))
    if cp:
        if tuple(core.shape) != (r[0],) or len(set(r)) != 1:
            raise ValueError("a CP form takes weights of shape (R,) and factors of R columns")
    elif tuple(core.shape) != tuple(r):
        raise ValueError("core shape must equal the factor ranks %s" % (tuple(r),))
    if not x.is_contiguous():
        raise ValueError("x must be contiguous")
    y = torch.empty_like(x) if out is None else out
    if out is not None:
        _require_like(out, x, x.shape, "out")
    lib = load()
    nn = (ctypes.c_int * 3)(n1, n2, n3)
    rr = (ctypes.c_int * 3)(*r)
    nbytes = lib.vie_tucker_hadamard_ws_bytes(nn, rr, int(bool(cp)), dt)
    ws = torch.empty(max(1, int(nbytes)), dtype=torch.uint8, device=x.device)
    _check(lib.vie_tucker_hadamard(nn, rr, int(bool(cp)), dt, _ptr(core), _ptr(factors[0]), _ptr(factors[1]),
                                   _ptr(factors[2]), _ptr(x), _ptr(y), _ptr(ws), nbytes, _stream()),
           "vie_tucker_hadamard")
    return y


def from_tucker(n, cores, factors):
    """Operator from a Tucker form computed elsewhere (vie_op_from_tucker):
    ``n`` = (n1, n2, n3); ``cores[c]`` complex (r1, r2, r3); ``factors[c]`` =
    (U1, U2, U3) real-space factors, U_a of shape (n_a, r_a)."""
    lib = load()
    nn = (ctypes.c_int * 3)(*[int(v) for v in n])
    ranks = (ctypes.c_int * 18)()
    cflat, fflat = [], []
    for c in range(6):
        G = np.ascontiguousarray(cores[c], dtype=np.complex128)
        for a in range(3):
            U = np.ascontiguousarray(factors[c][a], dtype=np.complex128)
            if U.shape != (n[a], G.shape[a]):
                raise ValueError("factor %d of component %d must be (n_a, r_a)" % (a, c))
            ranks[3 * c + a] = G.shape[a]
            fflat.append(U.ravel())
        cflat.append(G.ravel())
    cb = np.ascontiguousarray(np.concatenate(cflat))
    fb = np.ascontiguousarray(np.concatenate(fflat))
    info = CompressInfo()
    h = ctypes.c_void_p()
    _check(lib.vie_op_from_tucker(nn, ranks, cb.ctypes.data_as(ctypes.c_void_p), fb.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(h), ctypes.byref(info)), "vie_op_from_tucker")
    return Operator(h, tuple(int(v) for v in n), info)


def _as_batch(x, op):
    n1, n2, n3 = op.n
    if x.dim() == 4:
        x = x.unsqueeze(0)
    if x.dim() != 5 or tuple(x.shape[1:]) != (3, n3, n2, n1):
        raise ValueError("vector shape must be (nrhs, 3, %d, %d, %d)" % (n3, n2, n1))
    if not x.is_contiguous():
        raise ValueError("vectors must be contiguous")
    return x


def workspace_bytes(op, dtype, nrhs=1):
    """Device workspace (bytes) of vie_matvec for ``nrhs`` right-hand sides of
    torch ``dtype`` (complex64 or complex128)."""
    import torch
    dt = VIE_C128 if dtype == torch.complex128 else VIE_C64
    return int(load().vie_workspace_bytes(op.handle, dt, int(nrhs)))


def matvec(op, x, eps_c=None, kind="A", adjoint=False, recon="auto", out=None):
    """y = A x, N x (kind 'N'), or their adjoints, for a batch of vectors."""
    squeeze = x.dim() == 4
    xb = _as_batch(x, op)
    dt = _dt(xb)
    k = VIE_OP_A if kind == "A" else VIE_OP_N
    if k == VIE_OP_A:
        if eps_c is None:
            raise ValueError("eps_c required for kind 'A'")
        _require_like(eps_c, xb, xb.shape[2:], "eps_c")
    if out is not None:
        _require_like(_as_batch(out, op), xb, xb.shape, "out")
    _require_device(xb, "x")
    lib = load()
    y = torch.empty_like(xb) if out is None else _as_batch(out, op)
    nbytes = lib.vie_workspace_bytes(op.handle, dt, xb.shape[0])
    ws = op.workspace(nbytes, xb.device)
    fn = lib.vie_matvec_adjoint if adjoint else lib.vie_matvec
    _check(fn(op.handle, k, dt, _RECON[recon], _ptr(eps_c) if k == VIE_OP_A else None, _ptr(xb), _ptr(y),
              xb.shape[0], _ptr(ws), nbytes, _stream()), "vie_matvec")
    return y[0] if squeeze and out is None else y


def solve(op, b, eps_c, x0=None, tol=1e-6, restart=50, max_outer=200, adjoint=False, refine=False,
          inner_tol=1e-4, inner_recon="fp32", history=64):
    """GMRES solve of A x = b (or A^H x = b).  Returns (x, infos, status)."""
    squeeze = b.dim() == 4
    bb = _as_batch(b, op)
    dt = _dt(bb)
    nrhs = bb.shape[0]
    if eps_c is None:
        raise ValueError("eps_c required")
    _require_like(eps_c, bb, bb.shape[2:], "eps_c")
    if x0 is not None:
        _require_like(_as_batch(x0, op), bb, bb.shape, "x0")
    _require_device(bb, "b")
    lib = load()
    x = torch.zeros_like(bb) if x0 is None else _as_batch(x0, op).clone()
    opts = SolveOpts(float(tol), int(restart), int(max_outer), int(bool(adjoint)), int(bool(refine)),
                     _RECON[inner_recon], float(inner_tol))
    infos = (SolveInfo * nrhs)()
    hist = [(ctypes.c_double * history)() for _ in range(nrhs)]
    for s in range(nrhs):
        infos[s].history = ctypes.cast(hist[s], ctypes.POINTER(ctypes.c_double))
        infos[s].hist_cap = history
    nbytes = lib.vie_solve_workspace_bytes(op.handle, dt, nrhs, ctypes.byref(opts))
    if nbytes == 0:
        raise VieError(VIE_E_ARG, "vie_solve_workspace_bytes rejected the options")
    ws = op.workspace(nbytes, bb.device)
    st = _check(lib.vie_solve(op.handle, dt, _ptr(eps_c), _ptr(bb), _ptr(x), nrhs, ctypes.byref(opts), infos,
                              _ptr(ws), nbytes, _stream()), "vie_solve")
    out = []
    for s in range(nrhs):
        i = infos[s]
        out.append({"matvecs": i.matvecs, "matvecs_fp64": i.matvecs_fp64, "restarts": i.restarts,
                    "refine_steps": i.refine_steps, "converged": bool(i.converged),
                    "rel_residual": i.rel_residual, "history": [hist[s][t] for t in range(i.hist_len)]})
    if st == VIE_NOT_CONVERGED:
        warnings.warn("vie_solve: not every system reached tol %g" % tol)
    return (x[0] if squeeze else x), out, st


_multi_ws = {}


def _scratch(nbytes, device):
    key = (str(device), "multi")
    t = _multi_ws.get(key)
    if t is None or t.numel() < nbytes:
        t = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        _multi_ws[key] = t
    return t


def matvec_multi(items, kind="A", adjoint=False):
    """One multi-instance matvec: ``items`` is a list of (op, x, eps_c) with x of
    shape (nrhs, 3, n3, n2, n1) per instance (grids may differ); returns the
    list of outputs.  Every pass is one kernel launch over all instances."""
    arr = (Instance * len(items))()
    outs = []
    dt = None
    for op, x, eps_c in items:
        xb = _as_batch(x, op)
        dt = _dt(xb) if dt is None else dt
        if _dt(xb) != dt:
            raise ValueError("all instances must share a dtype")
        if kind == "A" and eps_c is None:
            raise ValueError("eps_c required for kind 'A'")
        if eps_c is not None:
            _require_like(eps_c, xb, xb.shape[2:], "eps_c")
    for op, x, _ in items:
        _require_device(x, "x")
    lib = load()
    for i, (op, x, eps_c) in enumerate(items):
        xb = _as_batch(x, op)
        y = torch.empty_like(xb)
        outs.append(y)
        arr[i] = Instance(op.handle, eps_c.data_ptr() if eps_c is not None else None, xb.data_ptr(), y.data_ptr(),
                          xb.shape[0])
    k = VIE_OP_A if kind == "A" else VIE_OP_N
    nbytes = lib.vie_matvec_multi_workspace_bytes(arr, len(items), dt)
    if nbytes == 0:
        raise VieError(VIE_E_ARG, "vie_matvec_multi_workspace_bytes rejected the batch")
    ws = _scratch(nbytes, outs[0].device)
    _check(lib.vie_matvec_multi(arr, len(items), k, int(bool(adjoint)), dt, _ptr(ws), nbytes, _stream()),
           "vie_matvec_multi")
    return outs


def solve_multi(items, tol=1e-6, restart=50, max_outer=200, adjoint=False, refine=False, inner_tol=1e-4,
                history=64, x0=None):
    """GMRES on several instances (op, b, eps_c) in lockstep; returns a list
    of (x, infos) per instance and the overall status.  ``x0``: optional list
    of initial guesses (one tensor per instance, shape of its b)."""
    arr = (SolveInstance * len(items))()
    keep = []
    xs = []
    dt = None
    if x0 is not None and len(x0) != len(items):
        raise ValueError("x0 must hold one tensor per instance")
    for i, (op, b, eps_c) in enumerate(items):
        bb = _as_batch(b, op)
        dt = _dt(bb) if dt is None else dt
        if _dt(bb) != dt:
            raise ValueError("all instances must share a dtype")
        if eps_c is None:
            raise ValueError("eps_c required")
        _require_like(eps_c, bb, bb.shape[2:], "eps_c")
        if x0 is not None:
            _require_like(_as_batch(x0[i], op), bb, bb.shape, "x0")
    for op, b, _ in items:
        _require_device(b, "b")
    lib = load()
    for i, (op, b, eps_c) in enumerate(items):
        bb = _as_batch(b, op)
        x = torch.zeros_like(bb) if x0 is None else _as_batch(x0[i], op).clone()
        xs.append(x)
        infos = (SolveInfo * bb.shape[0])()
        hist = [(ctypes.c_double * history)() for _ in range(bb.shape[0])]
        for s_ in range(bb.shape[0]):
            infos[s_].history = ctypes.cast(hist[s_], ctypes.POINTER(ctypes.c_double))
            infos[s_].hist_cap = history
        keep.append((infos, hist, bb))
        arr[i] = SolveInstance(op.handle, eps_c.data_ptr(), bb.data_ptr(), x.data_ptr(), bb.shape[0],
                               ctypes.cast(infos, ctypes.POINTER(SolveInfo)))
    opts = SolveOpts(float(tol), int(restart), int(max_outer), int(bool(adjoint)), int(bool(refine)),
                     VIE_RECON_FP32, float(inner_tol))
    nbytes = lib.vie_solve_multi_workspace_bytes(arr, len(items), dt, ctypes.byref(opts))
    if nbytes == 0:
        raise VieError(VIE_E_ARG, "vie_solve_multi_workspace_bytes rejected the batch")
    ws = _scratch(nbytes, xs[0].device)
    st = _check(lib.vie_solve_multi(arr, len(items), dt, ctypes.byref(opts), _ptr(ws), nbytes, _stream()),
                "vie_solve_multi")
    out = []
    for x, (infos, hist, bb) in zip(xs, keep):
        lst = []
        for s_ in range(bb.shape[0]):
            i_ = infos[s_]
            lst.append({"matvecs": i_.matvecs, "restarts": i_.restarts, "converged": bool(i_.converged),
                        "rel_residual": i_.rel_residual, "history": [hist[s_][t] for t in range(i_.hist_len)]})
        out.append((x, lst))
    return out, st


EPS0 = 8.8541878128e-12
C0 = 299792458.0
MU0 = 1.0 / (EPS0 * C0 * C0)


def _oe0(freq_hz):
    return 2.0 * np.pi * float(freq_hz) * EPS0


def _vec3(t, op, name):
    n1, n2, n3 = op.n
    if tuple(t.shape) != (3, n3, n2, n1) or not t.is_contiguous():
        raise ValueError("%s must be contiguous (3, %d, %d, %d)" % (name, n3, n2, n1))
    _dt(t)
    return _require_device(t, name)


def _same(ts, names):
    """Every tensor of ``ts`` shares the first one's dtype and device."""
    for t, nm in zip(ts[1:], names[1:]):
        if t.dtype != ts[0].dtype or t.device != ts[0].device:
            raise ValueError("%s must match %s in dtype and device" % (nm, names[0]))


def problem_setup(op, eps_r, sigma, e_inc, freq_hz):
    """eps_c = eps_r - i sigma/(omega eps0) and b = i omega eps0 (eps_c - 1) e_inc
    (real maps float32/float64 matching complex64/complex128 e_inc)."""
    _vec3(e_inc, op, "e_inc")
    rdt = torch.float32 if e_inc.dtype == torch.complex64 else torch.float64
    for t, nm in ((eps_r, "eps_r"), (sigma, "sigma")):
        if (t.dtype != rdt or not t.is_contiguous() or tuple(t.shape) != tuple(e_inc.shape[1:])
                or t.device != e_inc.device):
            raise ValueError("%s must be contiguous %s of shape %s on %s" % (nm, rdt, tuple(e_inc.shape[1:]),
                                                                             e_inc.device))
    eps_c = torch.empty(e_inc.shape[1:], dtype=e_inc.dtype, device=e_inc.device)
    b = torch.empty_like(e_inc)
    _check(load().vie_problem_setup(op.handle, _dt(e_inc), _ptr(eps_r), _ptr(sigma), _ptr(e_inc), _oe0(freq_hz),
                                    _ptr(eps_c), _ptr(b), _stream()), "vie_problem_setup")
    return eps_c, b


def total_field(op, e_inc, u, Nu, freq_hz):
    """E = e_inc + (N u - u) / (i omega eps0)."""
    for t, nm in ((e_inc, "e_inc"), (u, "u"), (Nu, "Nu")):
        _vec3(t, op, nm)
    _same((u, e_inc, Nu), ("u", "e_inc", "Nu"))
    E = torch.empty_like(u)
    _check(load().vie_total_field(op.handle, _dt(u), _ptr(e_inc), _ptr(u), _ptr(Nu), _oe0(freq_hz), _ptr(E),
                                  _stream()), "vie_total_field")
    return E


def adjoint_source(op, g, NHg):
    """t = N^H g - g."""
    _vec3(g, op, "g")
    _vec3(NHg, op, "NHg")
    _same((g, NHg), ("g", "NHg"))
    t = torch.empty_like(g)
    _check(load().vie_adjoint_source(op.handle, _dt(g), _ptr(g), _ptr(NHg), _ptr(t), _stream()),
           "vie_adjoint_source")
    return t


def field_gradient(op, z, E, freq_hz):
    """(dL/d eps_r, dL/d sigma) per voxel from the adjoint field z and the total field E."""
    _vec3(z, op, "z")
    _vec3(E, op, "E")
    _same((z, E), ("z", "E"))
    rdt = torch.float32 if z.dtype == torch.complex64 else torch.float64
    ge = torch.empty(z.shape[1:], dtype=rdt, device=z.device)
    gs = torch.empty_like(ge)
    _check(load().vie_field_gradient(op.handle, _dt(z), _ptr(z), _ptr(E), _oe0(freq_hz), _ptr(ge), _ptr(gs),
                                     _stream()), "vie_field_gradient")
    return ge, gs


def densify(op, with_c128=False):
    _check(load().vie_op_densify(op.handle, int(with_c128)), "vie_op_densify")


def set_nhat(op, source):
    _check(load().vie_op_set_nhat(op.handle, VIE_NHAT_DENSE if source == "dense" else VIE_NHAT_TUCKER),
           "vie_op_set_nhat")


def debug_nhat(op, idx, dtype=torch.complex64):
    """Fourier-domain tensor values at (c, k1, k2, k3) rows of ``idx``,
    including the 1/(8 n1 n2 n3) scale carried by the device core."""
    lib = load()
    a = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 4)
    out = np.empty((a.shape[0], 2), dtype=np.float64)
    dt = VIE_C128 if dtype == torch.complex128 else VIE_C64
    _check(lib.vie_debug_nhat(op.handle, dt, VIE_RECON_AUTO, a.ctypes.data_as(ctypes.c_void_p), a.shape[0],
                              out.ctypes.data_as(ctypes.c_void_p)), "vie_debug_nhat")
    return out[:, 0] + 1j * out[:, 1]


def pass_shape(op, layout, nrhs=1):
    """Shape of a pass buffer: 'vector' (nrhs, 3, n3, n2, n1), 'S1'/'S3'
    (nrhs, 3, n3, L1, n2) or 'S2' (nrhs, 3, L2, L1, n3), L_a = 2 n_a."""
    n1, n2, n3 = op.n
    if layout == "vector":
        return (nrhs, 3, n3, n2, n1)
    if layout in ("S1", "S3"):
        return (nrhs, 3, n3, 2 * n1, n2)
    if layout == "S2":
        return (nrhs, 3, 2 * n2, 2 * n1, n3)
    raise ValueError(layout)


_PASS_IO = {0: ("vector", "S1"), 1: ("S1", "S2"), 2: ("S2", "S2"), 3: ("S2", "S3"), 4: ("S3", "vector")}


def _pass_tensor(t, op, layout, name, ref=None):
    shape = pass_shape(op, layout, t.shape[0] if t.dim() == 5 else 1)
    if t.dim() != 5 or tuple(t.shape) != shape or not t.is_contiguous():
        raise ValueError("%s must be contiguous %s" % (name, shape))
    if ref is not None and (t.dtype != ref.dtype or t.device != ref.device):
        raise ValueError("%s must match the other buffers in dtype and device" % name)
    _dt(t)
    return t


def debug_pad(op, x):
    """vie_debug_pad: the X+ pass's zero padding and transpose (identity in
    place of the FFT); x (nrhs, 3, n3, n2, n1) -> S1 (nrhs, 3, n3, 2 n1, n2)."""
    _pass_tensor(x, op, "vector", "x")
    _require_device(x, "x")
    out = torch.empty(pass_shape(op, "S1", x.shape[0]), dtype=x.dtype, device=x.device)
    _check(load().vie_debug_pad(op.handle, _dt(x), _ptr(x), _ptr(out), x.shape[0], _stream()), "vie_debug_pad")
    return out


def debug_crop(op, s3):
    """vie_debug_crop: the X- pass's transpose and crop (identity in place of
    the FFT, bare epilogue); S3 (nrhs, 3, n3, 2 n1, n2) -> (nrhs, 3, n3, n2, n1)."""
    _pass_tensor(s3, op, "S3", "s3")
    _require_device(s3, "s3")
    out = torch.empty(pass_shape(op, "vector", s3.shape[0]), dtype=s3.dtype, device=s3.device)
    _check(load().vie_debug_crop(op.handle, _dt(s3), _ptr(s3), _ptr(out), s3.shape[0], _stream()), "vie_debug_crop")
    return out


def debug_pass(op, p, inp=None, x=None, eps_c=None, kind="A", adjoint=False, recon="auto", out=None):
    """vie_debug_pass: pass ``p`` (0 X+, 1 Y+, 2 Z*, 3 Y-, 4 X-) of the matvec on
    the pass layouts (see pass_shape); returns the output buffer."""
    lin, lout = _PASS_IO[int(p)]
    ref = x if p == 0 else inp
    if ref is None:
        raise ValueError("pass %d needs %s" % (p, "x" if p == 0 else "inp"))
    _pass_tensor(ref, op, lin, "input")
    nrhs = ref.shape[0]
    if x is not None:
        _pass_tensor(x, op, "vector", "x", ref)
        if x.shape[0] != nrhs:
            raise ValueError("x must have the input's right-hand-side count")
    if eps_c is not None:
        _require_like(eps_c, ref, tuple(reversed(op.n)), "eps_c")
    if out is not None:
        _pass_tensor(out, op, lout, "out", ref)
    _require_device(ref, "input")
    if out is None:
        out = torch.empty(pass_shape(op, lout, nrhs), dtype=ref.dtype, device=ref.device)
    k = VIE_OP_A if kind == "A" else VIE_OP_N
    _check(load().vie_debug_pass(op.handle, int(p), k, int(bool(adjoint)), _dt(ref), _RECON[recon], _ptr(eps_c),
                                 _ptr(x), _ptr(inp), _ptr(out), nrhs, _stream()), "vie_debug_pass")
    return out


def debug_hosvd(tensor, tol, rule=0, want_recon=True):
    """Host-only HOSVD of one defining tensor (numpy complex128 (n3, n2, n1)):
    returns (ranks, [s1, s2, s3], reconstruction, tail).  No device work."""
    lib = load()
    a = np.ascontiguousarray(tensor, dtype=np.complex128)
    n3, n2, n1 = a.shape
    n = (ctypes.c_int * 3)(n1, n2, n3)
    ranks = (ctypes.c_int * 3)()
    sv = np.empty(n1 + n2 + n3)
    rec = np.empty(a.shape, dtype=np.complex128) if want_recon else None
    tail = ctypes.c_double()
    _check(lib.vie_debug_hosvd(n, a.ctypes.data_as(ctypes.c_void_p), float(tol), int(rule), ranks,
                               sv.ctypes.data_as(ctypes.c_void_p),
                               rec.ctypes.data_as(ctypes.c_void_p) if want_recon else None,
                               ctypes.byref(tail)), "vie_debug_hosvd")
    return tuple(ranks), [sv[:n1], sv[n1:n1 + n2], sv[n1 + n2:]], rec, tail.value


def debug_cp(core, R, iters):
    """Host-only CP-ALS of one core (numpy complex128 (r1, r2, r3)) with R
    terms and ``iters`` sweeps: returns ([V1, V2, V3], relative error)."""
    lib = load()
    G = np.ascontiguousarray(core, dtype=np.complex128)
    r = (ctypes.c_int * 3)(*G.shape)
    V = np.empty(sum(G.shape) * R, dtype=np.complex128)
    err = ctypes.c_double()
    _check(lib.vie_debug_cp(r, G.ctypes.data_as(ctypes.c_void_p), int(R), int(iters),
                            V.ctypes.data_as(ctypes.c_void_p), ctypes.byref(err)), "vie_debug_cp")
    r1, r2, _ = G.shape
    return [V[:r1 * R].reshape(r1, R), V[r1 * R:(r1 + r2) * R].reshape(r2, R), V[(r1 + r2) * R:].reshape(-1, R)], err.value


def profile_enable(on=True):
    _check(load().vie_profile_enable(int(bool(on))), "vie_profile_enable")


def profile_collect():
    """Summed per-pass milliseconds and launch counts since the last collect."""
    ms = (ctypes.c_double * 5)()
    cnt = (ctypes.c_int * 5)()
    _check(load().vie_profile_collect(ctypes.cast(ms, ctypes.c_void_p), ctypes.cast(cnt, ctypes.c_void_p)),
           "vie_profile_collect")
    return list(ms), list(cnt)


def set_kernel_path(path):
    """0 = default kernel choice, 1 = mixed-radix LDS kernels only."""
    _check(load().vie_set_kernel_path(int(path)), "vie_set_kernel_path")


def set_batch_mode(mode):
    """0 = per-instance register-FFT launches (default), 1 = one mixed-radix
    launch per pass over every instance."""
    _check(load().vie_set_batch_mode(int(mode)), "vie_set_batch_mode")


def autotune(op, dtype=None, nrhs=1):
    """Time the z-pass launch shapes on the device and keep the fastest in the
    operator (vie_autotune).  Returns (quads per workgroup, {candidate: ms})."""
    lib = load()
    dtype = torch.complex64 if dtype is None else dtype
    dt = VIE_C128 if dtype == torch.complex128 else VIE_C64
    dev = torch.device("cuda", torch.cuda.current_device())
    nbytes = lib.vie_workspace_bytes(op.handle, dt, int(nrhs))
    ws = op.workspace(nbytes, dev)
    ms = (ctypes.c_double * 4)()
    chosen = ctypes.c_int(0)
    _check(lib.vie_autotune(op.handle, dt, int(nrhs), _ptr(ws), nbytes, _stream(), ctypes.cast(ms, ctypes.c_void_p),
                            ctypes.byref(chosen)), "vie_autotune")
    return int(chosen.value), {c: float(ms[i]) for i, c in enumerate((4, 8, 16, 32))}


class MatvecGraph:
    """One matvec captured into a HIP graph (vie_matvec_graph) on fixed
    tensors: write new input into ``x`` in place, call ``launch()``, read
    ``y``.  Owns its workspace; keeps x, y, eps_c and the operator alive."""

    def __init__(self, op, x, eps_c=None, kind="A", adjoint=False, recon="auto", out=None):
        self.handle = None
        xb = _as_batch(x, op)
        dt = _dt(xb)
        k = VIE_OP_A if kind == "A" else VIE_OP_N
        if k == VIE_OP_A:
            if eps_c is None:
                raise ValueError("eps_c required for kind 'A'")
            _require_like(eps_c, xb, xb.shape[2:], "eps_c")
        if out is not None:
            _require_like(_as_batch(out, op), xb, xb.shape, "out")
        _require_device(xb, "x")
        lib = load()
        self._lib = lib
        y = torch.empty_like(xb) if out is None else _as_batch(out, op)
        nbytes = lib.vie_workspace_bytes(op.handle, dt, xb.shape[0])
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=xb.device)
        self.op, self.x, self.y, self.eps_c = op, xb, y, eps_c
        h = ctypes.c_void_p()
        _check(lib.vie_matvec_graph(op.handle, k, int(bool(adjoint)), dt, _RECON[recon],
                                    _ptr(eps_c) if k == VIE_OP_A else None, _ptr(xb), _ptr(y), xb.shape[0],
                                    _ptr(self.ws), nbytes, ctypes.byref(h)), "vie_matvec_graph")
        self.handle = h

    def launch(self):
        _check(self._lib.vie_graph_launch(self.handle, _stream()), "vie_graph_launch")
        return self.y

    def close(self):
        if self.handle is not None and self.handle.value:
            self._lib.vie_graph_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exported_symbols():
    return list(_SIGS)
