"""Galerkin Green's tensors of the volume operators N and K (PWC basis) and
of N for the piecewise-linear basis (eq. 7b).

Thin wrapper over ``csrc/green.c``; see the header there for the reading of
the Galerkin entries used.  The result depends only on kappa = k0 h and the
grid size: entries are normalised by the voxel volume, so that the identity
part of the operator has unit diagonal.
"""
import ctypes

import numpy as np

from . import _native


def green_tensor(n, h, k0, near_order=16, far_boost=0):
    """Dense defining tensor, shape (6, n3, n2, n1) complex128.

    ``n``: grid (n1, n2, n3); ``h``: cubic voxel edge (m); ``k0``: free-space
    wavenumber (1/m).  ``near_order`` is the Gauss order of the singular
    (|offset|_inf <= 1) integrals and ``far_boost`` raises the order of every
    far-field shell (both only for convergence checks).
    """
    n1, n2, n3 = (int(v) for v in n)
    V = n1 * n2 * n3
    out = np.empty((6, n3, n2, n1, 2), dtype=np.float64)
    rc = _native.lib().vie_green_fill(n1, n2, n3, float(k0) * float(h), int(near_order),
                                      int(far_boost), out.ctypes.data, 0, V)
    if rc != 0:
        raise ValueError("vie_green_fill failed (%d)" % rc)
    return out[..., 0] + 1j * out[..., 1]


def green_k_tensor(n, h, k0, near_order=16, far_boost=0):
    """Dense defining tensor of the magnetic operator K (curl of the
    single-layer potential, eq. 5), shape (3, n3, n2, n1) complex128,
    components xy, xz, yz; entry [c, k, j, i] = Kt_c(offset (i, j, k)) with
    the observation voxel at the offset and the source voxel at 0, so that
    (K u)_p(m) = h sum_m' Kt_pq(m - m') u_q(m') (Kt_qp = -Kt_pq, zero
    diagonal).  Dimensionless: multiply by ``h`` for the physical operator."""
    n1, n2, n3 = (int(v) for v in n)
    V = n1 * n2 * n3
    out = np.empty((3, n3, n2, n1, 2), dtype=np.float64)
    rc = _native.lib().vie_green_k_fill(n1, n2, n3, float(k0) * float(h), int(near_order),
                                        int(far_boost), out.ctypes.data, 0, V)
    if rc != 0:
        raise ValueError("vie_green_k_fill failed (%d)" % rc)
    return out[..., 0] + 1j * out[..., 1]


def green_entries(idx, comp, h, k0, near_order=16, far_boost=0):
    """Entries Nt_comp(D) of the defining tensor at the offsets ``idx``
    (integer array (..., 3) of (i, j, k) >= 0), complex128 of shape
    idx.shape[:-1]; bitwise equal to ``green_tensor(...)[comp, k, j, i]``."""
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
    if idx.shape[-1] != 3:
        raise ValueError("idx must have shape (..., 3)")
    flat = idx.reshape(-1, 3)
    out = np.empty((flat.shape[0], 2), dtype=np.float64)
    rc = _native.lib().vie_green_entries(float(k0) * float(h), int(near_order), int(far_boost), int(comp),
                                         flat.shape[0], flat.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise ValueError("vie_green_entries failed (%d)" % rc)
    return (out[:, 0] + 1j * out[:, 1]).reshape(idx.shape[:-1])


class GreenEntryCallback:
    """C function pointer and context that evaluate defining-tensor entries
    (``vie_green_entry_cb`` in csrc/green.c), in the form a fiber-sampling
    compression takes: ``fn(ctx, comp, count, idx[count][3], out[count][2])``.
    Keep this object alive while the pointer is in use."""

    class _Ctx(ctypes.Structure):
        _fields_ = [("kappa", ctypes.c_double), ("near_q", ctypes.c_int), ("boost", ctypes.c_int)]

    def __init__(self, h, k0, near_order=16, far_boost=0):
        self.ctx = self._Ctx(float(k0) * float(h), int(near_order), int(far_boost))
        lib = _native.lib()
        self.fn = ctypes.cast(lib.vie_green_entry_cb, ctypes.c_void_p)

    @property
    def ctx_ptr(self):
        return ctypes.cast(ctypes.pointer(self.ctx), ctypes.c_void_p)


#: basis-function pairs (test l, basis l') of the stored PWL tensors;
#: 0 = pulse, 1..3 = pulse times (x - x_m)/h, (y - y_m)/h, (z - z_m)/h
PWL_PAIRS = ((0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3))


def pwl_pair_index(l, lp):
    """Index of the stored pair holding (l, l') and the sign that turns it
    into (l, l'): Nt^(l',l) = sigma Nt^(l,l'), sigma = -1 when exactly one
    of the two is the pulse."""
    a, b = (l, lp) if l <= lp else (lp, l)
    sign = 1.0 if (l <= lp or (a != 0) == (b != 0)) else -1.0
    return PWL_PAIRS.index((a, b)), sign


def green_pwl_tensor(n, h, k0, near_order=16, far_boost=0):
    """Dense PWL defining tensors, shape (10, 6, n3, n2, n1) complex128:
    entry [P, c, k, j, i] = Nt^{(l,l')}_c(offset (i, j, k)) for the pair
    P = PWL_PAIRS.index((l, l')) (test function l in voxel 0, basis
    function l' in the voxel at the offset) and c = xx, yy, zz, xy, xz, yz.
    The self products of the basis are (1, 1/12, 1/12, 1/12)."""
    n1, n2, n3 = (int(v) for v in n)
    V = n1 * n2 * n3
    out = np.empty((10, 6, n3, n2, n1, 2), dtype=np.float64)
    rc = _native.lib().vie_green_pwl_fill(n1, n2, n3, float(k0) * float(h), int(near_order),
                                          int(far_boost), out.ctypes.data, 0, V)
    if rc != 0:
        raise ValueError("vie_green_pwl_fill failed (%d)" % rc)
    return out[..., 0] + 1j * out[..., 1]


def green_pwl_entry(D, kappa, order, method=0):
    """All 60 PWL entries at one offset D (any signs), shape (10, 6):
    method 0 = the distributional form (any offset), 1 = the smooth dyadic
    form (max |D_i| >= 2), each at Gauss order ``order``; kappa = k0 h."""
    Dc = np.ascontiguousarray(np.asarray(D, dtype=np.int32).reshape(3))
    out = np.empty((60, 2), dtype=np.float64)
    rc = _native.lib().vie_green_pwl_entry(Dc.ctypes.data, float(kappa), int(order), int(method),
                                           out.ctypes.data)
    if rc != 0:
        raise ValueError("vie_green_pwl_entry failed (%d)" % rc)
    return (out[:, 0] + 1j * out[:, 1]).reshape(10, 6)


def green_pwl_entries(idx, comp, h, k0, near_order=16, far_boost=0):
    """Entries of the PWL component comp = 6 P + c (pair P of PWL_PAIRS,
    dyadic component c) at the offsets ``idx`` (integer array (..., 3) >= 0),
    complex128 of shape idx.shape[:-1]; equal to
    ``green_pwl_tensor(...)[P, c, k, j, i]`` up to rounding order."""
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
    if idx.shape[-1] != 3:
        raise ValueError("idx must have shape (..., 3)")
    flat = idx.reshape(-1, 3)
    out = np.empty((flat.shape[0], 2), dtype=np.float64)
    rc = _native.lib().vie_green_pwl_entries(float(k0) * float(h), int(near_order), int(far_boost), int(comp),
                                             flat.shape[0], flat.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise ValueError("vie_green_pwl_entries failed (%d)" % rc)
    return (out[:, 0] + 1j * out[:, 1]).reshape(idx.shape[:-1])


def green_pwl_k_tensor(n, h, k0, near_order=16, far_boost=0):
    """Dense PWL tensors of the magnetic operator K, shape (10, 3, n3, n2,
    n1) complex128: entry [P, c, k, j, i] = Kt^{(l,l')}_c(offset (i, j, k))
    for the pair P = PWL_PAIRS.index((l, l')) with the test function l in the
    observation voxel at the offset and the basis function l' in the source
    voxel 0 (the pulse K's convention), c = xy, xz, yz; Kt^(l',l) =
    sigma Kt^(l,l') as for N.  Dimensionless (physical: h times)."""
    n1, n2, n3 = (int(v) for v in n)
    V = n1 * n2 * n3
    out = np.empty((10, 3, n3, n2, n1, 2), dtype=np.float64)
    rc = _native.lib().vie_green_pwl_k_fill(n1, n2, n3, float(k0) * float(h), int(near_order),
                                            int(far_boost), out.ctypes.data, 0, V)
    if rc != 0:
        raise ValueError("vie_green_pwl_k_fill failed (%d)" % rc)
    return out[..., 0] + 1j * out[..., 1]


def green_pwl_k_entry(D, kappa, order, method=0):
    """All 30 PWL K entries at one offset D (any signs), shape (10, 3):
    method 0 = the volume form -int g^ d_s W (any offset), 1 = the smooth
    form int d_s g^ W (max |D_i| >= 2); no zero planes imposed."""
    Dc = np.ascontiguousarray(np.asarray(D, dtype=np.int32).reshape(3))
    out = np.empty((30, 2), dtype=np.float64)
    rc = _native.lib().vie_green_pwl_k_entry(Dc.ctypes.data, float(kappa), int(order), int(method),
                                             out.ctypes.data)
    if rc != 0:
        raise ValueError("vie_green_pwl_k_entry failed (%d)" % rc)
    return (out[:, 0] + 1j * out[:, 1]).reshape(10, 3)


def green_pwl_k_entries(idx, comp, h, k0, near_order=16, far_boost=0):
    """Entries of the PWL K component comp = 3 P + c at offsets ``idx`` >= 0."""
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int32))
    flat = idx.reshape(-1, 3)
    out = np.empty((flat.shape[0], 2), dtype=np.float64)
    rc = _native.lib().vie_green_pwl_k_entries(float(k0) * float(h), int(near_order), int(far_boost), int(comp),
                                               flat.shape[0], flat.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise ValueError("vie_green_pwl_k_entries failed (%d)" % rc)
    return (out[:, 0] + 1j * out[:, 1]).reshape(idx.shape[:-1])


class GreenPwlEntryCallback(GreenEntryCallback):
    """``GreenEntryCallback`` for the PWL components: comp 0..59 the N
    components 6 P + c, 60..89 the K components 60 + 3 P + c."""

    def __init__(self, h, k0, near_order=16, far_boost=0):
        super().__init__(h, k0, near_order, far_boost)
        self.fn = ctypes.cast(_native.lib().vie_green_pwl_entry_cb, ctypes.c_void_p)
