"""Galerkin Green's tensors of the volume operators N and K (PWC basis).

Thin wrapper over ``csrc/green.c``; see the header there for the reading of
the Galerkin entries used.  The result depends only on kappa = k0 h and the
grid size: entries are normalised by the voxel volume, so that the identity
part of the operator has unit diagonal.
"""
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
