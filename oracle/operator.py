"""Electric block of the FFT-VIE operator (FP64).  Test infrastructure only.

With piecewise-constant current coefficients u_q(m) on the voxel grid and
Galerkin rows divided by the voxel volume, the electric block of eq. 4
(M_eps - M_chi N, Sec. II) acts as

    (A u)_p(m) = eps_c(m) u_p(m) - chi(m) sum_q sum_m' Nt_pq(m - m') u_q(m')

with chi = eps_c - 1.  The sum is a 3-level Toeplitz (BTTB) product
(Sec. II-B) and is evaluated here three ways:

* ``brute_force_N`` -- the double sum written out (tiny grids only);
* ``apply_N`` with a Fourier-domain tensor from ``dense_operator`` -- zero
  padding, circulant embedding and FFT of the dense defining tensors;
* ``apply_N`` with ``tucker_operator`` -- the same with every component
  replaced by its HOSVD approximation, the Fourier-domain tensor built from
  embedded, transformed factors (Sec. V-A) and reconstructed densely.

Vectors use the storage layout of ``vie_inputs``: (3, n3, n2, n1), x fastest.
"""
import os

import numpy as np
import scipy.fft as sfft

from .circulant import COMPONENTS, axis_signs, component_index, fourier_tensor_dense, \
    fourier_tensor_tucker
from .cp import fourier_tensor_cp, tucker_cp
from .tucker import from_storage, hosvd, to_storage


def _workers():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


class FourierOperator:
    """Fourier-domain Green's tensor: ``nhat[c]`` has shape (2n1, 2n2, 2n3)
    (math order) for the components xx, yy, zz, xy, xz, yz."""

    def __init__(self, n, nhat, ranks=None, factors=None, cores=None, svals=None):
        self.n = tuple(int(v) for v in n)
        self.nhat = nhat
        self.ranks = ranks
        self.factors = factors
        self.cores = cores
        self.svals = svals


def dense_operator(green):
    """Fourier-domain tensor of the dense defining tensors (storage layout
    (6, n3, n2, n1))."""
    n = (green.shape[3], green.shape[2], green.shape[1])
    nhat = [fourier_tensor_dense(from_storage(green[c]), axis_signs(c)) for c in range(6)]
    return FourierOperator(n, nhat)


def tucker_operator(green, tol, rule=0):
    """HOSVD of each defining tensor (Alg. 1) at tolerance ``tol``, then the
    Fourier-domain tensor from the Tucker form (Sec. V-A)."""
    n = (green.shape[3], green.shape[2], green.shape[1])
    nhat, ranks, factors, cores, svals = [], [], [], [], []
    for c in range(6):
        G, Us, s = hosvd(from_storage(green[c]), tol, rule)
        nhat.append(fourier_tensor_tucker(G, Us, axis_signs(c)))
        ranks.append(tuple(U.shape[1] for U in Us))
        factors.append(Us)
        cores.append(G)
        svals.append(s)
    return FourierOperator(n, nhat, ranks, factors, cores, svals)


def cross_operator(n, entries_of, tol, rule=0, **kw):
    """Tucker cross approximation (Sec. IV-A's cross-Tucker, ``cross.tucker_cross``)
    of each defining tensor from its entries, then the Fourier-domain tensor
    from the Tucker forms (Sec. V-A).  ``entries_of(c)`` returns the entries
    callable (i, j, k) -> Nt_c of component c; the parity zeros of the odd
    components are imposed.  ``op.cross_info`` holds each component's
    counts."""
    from .cross import green_entries, tucker_cross
    nhat, ranks, factors, cores, infos = [], [], [], [], []
    for c in range(6):
        odd = [s < 0 for s in axis_signs(c)]
        G, Us, info = tucker_cross(green_entries(entries_of(c), odd), n, tol, rule, **kw)
        nhat.append(fourier_tensor_tucker(G, Us, axis_signs(c)))
        ranks.append(tuple(U.shape[1] for U in Us))
        factors.append(Us)
        cores.append(G)
        infos.append(info)
    op = FourierOperator(n, nhat, ranks, factors, cores)
    op.cross_info = infos
    return op


def tucker_cp_operator(green, tol, R=None, iters=1000, rule=0):
    """Tucker+CP of each defining tensor (Alg. 2: HOSVD at ``tol``, CP of the
    core with R terms by alternating least squares), then the Fourier-domain
    tensor of eq. 17 with the embedded, transformed Tucker+CP factors."""
    n = (green.shape[3], green.shape[2], green.shape[1])
    nhat, ranks, factors, errs = [], [], [], []
    for c in range(6):
        Ws, G, Us, Vs, e = tucker_cp(from_storage(green[c]), tol, R, iters, rule)
        nhat.append(fourier_tensor_cp(Ws, axis_signs(c)))
        ranks.append(tuple(U.shape[1] for U in Us))
        factors.append(Ws)
        errs.append(e[-1] if e else 0.0)
    op = FourierOperator(n, nhat, ranks, factors)
    op.cp_rel_err = errs
    return op


def apply_N(op, u, conj=False):
    """Bare Green's operator N u (or N^H u with ``conj``), by zero padding
    to (2n1, 2n2, 2n3), FFT, the 3x3 component product in the Fourier
    domain, inverse FFT and cropping.  N^H uses conj(N^) because the
    embedded tensors are even in the full offset and N is symmetric."""
    n1, n2, n3 = op.n
    U = np.stack([from_storage(u[q]) for q in range(3)])
    L = (2 * n1, 2 * n2, 2 * n3)
    w = _workers()
    Xh = []
    for q in range(3):
        pad = np.zeros(L, dtype=np.complex128)
        pad[:n1, :n2, :n3] = U[q]
        Xh.append(sfft.fftn(pad, workers=w))
    out = np.empty((3, n3, n2, n1), dtype=np.complex128)
    for p in range(3):
        Yh = np.zeros(L, dtype=np.complex128)
        for q in range(3):
            N = op.nhat[component_index(p, q)]
            Yh += (np.conj(N) if conj else N) * Xh[q]
        y = sfft.ifftn(Yh, workers=w)[:n1, :n2, :n3]
        out[p] = to_storage(y)
    return out


def matvec(op, eps_c, u, mode="A"):
    """Apply the electric block (eq. 4) or its pieces.

    mode 'A' : eps_c u - chi (N u)
    mode 'AH': conj(eps_c) u - N^H (conj(chi) u)      (adjoint of 'A')
    mode 'N' : N u,   mode 'NH': N^H u
    """
    if mode == "N":
        return apply_N(op, u)
    if mode == "NH":
        return apply_N(op, u, conj=True)
    eps_c = np.asarray(eps_c)
    chi = eps_c - 1.0
    if mode == "A":
        return eps_c[None] * u - chi[None] * apply_N(op, u)
    if mode == "AH":
        return np.conj(eps_c)[None] * u - apply_N(op, np.conj(chi)[None] * u, conj=True)
    raise ValueError(mode)


def signed_entry(green, c, D):
    """Nt_c at a signed offset D = (dx, dy, dz) using the component's parity."""
    s = axis_signs(c)
    sign = 1
    for a in range(3):
        if D[a] < 0:
            sign *= s[a]
    return sign * green[c, abs(D[2]), abs(D[1]), abs(D[0])]


def brute_force_N(green, u):
    """N u as the explicit Toeplitz double sum (tiny grids)."""
    n3, n2, n1 = u.shape[1:]
    out = np.zeros_like(u, dtype=np.complex128)
    idx = [(i, j, k) for k in range(n3) for j in range(n2) for i in range(n1)]
    for p in range(3):
        for (i, j, k) in idx:
            acc = 0j
            for q in range(3):
                c = component_index(p, q)
                for (i2, j2, k2) in idx:
                    acc += signed_entry(green, c, (i - i2, j - j2, k - k2)) * u[q, k2, j2, i2]
            out[p, k, j, i] = acc
    return out


def dense_matrix(green, eps_c=None, mode="N"):
    """Explicit 3V x 3V matrix of N (mode 'N') or A (mode 'A') for tiny
    grids; unknown ordering (q, k, j, i) as in the storage layout."""
    n3, n2, n1 = green.shape[1:]
    V = n1 * n2 * n3
    idx = [(i, j, k) for k in range(n3) for j in range(n2) for i in range(n1)]
    M = np.zeros((3 * V, 3 * V), dtype=np.complex128)
    for p in range(3):
        for q in range(3):
            c = component_index(p, q)
            for a, (i, j, k) in enumerate(idx):
                for b, (i2, j2, k2) in enumerate(idx):
                    M[p * V + a, q * V + b] = signed_entry(green, c, (i - i2, j - j2, k - k2))
    if mode == "N":
        return M
    e = np.tile(np.asarray(eps_c).ravel(), 3)
    return np.diag(e) - (e - 1.0)[:, None] * M
