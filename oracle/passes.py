"""The matvec of Sec. V-A split into its five passes (FP64).  Test
infrastructure only: imported by tests/, never by the library or its binding.

The FFT-based product of eq. 4's electric block pads the currents to the
circulant embedding (L_a = 2 n_a), transforms them, multiplies by the
Fourier-domain Green's tensor, transforms back and crops.  Done one axis at
a time, with the intermediate arrays in the layouts the device passes
exchange (per right-hand side, slowest index first):

    vector  (3, n3, n2, n1)     S1, S3  (3, n3, L1, n2)     S2  (3, L2, L1, n3)

    X+  S1[q, k, i', j] = sum_{i < n1} x[q, k, j, i] w1^(-i i')
    Y+  S2[q, j', i', k] = sum_{j < n2} S1[q, k, i', j] w2^(-j j')
    Z*  S2[p, j', i', k] = sum_{k3} w3^(k k3) sum_q Nh_pq(i', j', k3) / M
                             * sum_{m < n3} S2[q, j', i', m] w3^(-m k3),   k < n3
    Y-  S3[q, k, i', j] = sum_{j'} S2[q, j', i', k] w2^(j j'),   j < n2
    X-  r[q, k, j, i] = sum_{i'} S3[q, k, i', j] w1^(i i'),   i < n1

with w_a = exp(2 pi i / L_a) and M = L1 L2 L3 (the 1/M of the inverse
transforms is applied with the tensor), followed by the contrast epilogue
of eq. 4 (A: eps u - chi r; A^H: conj(eps) u - r with the input pre-scaled by
conj(chi) in X+; N: r).  Every DFT is an explicit matrix product whose
entries at multiples of a quarter turn are exactly 0 and +-1, so on
integer data of lengths 1, 2 and 4 every value is exact.
"""
import numpy as np

from .circulant import component_index


def dft_matrix(L, sign):
    """F[k, m] = exp(sign 2 pi i m k / L), exactly 0, +-1 at quarter turns."""
    mk = np.outer(np.arange(L), np.arange(L)) % L
    F = np.exp(sign * 2j * np.pi * mk / L)
    q = (4 * mk) % L == 0
    quarter = (4 * mk[q]) // L
    F[q] = np.array([1, 1j, -1, -1j])[quarter] if sign > 0 else np.array([1, -1j, -1, 1j])[quarter]
    return F


def _dft_along(a, axis, L, sign, keep=None):
    """Pad axis `axis` of `a` with zeros to L, DFT it, keep the first `keep`."""
    n = a.shape[axis]
    F = dft_matrix(L, sign)[:, :n]
    out = np.moveaxis(np.tensordot(F, np.moveaxis(a, axis, 0), axes=(1, 0)), 0, axis)
    if keep is not None:
        out = np.take(out, np.arange(keep), axis=axis)
    return out


def _batch(v):
    return v[None] if v.ndim == 4 else v


def pass_x_forward(x, eps_c=None, mode="A"):
    """X+: (nrhs, 3, n3, n2, n1) -> S1 (nrhs, 3, n3, L1, n2); the A^H mode
    pre-scales by conj(chi) = conj(eps_c) - 1."""
    x = _batch(np.asarray(x, dtype=np.complex128))
    if mode == "AH":
        x = (np.conj(np.asarray(eps_c)) - 1.0)[None, None] * x
    n1 = x.shape[4]
    X = _dft_along(x, 4, 2 * n1, -1)            # (b, q, k, j, i')
    return np.ascontiguousarray(np.swapaxes(X, 3, 4))


def pass_y_forward(S1):
    """Y+: S1 (nrhs, 3, n3, L1, n2) -> S2 (nrhs, 3, L2, L1, n3)."""
    n2 = S1.shape[4]
    Y = _dft_along(S1, 4, 2 * n2, -1)           # (b, q, k, i', j')
    return np.ascontiguousarray(np.transpose(Y, (0, 1, 4, 3, 2)))


def pass_z(S2, nhat, conj=False):
    """Z*: pad along z, DFT, Y_p = sum_q Nh_pq X_q / M (conj(Nh) for the
    adjoint), inverse DFT, keep k < n3.  ``nhat[c]`` has shape (L1, L2, L3)
    (math order), components xx, yy, zz, xy, xz, yz."""
    b, _, L2, L1, n3 = S2.shape
    L3 = 2 * n3
    M = L1 * L2 * L3
    X = _dft_along(S2, 4, L3, -1)               # (b, q, j', i', k3)
    Y = np.zeros_like(X)
    for p in range(3):
        for q in range(3):
            N = np.transpose(nhat[component_index(p, q)], (1, 0, 2)) / M   # (j', i', k3)
            Y[:, p] += (np.conj(N) if conj else N)[None] * X[:, q]
    return _dft_along(Y, 4, L3, +1, keep=n3)


def pass_y_inverse(S2, n2):
    """Y-: S2 (nrhs, 3, L2, L1, n3) -> S3 (nrhs, 3, n3, L1, n2)."""
    L2 = S2.shape[2]
    Y = _dft_along(S2, 2, L2, +1, keep=n2)       # (b, q, j, i', k)
    return np.ascontiguousarray(np.transpose(Y, (0, 1, 4, 3, 2)))


def pass_x_inverse(S3, n1, x=None, eps_c=None, mode="N"):
    """X-: S3 (nrhs, 3, n3, L1, n2) -> (nrhs, 3, n3, n2, n1) with the
    epilogue of eq. 4 for mode A / A^H, none for N / N^H."""
    L1 = S3.shape[3]
    r = _dft_along(S3, 3, L1, +1, keep=n1)       # (b, q, k, i, j)
    r = np.ascontiguousarray(np.swapaxes(r, 3, 4))
    if mode in ("N", "NH"):
        return r
    x = _batch(np.asarray(x, dtype=np.complex128))
    eps = np.asarray(eps_c)[None, None]
    if mode == "A":
        return eps * x - (eps - 1.0) * r
    return np.conj(eps) * x - r


def matvec_by_passes(op, eps_c, x, mode="A"):
    """The five passes in sequence (the whole matvec)."""
    n1, n2, _ = op.n
    conj = mode in ("AH", "NH")
    S1 = pass_x_forward(x, eps_c, mode)
    S2 = pass_y_forward(S1)
    S2 = pass_z(S2, op.nhat, conj)
    S3 = pass_y_inverse(S2, n2)
    return pass_x_inverse(S3, n1, x, eps_c, mode)
