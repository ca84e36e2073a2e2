"""Piecewise-linear (PWL) basis: the magnetic operator K (FP64).
Test infrastructure only.

K of eq. 5 (the curl of the single-layer potential) between the test
function (p, l) of voxel m and the basis function (q, l') of voxel m', rows
divided by the voxel volume, depends on the offset m - m' (observation minus
source, as for the pulse K):

    Z[(p, l, m), (q, l', m')] = Kt^{(l,l')}_pq(m - m'),   Kt_pq = eps_psq F_s,

with l, l' the four functions of eq. 7b per voxel (pulse, and the pulse
times the normalised local x, y, z).  The defining tensors hold the ten
pairs l <= l' and the three components xy, xz, yz (30 in all) at offsets in
[0, n1) x [0, n2) x [0, n3).  Every other entry follows from:

* the Levi-Civita symbol: zero diagonal, Kt_qp = -Kt_pq;
* reflecting axis a: component xy, xz or yz (the derivative axis s missing
  from the pair) of pair (l, l') is odd along a when
  [s = a] + [l = a + 1] + [l' = a + 1] is odd;
* swapping test and basis function: Kt^(l',l) = sigma Kt^(l,l'), sigma = -1
  when exactly one of l, l' is the pulse (as for N).

The sum applied is the bare K of eq. 4's coupling blocks (no contrast, no
h or frequency factor):

    y^{pl}(m) = sum_{q, l', m'} Kt^{(l,l')}_pq(m - m') u^{ql'}(m'),

vectors (4, 3, n3, n2, n1) = [l][p][k][j][i].  ``brute_force_k`` writes the
double sum out, ``pwl.apply`` with ``dense_kernels_k`` (or ``tucker_kernels_k``)
evaluates it through the circulant embedding of every ordered block.
"""
import numpy as np

from .pwl import PAIRS, SCALE, apply, swap_sign
from .tucker import from_storage, hosvd, to_storage, tucker_reconstruct

K_COMPONENTS = ((0, 1), (0, 2), (1, 2))


def k_deriv_axis(c):
    """The derivative axis s of stored component c (xy: z, xz: y, yz: x)."""
    return 2 - c


def k_odd_axes(l, lp, c):
    """Axes along which stored component c of the pair (l, l') is odd."""
    s = k_deriv_axis(c)
    return tuple(((s == a) + (l == a + 1) + (lp == a + 1)) % 2 == 1 for a in range(3))


def signed_entry_k(kt, l, lp, p, q, D):
    """Kt^{(l,l')}_pq(D) for any basis pair, any (p, q) and signed offset
    D = (dx, dy, dz); ``kt`` is the (10, 3, n3, n2, n1) array of the stored
    pairs and components."""
    if p == q:
        return 0j
    sign = 1.0
    if p > q:
        p, q = q, p
        sign = -sign
    a, b = l, lp
    if l > lp:
        a, b = lp, l
        sign *= swap_sign(l, lp)
    c = K_COMPONENTS.index((p, q))
    odd = k_odd_axes(l, lp, c)
    for ax in range(3):
        if D[ax] < 0 and odd[ax]:
            sign = -sign
    return sign * kt[PAIRS.index((a, b)), c, abs(D[2]), abs(D[1]), abs(D[0])]


def brute_force_k(kt, u):
    """sum_{q, l', m'} Kt^{(l,l')}_pq(m - m') u^{ql'}(m') written out (tiny grids)."""
    n3, n2, n1 = u.shape[2:]
    idx = [(i, j, k) for k in range(n3) for j in range(n2) for i in range(n1)]
    out = np.zeros(u.shape, dtype=np.complex128)
    for l in range(4):
        for p in range(3):
            for (i, j, k) in idx:
                acc = 0j
                for lp in range(4):
                    for q in range(3):
                        for (i2, j2, k2) in idx:
                            acc += signed_entry_k(kt, l, lp, p, q, (i - i2, j - j2, k - k2)) * u[lp, q, k2, j2, i2]
                out[l, p, k, j, i] = acc
    return out


def dense_matrix_k(kt):
    """Explicit 12V x 12V matrix of the sum, unknowns ordered (l, p, k, j, i)
    (tiny grids)."""
    n3, n2, n1 = kt.shape[2:]
    V = n1 * n2 * n3
    idx = [(i, j, k) for k in range(n3) for j in range(n2) for i in range(n1)]
    M = np.zeros((12 * V, 12 * V), dtype=np.complex128)
    for l in range(4):
        for p in range(3):
            for lp in range(4):
                for q in range(3):
                    r0, c0 = (3 * l + p) * V, (3 * lp + q) * V
                    for s, (i, j, k) in enumerate(idx):
                        for t, (i2, j2, k2) in enumerate(idx):
                            M[r0 + s, c0 + t] = signed_entry_k(kt, l, lp, p, q, (i - i2, j - j2, k - k2))
    return M


def _kernel_k(kt, l, lp, p, q):
    """Convolution kernel K(E) = Kt^{(l,l')}_pq(E) of one block, embedded
    circulantly in (2n1, 2n2, 2n3) (index e of an axis of length 2n is the
    offset e for e < n, e - 2n for e > n, zero at e = n) and transformed."""
    n3, n2, n1 = kt.shape[2:]
    L = (2 * n1, 2 * n2, 2 * n3)
    if p == q:
        return np.zeros(L, dtype=np.complex128)
    sign0 = 1.0
    pp, qq = (p, q) if p < q else (q, p)
    if p > q:
        sign0 = -sign0
    a, b = (l, lp) if l <= lp else (lp, l)
    if l > lp:
        sign0 *= swap_sign(l, lp)
    c = K_COMPONENTS.index((pp, qq))
    base = from_storage(kt[PAIRS.index((a, b)), c])
    odd = k_odd_axes(l, lp, c)
    idx, sgn, keep = [], [], []
    for ax, n in enumerate((n1, n2, n3)):
        e = np.arange(2 * n)
        E = np.where(e < n, e, e - 2 * n)
        idx.append(np.abs(E) % n)
        sgn.append(np.where((E < 0) & odd[ax], -1.0, 1.0))
        keep.append(e != n)
    K = base[np.ix_(idx[0], idx[1], idx[2])]
    K = K * (sign0 * sgn[0][:, None, None] * sgn[1][None, :, None] * sgn[2][None, None, :])
    K = K * (keep[0][:, None, None] & keep[1][None, :, None] & keep[2][None, None, :])
    return np.fft.fftn(K)


def dense_kernels_k(kt):
    """Fourier-domain kernels of all ordered blocks, khat[l][l'][p][q], in the
    form ``pwl.apply`` takes."""
    return [[[[_kernel_k(kt, l, lp, p, q) for q in range(3)] for p in range(3)] for lp in range(4)]
            for l in range(4)]


def tucker_tensors_k(kt, tol, rule=0):
    """The 30 defining tensors, each replaced by its HOSVD approximation at
    ``tol`` (Alg. 1; the zero planes of an odd component imposed first).
    Returns the approximated tensors (storage layout) and the ranks."""
    out = np.empty_like(kt)
    ranks = np.zeros((10, 3, 3), dtype=int)
    for P, (l, lp) in enumerate(PAIRS):
        for c in range(3):
            A = from_storage(kt[P, c]).copy()
            odd = k_odd_axes(l, lp, c)
            if odd[0]:
                A[0, :, :] = 0
            if odd[1]:
                A[:, 0, :] = 0
            if odd[2]:
                A[:, :, 0] = 0
            G, Us, _ = hosvd(A, tol, rule)
            ranks[P, c] = [U.shape[1] for U in Us]
            out[P, c] = to_storage(tucker_reconstruct(G, *Us))
    return out, ranks


def tucker_kernels_k(kt, tol, rule=0):
    """Fourier-domain kernels of the HOSVD-approximated tensors, and the ranks."""
    approx, ranks = tucker_tensors_k(kt, tol, rule)
    return dense_kernels_k(approx), ranks


def sampled_outputs_k(kt, u, samples):
    """y^{pl}(m) at the sampled (l, p, k, j, i) one by one, each as the sum
    over every basis function of the grid written out (offsets D = m - m'):
    for grids too large for ``dense_kernels_k``."""
    n3, n2, n1 = u.shape[2:]
    out = []
    for (l, p, k, j, i) in samples:
        acc = 0j
        for lp in range(4):
            for q in range(3):
                if p == q:
                    continue
                sign0 = 1.0
                pp, qq = (p, q) if p < q else (q, p)
                if p > q:
                    sign0 = -sign0
                a, b = (l, lp) if l <= lp else (lp, l)
                if l > lp:
                    sign0 *= swap_sign(l, lp)
                c = K_COMPONENTS.index((pp, qq))
                odd = k_odd_axes(l, lp, c)
                T = kt[PAIRS.index((a, b)), c]
                D = [i - np.arange(n1), j - np.arange(n2), k - np.arange(n3)]
                sg = [np.where((d < 0) & o, -1.0, 1.0) for d, o in zip(D, odd)]
                vals = T[np.ix_(np.abs(D[2]), np.abs(D[1]), np.abs(D[0]))]
                vals = vals * (sign0 * sg[2][:, None, None] * sg[1][None, :, None] * sg[0][None, None, :])
                acc += np.sum(vals * u[lp, q])
        out.append(acc)
    return np.array(out)


def to_normalised_k(khat, u):
    """The sum in the mass-normalised basis (linear functions times sqrt 12):
    S K S u."""
    S = SCALE[:, None, None, None, None]
    return S * apply(khat, S * u)
