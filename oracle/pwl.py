"""Piecewise-linear (PWL) basis: the 12-unknown electric block (FP64).
Test infrastructure only.

Eq. 7a-7b expand each current component in four functions per voxel: the
pulse (l = 0) and the pulse times the normalised local coordinate
(x - x_m)/h, (y - y_m)/h, (z - z_m)/h (l = 1, 2, 3), so there are twelve
unknowns u^{pl}(m) per voxel.  The Galerkin entries of eq. 8a-8b between the
test function (p, l) of voxel m and the basis function (q, l') of voxel m'
depend on the offset m' - m only:

    Z[(p, l, m), (q, l', m')] = Nt^{(l,l')}_pq(m' - m).

The defining tensors hold the ten pairs l <= l' (six components each, 60 in
all, Sec. II-B) at offsets in [0, n1) x [0, n2) x [0, n3).  Every other entry
follows from two facts of the integrals:

* reflecting axis a flips x_a, the a-components of both vectors and the
  linear functions along a, so component (l, l', p, q) is odd along a when
  [p = a] + [q = a] + [l = a + 1] + [l' = a + 1] is odd;
* swapping test and basis function negates the per-axis correlation of a
  pulse with a linear function, so Nt^(l',l) = sigma Nt^(l,l') with
  sigma = -1 when exactly one of l, l' is the pulse.

With rows divided by the voxel volume and the contrast constant in each
voxel, the electric block of eq. 4 acts as

    (A u)^{pl}(m) = eps_c(m) m_l u^{pl}(m)
                    - chi(m) sum_{q, l', m'} Nt^{(l,l')}_pq(m' - m) u^{ql'}(m'),

m_l = (1, 1/12, 1/12, 1/12) the self products of the basis functions and
chi = eps_c - 1.  Vectors are (4, 3, n3, n2, n1) = [l][p][k][j][i] complex.

Three evaluations of the sum: ``brute_force`` (the double sum written out),
``apply`` with ``dense_kernels`` (the convolution kernel of every ordered
block, circulant-embedded and transformed) and ``apply`` with
``tucker_kernels`` (each of the 60 components replaced by its HOSVD
approximation first, Alg. 1).

In the mass-normalised basis (linear functions times sqrt 12, unit self
products) the block is S A S with S = diag(1, sqrt 12, sqrt 12, sqrt 12)
over l; ``to_normalised`` maps an operator application to that basis.
"""
import numpy as np
import scipy.fft as sfft

from .tucker import from_storage, hosvd, to_storage, tucker_reconstruct

PAIRS = ((0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3))
COMPONENTS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
MASS = np.array([1.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0])
SCALE = np.array([1.0, np.sqrt(12.0), np.sqrt(12.0), np.sqrt(12.0)])


def comp_index(p, q):
    return COMPONENTS.index((min(p, q), max(p, q)))


def odd_axes(l, lp, p, q):
    """Axes along which component (l, l', p, q) is odd."""
    return tuple(((p == a) + (q == a) + (l == a + 1) + (lp == a + 1)) % 2 == 1 for a in range(3))


def swap_sign(l, lp):
    """sigma of Nt^(l',l) = sigma Nt^(l,l')."""
    return -1.0 if (l == 0) != (lp == 0) else 1.0


def signed_entry(green, l, lp, p, q, D):
    """Nt^{(l,l')}_pq(D) for any basis pair and signed offset D = (dx, dy, dz);
    ``green`` is the (10, 6, n3, n2, n1) array of the stored pairs."""
    sign = 1.0
    a, b = l, lp
    if l > lp:
        a, b = lp, l
        sign *= swap_sign(l, lp)
    odd = odd_axes(l, lp, p, q)
    for ax in range(3):
        if D[ax] < 0 and odd[ax]:
            sign = -sign
    return sign * green[PAIRS.index((a, b)), comp_index(p, q), abs(D[2]), abs(D[1]), abs(D[0])]


def brute_force(green, u):
    """The Galerkin sum sum_{q, l', m'} Nt^{(l,l')}_pq(m' - m) u^{ql'}(m') (tiny grids)."""
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
                            acc += signed_entry(green, l, lp, p, q, (i2 - i, j2 - j, k2 - k)) * u[lp, q, k2, j2, i2]
                out[l, p, k, j, i] = acc
    return out


def dense_matrix(green):
    """Explicit 12V x 12V matrix of the Galerkin sum, unknowns ordered
    (l, p, k, j, i) as in the storage layout (tiny grids)."""
    n3, n2, n1 = green.shape[2:]
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
                            M[r0 + s, c0 + t] = signed_entry(green, l, lp, p, q, (i2 - i, j2 - j, k2 - k))
    return M


def _kernel(green, l, lp, p, q):
    """Convolution kernel K(E) = Nt^{(l,l')}_pq(-E) of one block (the sum over
    m' is a sum of K(m - m') u(m')), embedded circulantly in (2n1, 2n2, 2n3)
    and transformed (forward FFT, unnormalised).  Index e of an axis of
    length 2n holds the offset E = e (e < n) or e - 2n (e > n); index n, which
    no product of two length-n sequences reaches, is zero."""
    n3, n2, n1 = green.shape[2:]
    a, b = (l, lp) if l <= lp else (lp, l)
    base = from_storage(green[PAIRS.index((a, b)), comp_index(p, q)])
    sign0 = swap_sign(l, lp) if l > lp else 1.0
    odd = odd_axes(l, lp, p, q)
    idx, sgn, keep = [], [], []
    for ax, n in enumerate((n1, n2, n3)):
        e = np.arange(2 * n)
        E = np.where(e < n, e, e - 2 * n)
        D = -E                                   # the entry is taken at -E
        idx.append(np.abs(D) % n)
        sgn.append(np.where((D < 0) & odd[ax], -1.0, 1.0))
        keep.append(e != n)
    K = base[np.ix_(idx[0], idx[1], idx[2])]
    K = K * (sign0 * sgn[0][:, None, None] * sgn[1][None, :, None] * sgn[2][None, None, :])
    K = K * (keep[0][:, None, None] & keep[1][None, :, None] & keep[2][None, None, :])
    return np.fft.fftn(K)


def dense_kernels(green):
    """Fourier-domain kernels of all ordered blocks: khat[l][l'][p][q]."""
    return [[[[_kernel(green, l, lp, p, q) for q in range(3)] for p in range(3)] for lp in range(4)]
            for l in range(4)]


def tucker_tensors(green, tol, rule=0):
    """The 60 defining tensors, each replaced by its HOSVD approximation at
    ``tol`` (Alg. 1; the zero planes of an odd component are imposed first).
    Returns the approximated tensors (storage layout) and the ranks."""
    out = np.empty_like(green)
    ranks = np.zeros((10, 6, 3), dtype=int)
    for P, (l, lp) in enumerate(PAIRS):
        for c, (p, q) in enumerate(COMPONENTS):
            A = from_storage(green[P, c]).copy()
            odd = odd_axes(l, lp, p, q)
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


def tucker_kernels(green, tol, rule=0):
    """Fourier-domain kernels of the HOSVD-approximated tensors, and the ranks."""
    approx, ranks = tucker_tensors(green, tol, rule)
    return dense_kernels(approx), ranks


def apply(khat, u, adjoint=False):
    """The Galerkin sum by zero padding, FFT, the 12 x 12 product per
    frequency and inverse FFT.  ``adjoint``: the conjugate transpose of the
    sum."""
    n3, n2, n1 = u.shape[2:]
    L = (2 * n1, 2 * n2, 2 * n3)
    Xh = np.empty((4, 3) + L, dtype=np.complex128)
    for lp in range(4):
        for q in range(3):
            pad = np.zeros(L, dtype=np.complex128)
            pad[:n1, :n2, :n3] = from_storage(u[lp, q])
            Xh[lp, q] = sfft.fftn(pad)
    out = np.empty(u.shape, dtype=np.complex128)
    for l in range(4):
        for p in range(3):
            Yh = np.zeros(L, dtype=np.complex128)
            for lp in range(4):
                for q in range(3):
                    if adjoint:
                        # the adjoint's kernel is conj(K_(l'q, lp)(-E)),
                        # whose transform is conj(K^_(l'q, lp))
                        K = np.conj(khat[lp][l][q][p])
                    else:
                        K = khat[l][lp][p][q]
                    Yh += K * Xh[lp, q]
            out[l, p] = to_storage(sfft.ifftn(Yh)[:n1, :n2, :n3])
    return out


def matvec(khat, eps_c, u, mode="A"):
    """Electric block in the paper's PWL basis.

    mode 'A' : eps_c m_l u - chi (sum u)
    mode 'AH': conj(eps_c) m_l u - sum^H (conj(chi) u)      (adjoint of 'A')
    mode 'N' : the bare sum,  mode 'NH': its adjoint
    """
    if mode == "N":
        return apply(khat, u)
    if mode == "NH":
        return apply(khat, u, adjoint=True)
    eps_c = np.asarray(eps_c)
    chi = eps_c - 1.0
    m = MASS[:, None, None, None, None]
    if mode == "A":
        return eps_c[None, None] * m * u - chi[None, None] * apply(khat, u)
    if mode == "AH":
        return np.conj(eps_c)[None, None] * m * u - apply(khat, np.conj(chi)[None, None] * u, adjoint=True)
    raise ValueError(mode)


def to_normalised(op, u):
    """Apply ``op`` (a function of paper-basis coefficients) in the
    mass-normalised basis: S op(S u)."""
    S = SCALE[:, None, None, None, None]
    return S * op(S * u)


def sampled_outputs(green, eps_c, u, samples):
    """(A u)^{pl}(m) at the sampled (l, p, k, j, i) one by one, each as the
    Galerkin sum written out over every basis function of the grid (the
    offsets D = m' - m of all m', with the parities and the pair swap of the
    stored tensors): for grids too large for ``dense_kernels``."""
    n3, n2, n1 = u.shape[2:]
    out = []
    for (l, p, k, j, i) in samples:
        acc = 0j
        for lp in range(4):
            for q in range(3):
                a, b = (l, lp) if l <= lp else (lp, l)
                sign0 = swap_sign(l, lp) if l > lp else 1.0
                odd = odd_axes(l, lp, p, q)
                T = green[PAIRS.index((a, b)), comp_index(p, q)]
                D = [np.arange(n1) - i, np.arange(n2) - j, np.arange(n3) - k]
                sg = [np.where((d < 0) & o, -1.0, 1.0) for d, o in zip(D, odd)]
                vals = T[np.ix_(np.abs(D[2]), np.abs(D[1]), np.abs(D[0]))]
                vals = vals * (sign0 * sg[2][:, None, None] * sg[1][None, :, None] * sg[0][None, None, :])
                acc += np.sum(vals * u[lp, q])
        e = eps_c[k, j, i]
        out.append(e * MASS[l] * u[l, p, k, j, i] - (e - 1.0) * acc)
    return np.array(out)
