"""Tucker+CP (Sec. IV-B, Alg. 2, eq. 17) in FP64.  Test infrastructure only.

Alg. 2: HOSVD of the defining tensor (Alg. 1), a canonical polyadic (CP)
decomposition of the small Tucker core by alternating least squares (the
usual CP algorithm the paper names), and the Tucker+CP factors
W^i = U^i V^i, so that the tensor is approximated by the sum of R rank-one
terms W^1_l (x) W^2_l (x) W^3_l (eq. 17).

CP by alternating least squares: with the unfolding convention of
``tucker.unfold`` (mode-1 columns ordered (j, k) with k fastest), a CP
tensor has G^(1) = V1 K1^T with K1 = khatri_rao(V2, V3); the least-squares
update of V1 for fixed V2, V3 is G^(1) conj(K1) M1^{-1} with
M1 = (V2^T conj V2) * (V3^T conj V3) (element-wise), and likewise for
modes 2 and 3 in that order.  The start is deterministic: the leading R left
singular vectors of each unfolding of the core; a CP rank R above that
mode's Tucker rank r (allowed: more terms fit the core better) adds columns
of generic deterministic phases (``start_columns``).

Parity pins (tests/test_oracle_cp.py): exact recovery of tensors built from
known rank-R CP factors, rank-one exactness, a fit that never increases over
the sweeps, the Tucker+CP error bound ||A - A_tcp|| <= ||A - A_t|| +
||G - G_cp||, and eq. 17 equal to the CP core multiplied out by the Tucker
factors.
"""
import numpy as np

from .circulant import fourier_factor
from .tucker import hosvd, mode_product, unfold


def khatri_rao(X, Y):
    """Column-wise Kronecker product: K[x * ny + y, l] = X[x, l] Y[y, l]."""
    return (X[:, None, :] * Y[None, :, :]).reshape(X.shape[0] * Y.shape[0], X.shape[1])


def cp_reconstruct(Vs, lam=None):
    """sum_l lam_l V1[:, l] (x) V2[:, l] (x) V3[:, l] (eq. 17 with the Tucker+CP
    factors, eq. 11 of the CP model)."""
    V1, V2, V3 = Vs
    w = np.ones(V1.shape[1]) if lam is None else lam
    return np.einsum("l,il,jl,kl->ijk", w, V1, V2, V3)


GOLDEN = (np.sqrt(5.0) - 1.0) / 2.0


def start_columns(U, R):
    """CP start of one mode: the leading R left singular vectors of the
    unfolding (its r columns); when R > r, columns j = r..R-1 are
    exp(2 pi i frac(g (a + 1) (j + 1))) / sqrt(r) over the rows a, with g
    the golden ratio conjugate (deterministic, generic phases)."""
    r = U.shape[1]
    if R <= r:
        return U[:, :R].copy()
    a = np.arange(U.shape[0], dtype=np.float64)[:, None] + 1.0
    j = np.arange(r, R, dtype=np.float64)[None, :] + 1.0
    ph = np.mod(GOLDEN * a * j, 1.0)
    extra = np.exp(2j * np.pi * ph) / np.sqrt(r)
    return np.concatenate([U, extra], axis=1)


def cp_als(G, R, iters=1000, tol=0.0):
    """CP of G (r1 x r2 x r3) with R terms by alternating least squares.
    Returns ([V1, V2, V3], errors) with the relative Frobenius error after
    every sweep; stops early when a sweep improves it by less than ``tol``."""
    G = np.asarray(G, dtype=np.complex128)
    Vs = []
    for mode in (1, 2, 3):
        U, _, _ = np.linalg.svd(unfold(G, mode), full_matrices=False)
        Vs.append(start_columns(U, R))
    norm = np.linalg.norm(G)
    errs = []
    for _ in range(iters):
        for mode in (1, 2, 3):
            others = [Vs[m - 1] for m in (1, 2, 3) if m != mode]
            K = khatri_rao(others[0], others[1])
            M = (others[0].T @ others[0].conj()) * (others[1].T @ others[1].conj())
            B = unfold(G, mode) @ K.conj()
            Vs[mode - 1] = B @ np.linalg.pinv(M)
        errs.append(np.linalg.norm(G - cp_reconstruct(Vs)) / norm if norm > 0 else 0.0)
        if tol > 0 and len(errs) > 1 and errs[-2] - errs[-1] < tol:
            break
    return Vs, errs


def tucker_cp(A, tol, R=None, iters=1000, rule=0):
    """Alg. 2: HOSVD at ``tol`` then CP of the core with R terms (default
    min(r1, r2, r3)); returns (Ws, G, Us, Vs, errs) with W^i = U^i V^i."""
    G, Us, _ = hosvd(A, tol, rule)
    R = min(G.shape) if R is None else R
    Vs, errs = cp_als(G, R, iters)
    Ws = [U @ V for U, V in zip(Us, Vs)]
    return Ws, G, Us, Vs, errs


def fourier_tensor_cp(Ws, signs):
    """Fourier-domain circulant tensor of the Tucker+CP form: the embedded
    and transformed factor columns (Sec. V-A) combined by eq. 17."""
    Wh = [fourier_factor(W, s) for W, s in zip(Ws, signs)]
    return cp_reconstruct(Wh)


def core_times_factors(Vs, Us):
    """The CP core multiplied out by the Tucker factors,
    (sum_l V1_l (x) V2_l (x) V3_l) x1 U1 x2 U2 x3 U3."""
    Gc = cp_reconstruct(Vs)
    return mode_product(mode_product(mode_product(Gc, Us[0], 1), Us[1], 2), Us[2], 3)
