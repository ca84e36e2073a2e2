"""Tucker model and HOSVD (FP64).  Test infrastructure only.

Index convention: a tensor A is a numpy array indexed A[i, j, k] with
i along x (n1), j along y (n2), k along z (n3) -- the paper's order.  Arrays
from ``vie_inputs`` are stored (n3, n2, n1); use ``from_storage`` /
``to_storage`` to switch.

Parity pins: exact recovery of tensors built from known low-rank factors,
the discarded-singular-value bound on the HOSVD error, rank-1 exactness.
"""
import numpy as np


def from_storage(a):
    """(n3, n2, n1) storage order -> math order A[i, j, k]."""
    return np.ascontiguousarray(np.transpose(a, (2, 1, 0)))


def to_storage(A):
    return np.ascontiguousarray(np.transpose(A, (2, 1, 0)))


def unfold(A, mode):
    """Mode-``mode`` unfolding A^(mode) (Sec. IV-A, Alg. 1, Fig. 2): rows are
    indexed by axis ``mode`` (1, 2 or 3), columns by the other two axes."""
    ax = mode - 1
    return np.moveaxis(A, ax, 0).reshape(A.shape[ax], -1)


def mode_product(A, U, mode):
    """n-mode product B = A x_mode U (App. I, Def. A.3):
    B[.., i, ..] = sum_t A[.., t, ..] U[i, t] along axis ``mode``."""
    ax = mode - 1
    B = np.tensordot(U, A, axes=([1], [ax]))       # new axis first
    return np.moveaxis(B, 0, ax)


def tucker_reconstruct(G, U1, U2, U3):
    """A~ = G x1 U1 x2 U2 x3 U3 (eq. 14), i.e. eq. 13 element-wise."""
    return mode_product(mode_product(mode_product(G, U1, 1), U2, 2), U3, 3)


def truncation_rank(s, tol, rule, fro_norm):
    """Rank kept for one unfolding with singular values ``s`` (descending).

    rule 0 (default): smallest r with sqrt(sum_{k>=r} s_k^2) <= tol/sqrt(3) *
    ||A||_F, so that the three discarded tails together bound the relative
    Frobenius error by tol (the error model of eq. 12).
    rule 1: keep s_k >= tol/sqrt(3) * s_max (the per-value cut printed in
    Alg. 1).
    At least one column is always kept.
    """
    s = np.asarray(s, dtype=np.float64)
    if s.size == 0 or s[0] == 0.0:
        return 1
    if rule == 1:
        return max(1, int(np.sum(s >= tol / np.sqrt(3.0) * s[0])))
    thr2 = (tol / np.sqrt(3.0) * fro_norm) ** 2
    # tail2[r] = sum_{k >= r} s_k^2
    tail2 = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1], [0.0]])
    for r in range(1, s.size + 1):
        if tail2[r] <= thr2:
            return r
    return s.size


def hosvd(A, tol, rule=0):
    """HOSVD (Sec. IV-A, Alg. 1).

    For i = 1, 2, 3 take the SVD of the unfolding A^(i), keep the leading r_i
    left singular vectors as the Tucker factor U^i; the core is
    G = A x1 U1^* x2 U2^* x3 U3^* (conjugate transposes).
    Returns (G, [U1, U2, U3], [s1, s2, s3]) with the full singular-value lists.
    """
    A = np.asarray(A, dtype=np.complex128)
    fro = np.linalg.norm(A)
    Us, svals = [], []
    for mode in (1, 2, 3):
        U, s, _ = np.linalg.svd(unfold(A, mode), full_matrices=False)
        r = truncation_rank(s, tol, rule, fro)
        Us.append(U[:, :r])
        svals.append(s)
    G = A
    for mode, U in zip((1, 2, 3), Us):
        G = mode_product(G, U.conj().T, mode)
    return G, Us, svals


def hosvd_error_bound(svals, ranks):
    """sqrt(sum_i sum_{k >= r_i} s_k^(i)^2): the bound on ||A - A~||_F that
    follows from the orthogonal projections of the HOSVD (the bound behind
    the quasi-optimality statement, eq. 16)."""
    tot = 0.0
    for s, r in zip(svals, ranks):
        tot += float(np.sum(np.asarray(s)[r:] ** 2))
    return np.sqrt(tot)
