"""Tucker cross approximation (FP64).  Test infrastructure only.

Sec. IV-A names a second way to reach the Tucker form of eq. 13-14: a
cross-Tucker algorithm (Oseledets, Savostyanov, Tyrtyshnikov 2008; Rakhuba,
Oseledets 2015) that reads only some fibers of the tensor, at a cost linear
in n (O(n r1 r2 r3)) against the O(n^3) of the HOSVD, and that rests on the
2-D (matrix) cross approximation (Goreinov et al.).  The paper gives no
steps; the reading taken here is the alternating fiber scheme of those
references, written out plainly:

1. Index sets J1, J2, J3 (one per mode) start as a few evenly spaced indices.
2. Sweep over the modes m = 1, 2, 3: take every mode-m fiber through the
   index pairs of the other two sets, C_m = A(:, J_a, J_b) unfolded to
   n_m x (|J_a| |J_b|); its SVD gives the rank r_m by the truncation rule of
   the HOSVD (relative to the fibers' own Frobenius norm), and J_m becomes
   the maxvol rows of the leading min(r_m + p, rank) left singular vectors
   (p = 8 extra columns let the sets grow while the rank is still rising,
   and give the interpolation enough fibers through the smooth far field:
   with p = 2 the 256^3 Green's tensor at tol 1e-6 came out 7x the tolerance
   in Frobenius norm and 8e-3 off in its sum, with p = 8 as accurate as the
   HOSVD in both).
3. Stop when a sweep leaves every index set unchanged (or after a sweep
   limit).
4. Interpolation form: A ~= A(J1, J2, J3) x1 B1 x2 B2 x3 B3 with
   B_m = U_m U_m[J_m]^{-1}, U_m the singular vectors J_m was last chosen
   from (exact for tensors whose fibers span the true column spaces).
5. Recompression: B_m = Q_m R_m (QR), core A(J) x_m R_m, HOSVD of that
   small core at the same tolerance (Alg. 1), factors Q_m V_m: a Tucker form
   with orthonormal factors and tolerance-based ranks, as the HOSVD gives.

``maxvol`` is the square maxvol row selection (Goreinov et al.): start from
the pivots of a column-pivoted QR of U^T, then swap rows while some entry of
U U[I]^{-1} exceeds 1 + delta in modulus (each swap multiplies |det U[I]| by
that entry; the largest entry, the first in row-major order on ties).

Pins (tests/test_oracle_cross.py): exact recovery of tensors of known
multilinear rank with far fewer entries read than n1 n2 n3; the maxvol
dominance property; interpolation of the chosen fibers; agreement with the
HOSVD and with the dense tensor on Green's tensors within a small multiple
of the tolerance; the count of entries read.
"""
import numpy as np

from .tucker import hosvd, mode_product, truncation_rank


def maxvol(U, delta=0.05, max_swaps=1000):
    """Rows I (len r) of a tall n x r matrix U of full column rank such that
    every entry of U U[I]^{-1} has modulus <= 1 + delta."""
    U = np.asarray(U)
    n, r = U.shape
    if r == 0:
        return np.zeros(0, dtype=np.int64)
    rows = greedy_rows(U)
    for _ in range(max_swaps):
        B = U @ np.linalg.inv(U[rows])
        i, j = np.unravel_index(np.argmax(np.abs(B)), B.shape)
        if abs(B[i, j]) <= 1.0 + delta:
            break
        rows[j] = int(i)
    return np.array(rows, dtype=np.int64)


def greedy_rows(U):
    """The pivot rows of a column-pivoted QR of U^T (Businger-Golub): r times
    take the row of largest residual norm (the first on ties), then remove
    its direction from every row."""
    Rm = np.array(U, dtype=np.complex128)
    rows = []
    for _ in range(U.shape[1]):
        norms = np.sum(np.abs(Rm) ** 2, axis=1)
        norms[rows] = -1.0
        i = int(np.argmax(norms))
        rows.append(i)
        q = Rm[i] / np.sqrt(norms[i])
        Rm = Rm - np.outer(Rm @ q.conj(), q)
    return rows


def start_indices(n, s):
    """Deterministic start of an index set: s evenly spaced indices
    floor((t + 1/2) n / s), t < s."""
    s = min(n, s)
    return np.array([((2 * t + 1) * n) // (2 * s) for t in range(s)], dtype=np.int64)


def _fibers(entries, n, m, Ja, Jb):
    """Mode-m fibers through every (Ja x Jb) pair, as an n_m x (|Ja||Jb|)
    matrix (columns ordered with the later set fastest)."""
    a, b = [x for x in range(3) if x != m]
    t = np.arange(n[m])
    ga, gb = np.meshgrid(Ja, Jb, indexing="ij")
    ga, gb = ga.ravel(), gb.ravel()
    idx = [None, None, None]
    idx[m] = t[:, None]
    idx[a] = ga[None, :]
    idx[b] = gb[None, :]
    return np.asarray(entries(*np.broadcast_arrays(*idx)), dtype=np.complex128)


def tucker_cross(entries, n, tol, rule=0, oversample=8, start=2, max_sweeps=8):
    """Tucker form (G, [U1, U2, U3]) of the n1 x n2 x n3 tensor whose entries
    ``entries(i, j, k)`` returns for integer index arrays of equal shape.
    Returns (G, Us, info) with info = dict(evals, sweeps, index_sets,
    cross_ranks)."""
    n = tuple(int(v) for v in n)
    J = [start_indices(n[m], start + oversample) for m in range(3)]
    U = [None, None, None]
    evals = 0
    cross_ranks = [0, 0, 0]
    sweeps = 0
    for sweep in range(max_sweeps):
        sweeps = sweep + 1
        old = [j.copy() for j in J]
        for m in range(3):
            a, b = [x for x in range(3) if x != m]
            C = _fibers(entries, n, m, J[a], J[b])
            evals += C.size
            Uc, s, _ = np.linalg.svd(C, full_matrices=False)
            fro = np.linalg.norm(C)
            r = truncation_rank(s, tol, rule, fro) if fro > 0 else 1
            numerical = int(np.sum(s > s[0] * 1e-14)) if s.size and s[0] > 0 else 1
            k = max(1, min(r + oversample, numerical))
            cross_ranks[m] = r
            U[m] = Uc[:, :k]
            J[m] = np.sort(maxvol(U[m]))
        if sweep > 0 and all(np.array_equal(o, j) for o, j in zip(old, J)):
            break
    # interpolation form: each U_m is the factor its index set J_m was
    # chosen from, so U_m[J_m] is the nonsingular maxvol submatrix
    core = np.asarray(entries(*np.meshgrid(J[0], J[1], J[2], indexing="ij")), dtype=np.complex128)
    evals += core.size
    Bs = [U[m] @ np.linalg.inv(U[m][J[m]]) for m in range(3)]
    # recompression (step 5)
    Qs = []
    for m in range(3):
        Q, R = np.linalg.qr(Bs[m])
        Qs.append(Q)
        core = mode_product(core, R, m + 1)
    G, Vs, _ = hosvd(core, tol, rule)
    Us = [Qs[m] @ Vs[m] for m in range(3)]
    info = {"evals": int(evals), "sweeps": sweeps, "index_sets": [j.tolist() for j in J],
            "cross_ranks": list(cross_ranks)}
    return G, Us, info


def dense_entries(A):
    """``entries`` callable of a dense tensor A[i, j, k] (math order)."""
    A = np.asarray(A)
    return lambda i, j, k: A[i, j, k]


def green_entries(green_component_fn, odd):
    """``entries`` of one defining Green's component from an entry-wise
    generator ``green_component_fn(i, j, k)``, with the parity zeros of an
    odd component (zero at offset 0 along each axis where it is odd)."""
    def f(i, j, k):
        v = np.asarray(green_component_fn(i, j, k), dtype=np.complex128)
        zero = np.zeros(v.shape, dtype=bool)
        for ax, idx in enumerate((i, j, k)):
            if odd[ax]:
                zero |= np.asarray(idx) == 0
        return np.where(zero, 0.0, v)
    return f
