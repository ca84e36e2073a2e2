"""Pins of the oracle's Tucker model and HOSVD (Sec. III-IV, Alg. 1)."""
import numpy as np
import pytest

from oracle import tucker
from vie_inputs import random_complex


def _unitary(n, r, seed):
    q, _ = np.linalg.qr(random_complex((n, r), seed))
    return q


def _low_rank(shape, ranks, seed):
    G = random_complex(ranks, seed)
    Us = [_unitary(n, r, seed + 1 + a) for a, (n, r) in enumerate(zip(shape, ranks))]
    A = np.einsum("abc,ia,jb,kc->ijk", G, Us[0], Us[1], Us[2])
    return A, G, Us


def test_mode_product_definition():
    # App. I, Def. A.3 written as an explicit triple loop on a tiny case
    A = random_complex((2, 3, 4), 1)
    U = random_complex((5, 3), 2)
    B = tucker.mode_product(A, U, 2)
    ref = np.zeros((2, 5, 4), dtype=complex)
    for i in range(2):
        for j in range(5):
            for k in range(4):
                ref[i, j, k] = sum(A[i, t, k] * U[j, t] for t in range(3))
    np.testing.assert_allclose(B, ref, rtol=1e-14)


def test_exact_low_rank_recovery():
    # a tensor of multilinear rank (5, 7, 9) on 16 x 20 x 24 is recovered
    # exactly with exactly those ranks
    A, _, _ = _low_rank((16, 20, 24), (5, 7, 9), 10)
    G, Us, s = tucker.hosvd(A, 1e-12)
    assert [U.shape[1] for U in Us] == [5, 7, 9]
    At = tucker.tucker_reconstruct(G, *Us)
    assert np.linalg.norm(A - At) <= 1e-13 * np.linalg.norm(A)
    # factors are orthonormal
    for U in Us:
        np.testing.assert_allclose(U.conj().T @ U, np.eye(U.shape[1]), atol=1e-13)


def test_rank_one_separable_exact():
    a, b, c = random_complex(6, 1), random_complex(7, 2), random_complex(8, 3)
    A = np.einsum("i,j,k->ijk", a, b, c)
    G, Us, _ = tucker.hosvd(A, 1e-10)
    assert [U.shape[1] for U in Us] == [1, 1, 1]
    np.testing.assert_allclose(tucker.tucker_reconstruct(G, *Us), A, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("tol", [1e-2, 1e-4, 1e-6])
def test_error_bound_and_tolerance(tol):
    # a tensor with geometrically decaying multilinear spectrum
    rng = np.random.default_rng(5)
    n = (18, 15, 12)
    A = np.zeros(n, dtype=complex)
    for t in range(12):
        vecs = [random_complex(m, 100 + 3 * t + a) for a, m in enumerate(n)]
        A += 0.3 ** t * np.einsum("i,j,k->ijk", *vecs)
    A += 1e-9 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    G, Us, s = tucker.hosvd(A, tol)
    ranks = [U.shape[1] for U in Us]
    err = np.linalg.norm(A - tucker.tucker_reconstruct(G, *Us))
    bound = tucker.hosvd_error_bound(s, ranks)
    assert err <= bound * (1 + 1e-12) + 1e-15
    assert bound <= tol * np.linalg.norm(A) * (1 + 1e-12)     # rule 0 guarantee
    # each dropped tail is within its share tol/sqrt(3) ||A||
    for si, r in zip(s, ranks):
        assert np.sqrt(np.sum(si[r:] ** 2)) <= tol / np.sqrt(3) * np.linalg.norm(A) * (1 + 1e-12)
        if r > 1:   # and keeping one fewer column would break it
            assert np.sqrt(np.sum(si[r - 1:] ** 2)) > tol / np.sqrt(3) * np.linalg.norm(A)


def test_error_monotone_in_tolerance():
    rng = np.random.default_rng(7)
    A = np.cumsum(np.cumsum(rng.standard_normal((14, 13, 12)), axis=0), axis=1) + 0j
    errs, sizes = [], []
    for tol in (1e-1, 1e-2, 1e-3, 1e-4):
        G, Us, _ = tucker.hosvd(A, tol)
        errs.append(np.linalg.norm(A - tucker.tucker_reconstruct(G, *Us)))
        sizes.append(G.size)
    assert all(e1 >= e2 for e1, e2 in zip(errs, errs[1:]))
    assert all(s1 <= s2 for s1, s2 in zip(sizes, sizes[1:]))


def test_literal_rule_keeps_values_above_cut():
    s = np.array([1.0, 0.5, 1e-3, 1e-7, 1e-9])
    assert tucker.truncation_rank(s, 1e-6 * np.sqrt(3), 1, None) == 3
