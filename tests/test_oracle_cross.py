"""Pins of the oracle's Tucker cross approximation (oracle/cross.py, the
cross-Tucker compression named in Sec. IV-A) against facts that do not come
from the oracle itself: exact recovery of tensors of known multilinear rank,
the maxvol dominance property, interpolation of the fibers it read, the
count of entries read, and agreement with the dense Green's tensor within
the tolerance (its HOSVD as the yardstick)."""
import numpy as np
import pytest

import vie_inputs as vi
from oracle import circulant, cross, tucker

F = 298e6
K0 = vi.wavenumber(F)


def _low_rank(n, r, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal(r) + 1j * rng.standard_normal(r)
    Us = [rng.standard_normal((n[a], r[a])) + 1j * rng.standard_normal((n[a], r[a])) for a in range(3)]
    return tucker.tucker_reconstruct(G, *Us)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n,r", [((20, 24, 28), (3, 4, 5)), ((40, 9, 33), (6, 2, 7)), ((17, 17, 17), (1, 1, 1))])
def test_exact_recovery_of_known_multilinear_rank(n, r):
    A = _low_rank(n, r, sum(n))
    G, Us, info = cross.tucker_cross(cross.dense_entries(A), n, 1e-10)
    assert G.shape == r
    assert _rel(tucker.tucker_reconstruct(G, *Us), A) <= 1e-12
    # factors are orthonormal (the recompression's QR and HOSVD)
    for U in Us:
        assert np.allclose(U.conj().T @ U, np.eye(U.shape[1]), atol=1e-12)
    # linear cost: only fibers through the index sets were read
    assert info["evals"] < A.size


def test_entries_read_grow_linearly_with_n():
    evals = []
    for m in (40, 80, 160):
        n = (m, m, m)
        A = _low_rank(n, (4, 4, 4), 7)
        _, _, info = cross.tucker_cross(cross.dense_entries(A), n, 1e-10)
        evals.append(info["evals"])
    # doubling n roughly doubles the entries read (an n^3 method would take 8x)
    assert evals[1] / evals[0] < 3.0 and evals[2] / evals[1] < 3.0


def test_maxvol_dominance_and_a_planted_maximum():
    rng = np.random.default_rng(3)
    U = rng.standard_normal((50, 6)) + 1j * rng.standard_normal((50, 6))
    rows = cross.maxvol(U)
    assert len(set(rows.tolist())) == 6
    B = U @ np.linalg.inv(U[rows])
    assert np.abs(B).max() <= 1.05 + 1e-12
    # rows that are 10x the identity dominate every other row (entries <= 0.1
    # after division), so the maximum-volume rows are exactly those
    V = 0.1 * (rng.standard_normal((40, 4)) + 1j * rng.standard_normal((40, 4))) / 4
    planted = [5, 17, 23, 31]
    V[planted] = 10 * np.eye(4)
    assert sorted(cross.maxvol(V).tolist()) == planted


def test_greedy_rows_are_the_pivots_of_a_pivoted_qr():
    import scipy.linalg
    rng = np.random.default_rng(5)
    U = rng.standard_normal((30, 5)) + 1j * rng.standard_normal((30, 5))
    _, _, piv = scipy.linalg.qr(U.T, pivoting=True)
    assert cross.greedy_rows(U) == piv[:5].tolist()


def test_interpolation_of_the_fibers_read():
    # before recompression the cross form equals A on every fiber through
    # the final index sets; after it, on those fibers up to the tolerance
    n = (30, 26, 22)
    A = _low_rank(n, (5, 5, 5), 11) + 1e-3 * _low_rank(n, (9, 9, 9), 12)
    G, Us, info = cross.tucker_cross(cross.dense_entries(A), n, 1e-12)
    B = tucker.tucker_reconstruct(G, *Us)
    J = info["index_sets"]
    for m in range(3):
        sl = [np.array(J[0]), np.array(J[1]), np.array(J[2])]
        sl[m] = np.arange(n[m])
        ix = np.ix_(*sl)
        assert _rel(B[ix], A[ix]) <= 1e-10


def test_start_indices_are_evenly_spaced():
    assert cross.start_indices(10, 4).tolist() == [1, 3, 6, 8]
    assert cross.start_indices(3, 4).tolist() == [0, 1, 2]


@pytest.mark.parametrize("n,h", [((32, 32, 32), 0.005), ((48, 40, 36), 0.004)])
@pytest.mark.parametrize("tol", [1e-6, 1e-8])
@pytest.mark.parametrize("c", [0, 3, 5])
def test_green_tensor_within_tolerance_like_the_hosvd(n, h, tol, c):
    Gd = vi.green_tensor(n, h, K0)
    odd = [s < 0 for s in circulant.axis_signs(c)]
    A = tucker.from_storage(Gd[c])
    A0 = A.copy()
    for ax in range(3):
        if odd[ax]:
            sl = [slice(None)] * 3
            sl[ax] = 0
            A0[tuple(sl)] = 0
    # entries from the entry-wise generator, not from the dense array
    fn = cross.green_entries(lambda i, j, k: vi.green_entries(np.stack([i, j, k], -1), c, h, K0), odd)
    G, Us, info = cross.tucker_cross(fn, n, tol)
    err = _rel(tucker.tucker_reconstruct(G, *Us), A0)
    Gh, Uh, _ = tucker.hosvd(A0, tol)
    err_h = _rel(tucker.tucker_reconstruct(Gh, *Uh), A0)
    assert err <= tol
    assert err <= 1.2 * err_h
    assert all(abs(a - b) <= 1 for a, b in zip(G.shape, Gh.shape))
    # the odd component's parity zeros hold in the form (up to rounding)
    B = tucker.tucker_reconstruct(G, *Us)
    for ax in range(3):
        if odd[ax]:
            assert np.linalg.norm(np.take(B, 0, axis=ax)) <= 1e-12 * np.linalg.norm(A0)


def test_entry_generator_equals_the_dense_tensor():
    n = (11, 9, 7)
    h = 0.004
    G = vi.green_tensor(n, h, K0)
    rng = np.random.default_rng(2)
    idx = np.stack([rng.integers(0, n[a], 200) for a in range(3)], axis=1)
    idx[:8] = [[0, 0, 0], [1, 0, 0], [0, 1, 1], [1, 1, 1], [2, 0, 0], [10, 8, 6], [0, 8, 0], [2, 2, 2]]
    for c in range(6):
        assert np.array_equal(vi.green_entries(idx, c, h, K0), G[c][idx[:, 2], idx[:, 1], idx[:, 0]])
