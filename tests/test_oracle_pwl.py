"""Pins of the oracle's piecewise-linear electric block (oracle/pwl.py)
against the definition of the Galerkin sum, the pulse-basis oracle, the
symmetry of the Galerkin matrix and the generator's direct evaluation of
signed offsets."""
import numpy as np
import pytest

from oracle import pwl
from oracle.operator import apply_N, dense_operator
from vie_inputs import green_pwl_entry, green_pwl_tensor, random_complex

from test_inputs_pwl import _brute6


def _vec(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("n", [(3, 2, 2), (1, 2, 3), (2, 3, 1)])
def test_fft_sum_matches_brute_force(n):
    g = green_pwl_tensor(n, 1.0, 0.4)
    u = _vec((4, 3, n[2], n[1], n[0]), 3)
    np.testing.assert_allclose(pwl.apply(pwl.dense_kernels(g), u), pwl.brute_force(g, u), rtol=0, atol=1e-13)


def test_galerkin_matrix_is_complex_symmetric():
    # reciprocity: the Galerkin matrix of the symmetric operator N equals its
    # transpose; it fixes the signs that relate the stored pairs to the others
    g = green_pwl_tensor((3, 2, 2), 1.0, 0.6)
    M = pwl.dense_matrix(g)
    np.testing.assert_allclose(M, M.T, rtol=0, atol=1e-14)
    assert np.abs(M).max() > 0.1


def test_signed_entries_match_direct_evaluation():
    # negative offsets against the generator's direct evaluation there, and
    # pairs l > l' against a 6-D integral over the two voxels
    kappa, n = 0.3, (4, 3, 3)
    g = green_pwl_tensor(n, 1.0, kappa, near_order=16)
    for D in [(-1, 0, 1), (2, -1, -2), (-3, -2, 0), (-1, -1, -1)]:
        E = green_pwl_entry(D, kappa, 16, method=0)
        for P, (l, lp) in enumerate(pwl.PAIRS):
            for c, (p, q) in enumerate(pwl.COMPONENTS):
                assert abs(pwl.signed_entry(g, l, lp, p, q, D) - E[P, c]) < 1e-10, (D, P, c)
    D = (3, -2, 1)
    gb = green_pwl_tensor((4, 3, 2), 1.0, kappa)
    B = _brute6(D, kappa)
    for l in range(4):
        for lp in range(4):
            for c, (p, q) in enumerate(pwl.COMPONENTS):
                v = pwl.signed_entry(gb, l, lp, p, q, D)
                assert abs(v - B[l, lp, c]) < 1e-8 * np.abs(B[l, lp]).max(), (l, lp, c)


def test_pulse_unknowns_reduce_to_the_pulse_operator():
    # with only pulse coefficients the pulse rows are the PWC operator of the
    # (pulse, pulse) tensor, evaluated by the independent PWC oracle
    n = (5, 4, 3)
    g = green_pwl_tensor(n, 1.0, 0.5)
    u = np.zeros((4, 3, n[2], n[1], n[0]), complex)
    u[0] = _vec((3, n[2], n[1], n[0]), 5)
    y = pwl.apply(pwl.dense_kernels(g), u)
    y0 = apply_N(dense_operator(g[0]), u[0])
    np.testing.assert_allclose(y[0], y0, rtol=0, atol=1e-13)
    assert np.abs(y[1:]).max() > 1e-3          # the linear rows see the pulses


@pytest.mark.parametrize("mode", ["A", "N"])
def test_adjoint_identity(mode):
    n = (4, 3, 2)
    g = green_pwl_tensor(n, 1.0, 0.5)
    kh = pwl.dense_kernels(g)
    eps = 1.0 + _vec((n[2], n[1], n[0]), 7)
    u, v = _vec((4, 3, n[2], n[1], n[0]), 8), _vec((4, 3, n[2], n[1], n[0]), 9)
    Au = pwl.matvec(kh, eps, u, mode)
    AHv = pwl.matvec(kh, eps, v, mode + "H")
    assert abs(np.vdot(v, Au) - np.vdot(AHv, u)) < 1e-12 * np.abs(np.vdot(v, Au))


def test_dense_matrix_and_matvec_agree():
    n = (2, 2, 3)
    g = green_pwl_tensor(n, 1.0, 0.7)
    eps = 1.0 + _vec((n[2], n[1], n[0]), 11)
    u = _vec((4, 3, n[2], n[1], n[0]), 12)
    M = pwl.dense_matrix(g)
    e = np.concatenate([m * eps.ravel() for m in pwl.MASS for _ in range(3)])
    chi = np.tile(eps.ravel() - 1.0, 12)
    A = np.diag(e) - chi[:, None] * M
    np.testing.assert_allclose(pwl.matvec(pwl.dense_kernels(g), eps, u, "A").ravel(), A @ u.ravel(),
                               rtol=0, atol=1e-13)


def test_normalised_basis_has_unit_mass():
    # eps_c = 1 leaves the mass term only: S M S = I
    n = (3, 2, 2)
    g = green_pwl_tensor(n, 1.0, 0.3)
    kh = pwl.dense_kernels(g)
    u = _vec((4, 3, n[2], n[1], n[0]), 13)
    y = pwl.to_normalised(lambda w: pwl.matvec(kh, np.ones((n[2], n[1], n[0])), w, "A"), u)
    np.testing.assert_allclose(y, u, rtol=0, atol=1e-14)


def test_tucker_kernels_approach_the_dense_ones():
    n = (6, 5, 4)
    g = green_pwl_tensor(n, 1.0, 0.5)
    u = _vec((4, 3, n[2], n[1], n[0]), 14)
    yd = pwl.apply(pwl.dense_kernels(g), u)
    kt, ranks = pwl.tucker_kernels(g, 1e-12)
    yt = pwl.apply(kt, u)
    assert np.linalg.norm(yt - yd) < 1e-10 * np.linalg.norm(yd)
    kt6, ranks6 = pwl.tucker_kernels(g, 1e-4)
    assert ranks6.sum() < ranks.sum()
    assert np.linalg.norm(pwl.apply(kt6, u) - yd) < 1e-3 * np.linalg.norm(yd)


def test_sampled_outputs_equal_the_fft_matvec():
    n = (5, 4, 3)
    g = green_pwl_tensor(n, 1.0, 0.45)
    eps = 1.0 + _vec((n[2], n[1], n[0]), 21)
    u = _vec((4, 3, n[2], n[1], n[0]), 22)
    y = pwl.matvec(pwl.dense_kernels(g), eps, u, "A")
    samples = [(0, 0, 0, 0, 0), (3, 2, 2, 3, 4), (1, 1, 1, 2, 0), (2, 0, 0, 1, 3), (1, 2, 2, 0, 2)]
    ys = pwl.sampled_outputs(g, eps, u, samples)
    np.testing.assert_allclose(ys, [y[s] for s in samples], rtol=0, atol=1e-13)
