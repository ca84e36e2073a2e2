"""Pins of the oracle's piecewise-linear magnetic operator (oracle/pwl_k.py)
against the generator's direct evaluation at signed offsets, a 6-D integral
over the two voxels for the pairs l > l', the symmetry of the Galerkin
matrix, the pulse-basis K oracle and the written-out sum."""
import numpy as np
import pytest

from oracle import pwl, pwl_k
from oracle.magnetic import apply_K, dense_k_operator
from vie_inputs import green_pwl_k_entry, green_pwl_k_tensor

from test_inputs_pwl import _brute6_k


def _vec(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("n", [(3, 2, 2), (1, 2, 3), (2, 3, 1)])
def test_fft_sum_matches_brute_force(n):
    kt = green_pwl_k_tensor(n, 1.0, 0.4)
    u = _vec((4, 3, n[2], n[1], n[0]), 31)
    y = pwl.apply(pwl_k.dense_kernels_k(kt), u)
    np.testing.assert_allclose(y, pwl_k.brute_force_k(kt, u), rtol=0, atol=1e-13)
    assert np.abs(y).max() > 1e-2


def test_signed_entries_match_direct_evaluation():
    # stored pairs at negative offsets against the generator's integral there
    # (no parity rule), the pairs l > l' and the lower triangle against a 6-D
    # integral over the observation and source voxels
    kappa, n = 0.3, (4, 3, 3)
    kt = green_pwl_k_tensor(n, 1.0, kappa, near_order=16)
    for D in [(-1, 0, 1), (2, -1, -2), (-3, -2, 0), (-1, -1, -1)]:
        E = green_pwl_k_entry(D, kappa, 16, method=0)
        for P, (l, lp) in enumerate(pwl.PAIRS):
            for c, (p, q) in enumerate(pwl_k.K_COMPONENTS):
                assert abs(pwl_k.signed_entry_k(kt, l, lp, p, q, D) - E[P, c]) < 1e-10, (D, P, c)
    D = (3, -2, 1)
    kb = green_pwl_k_tensor((4, 3, 2), 1.0, kappa)
    B = _brute6_k(D, kappa)
    for l in range(4):
        for lp in range(4):
            scale = np.abs(B[l, lp]).max()
            for c, (p, q) in enumerate(pwl_k.K_COMPONENTS):
                v = pwl_k.signed_entry_k(kb, l, lp, p, q, D)
                assert abs(v - B[l, lp, c]) < 1e-8 * scale, (l, lp, c)
                assert abs(pwl_k.signed_entry_k(kb, l, lp, q, p, D) + B[l, lp, c]) < 1e-8 * scale
            assert pwl_k.signed_entry_k(kb, l, lp, 1, 1, D) == 0


def test_galerkin_matrix_is_symmetric():
    # K is symmetric under the real bilinear pairing (curl is self-adjoint on
    # the volume); with Kt_qp = -Kt_pq this fixes the pair-swap sign and the
    # parities of the embedding (reflecting all three axes gives -sigma)
    kt = green_pwl_k_tensor((3, 2, 2), 1.0, 0.6)
    M = pwl_k.dense_matrix_k(kt)
    np.testing.assert_allclose(M, M.T, rtol=0, atol=1e-14)
    assert np.abs(M).max() > 0.05


def test_pulse_unknowns_reduce_to_the_pulse_k():
    # with only pulse coefficients the pulse rows are the pulse K of the
    # (pulse, pulse) tensors, evaluated by the pulse-basis oracle
    n = (5, 4, 3)
    kt = green_pwl_k_tensor(n, 1.0, 0.5)
    u = np.zeros((4, 3, n[2], n[1], n[0]), complex)
    u[0] = _vec((3, n[2], n[1], n[0]), 33)
    y = pwl.apply(pwl_k.dense_kernels_k(kt), u)
    np.testing.assert_allclose(y[0], apply_K(dense_k_operator(kt[0]), u[0]), rtol=0, atol=1e-13)
    assert np.abs(y[1:]).max() > 1e-3


def test_tucker_kernels_approach_the_dense_ones():
    n = (6, 5, 4)
    kt = green_pwl_k_tensor(n, 1.0, 0.5)
    u = _vec((4, 3, n[2], n[1], n[0]), 34)
    yd = pwl.apply(pwl_k.dense_kernels_k(kt), u)
    kh, ranks = pwl_k.tucker_kernels_k(kt, 1e-12)
    assert np.linalg.norm(pwl.apply(kh, u) - yd) < 1e-10 * np.linalg.norm(yd)
    kh4, ranks4 = pwl_k.tucker_kernels_k(kt, 1e-4)
    assert ranks4.sum() < ranks.sum()
    assert np.linalg.norm(pwl.apply(kh4, u) - yd) < 1e-3 * np.linalg.norm(yd)


def test_sampled_outputs_equal_the_fft_sum():
    n = (5, 4, 3)
    kt = green_pwl_k_tensor(n, 1.0, 0.45)
    u = _vec((4, 3, n[2], n[1], n[0]), 35)
    y = pwl.apply(pwl_k.dense_kernels_k(kt), u)
    samples = [(0, 0, 0, 0, 0), (3, 2, 2, 3, 4), (1, 1, 1, 2, 0), (2, 0, 0, 1, 3), (1, 2, 2, 0, 2)]
    np.testing.assert_allclose(pwl_k.sampled_outputs_k(kt, u, samples), [y[s] for s in samples], rtol=0,
                               atol=1e-13)


def test_normalised_form():
    n = (3, 3, 2)
    kt = green_pwl_k_tensor(n, 1.0, 0.4)
    kh = pwl_k.dense_kernels_k(kt)
    u = _vec((4, 3, n[2], n[1], n[0]), 36)
    S = pwl.SCALE[:, None, None, None, None]
    np.testing.assert_allclose(pwl_k.to_normalised_k(kh, u), S * pwl_k.brute_force_k(kt, S * u), rtol=0,
                               atol=1e-12)
