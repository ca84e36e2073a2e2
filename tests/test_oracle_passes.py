"""Pins of the oracle's five-pass split of the matvec (Sec. V-A): the DFT
matrices against scipy's FFT and exact at quarter turns, each pass's layout
on separable inputs whose transform is known in closed form, and the five
passes in sequence against the oracle's whole-array FFT convolution (which
is itself pinned to the direct Toeplitz sum) in all four modes."""
import numpy as np
import pytest
import scipy.fft as sfft

import vie_inputs as vi
from oracle import operator as opm, passes


@pytest.mark.parametrize("L", [1, 2, 3, 4, 8, 12, 128])
def test_dft_matrix_matches_fft_and_is_exact_at_quarter_turns(L):
    rng = np.random.default_rng(L)
    a = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    np.testing.assert_allclose(passes.dft_matrix(L, -1) @ a, sfft.fft(a), rtol=0, atol=1e-12 * np.abs(a).sum())
    np.testing.assert_allclose(passes.dft_matrix(L, +1) @ a, L * sfft.ifft(a), rtol=0, atol=1e-12 * np.abs(a).sum())
    F = passes.dft_matrix(L, -1)
    mk = np.outer(np.arange(L), np.arange(L)) % L
    q = (4 * mk) % L == 0
    assert set(np.unique(F[q])) <= {1, -1, 1j, -1j}


def _sep(n, i0, rng):
    """x[b, q, k, j, i] = f[b, q, k, j] delta(i, i0)."""
    n1, n2, n3 = n
    f = rng.standard_normal((2, 3, n3, n2)) + 1j * rng.standard_normal((2, 3, n3, n2))
    x = np.zeros((2, 3, n3, n2, n1), complex)
    x[..., i0] = f
    return x, f


def test_x_passes_layout_on_a_shifted_impulse():
    n = (5, 4, 3)
    rng = np.random.default_rng(1)
    x, f = _sep(n, 2, rng)
    S1 = passes.pass_x_forward(x, mode="N")
    L1 = 10
    assert S1.shape == (2, 3, 3, L1, 4)
    w = np.exp(-2j * np.pi * 2 * np.arange(L1) / L1)
    np.testing.assert_allclose(S1, f[:, :, :, None, :] * w[None, None, None, :, None], atol=1e-13)
    # X- of S3 = L1 * delta spectrum recovers the impulse (times L1), cropped to n1
    y = passes.pass_x_inverse(S1, 5, mode="N")
    np.testing.assert_allclose(y, L1 * x, atol=1e-12)


def test_y_passes_layout_on_a_shifted_impulse():
    n2, n3, L1 = 4, 3, 6
    rng = np.random.default_rng(2)
    g = rng.standard_normal((1, 3, n3, L1)) + 1j * rng.standard_normal((1, 3, n3, L1))
    S1 = np.zeros((1, 3, n3, L1, n2), complex)
    S1[..., 1] = g
    S2 = passes.pass_y_forward(S1)
    assert S2.shape == (1, 3, 8, L1, n3)
    w = np.exp(-2j * np.pi * np.arange(8) / 8)
    expect = np.transpose(g, (0, 1, 3, 2))[:, :, None, :, :] * w[None, None, :, None, None]
    np.testing.assert_allclose(S2, expect, atol=1e-13)
    S3 = passes.pass_y_inverse(S2, n2)
    np.testing.assert_allclose(S3, 8 * S1, atol=1e-12)


def test_z_pass_with_a_constant_tensor_is_a_scaled_identity():
    # Nh_pq = M delta_pq (the Fourier tensor of M times the identity): the
    # z pass returns L3 times its input (forward and inverse DFT unnormalised)
    L1, L2, n3 = 4, 6, 5
    M = L1 * L2 * 2 * n3
    nhat = [M * np.ones((L1, L2, 2 * n3)) if c < 3 else np.zeros((L1, L2, 2 * n3)) for c in range(6)]
    rng = np.random.default_rng(3)
    S2 = rng.standard_normal((2, 3, L2, L1, n3)) + 1j * rng.standard_normal((2, 3, L2, L1, n3))
    np.testing.assert_allclose(passes.pass_z(S2, nhat), 2 * n3 * S2, atol=1e-11)


@pytest.mark.parametrize("mode", ["A", "AH", "N", "NH"])
def test_five_passes_equal_the_whole_array_matvec(mode):
    n = (7, 6, 5)
    h = 0.004
    G = vi.green_tensor(n, h, vi.wavenumber(298e6))
    op = opm.tucker_operator(G, 1e-8)
    rng = np.random.default_rng(4)
    shape = (3, n[2], n[1], n[0])
    u = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    eps = 1 + rng.uniform(0, 40, shape[1:]) - 1j * rng.uniform(0, 20, shape[1:])
    y = passes.matvec_by_passes(op, eps, u, mode)[0]
    yo = opm.matvec(op, eps, u, mode)
    assert np.linalg.norm(y - yo) <= 1e-12 * np.linalg.norm(yo)
