"""Pins of the oracle's JMVIE operator in the piecewise-linear basis
(oracle/pwl_jm.py): pulse-only currents reduce to the pulse-basis JM oracle,
Maxwell duality, and the electric operator without magnetic contrast."""
import numpy as np

import vie_inputs as vi
from oracle import magnetic as mg
from oracle import pwl, pwl_jm, pwl_k
from oracle.operator import dense_operator


def _problem(n, h, seed):
    f = 298e6
    k0 = vi.wavenumber(f)
    G = vi.green_pwl_tensor(n, h, k0)
    kt = vi.green_pwl_k_tensor(n, h, k0)
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    eps_c = 1 + rng.uniform(0, 50, shape) - 1j * rng.uniform(0, 30, shape)
    mu_c = 1 + rng.uniform(0, 2, shape) - 1j * rng.uniform(0, 0.5, shape)
    xs = (2, 4, 3) + shape
    x = rng.standard_normal(xs) + 1j * rng.standard_normal(xs)
    return f, G, kt, eps_c, mu_c, x


def test_pulse_currents_reduce_to_the_pulse_jm_operator():
    n, h = (5, 4, 3), 0.005
    f, G, kt, eps_c, mu_c, x = _problem(n, h, 21)
    x[:, 1:] = 0
    y = pwl_jm.jm_matvec(pwl.dense_kernels(G), pwl_k.dense_kernels_k(kt), eps_c, mu_c, x, h, f)
    y0 = mg.jm_matvec(dense_operator(G[0]), mg.dense_k_operator(kt[0]), eps_c, mu_c, x[:, 0], h, f)
    np.testing.assert_allclose(y[:, 0], y0, rtol=0, atol=1e-13 * np.abs(y0).max())
    assert np.abs(y[:, 1:]).max() > 1e-4 * np.abs(y0).max()


def test_duality():
    # (E, H, eps, mu) -> (H, -E, mu, eps): with alpha = -eps0/mu0,
    # A(mu_c, eps_c) [alpha M; J] = [alpha y_M; y_J]
    n, h = (4, 3, 3), 0.004
    f, G, kt, eps_c, mu_c, x = _problem(n, h, 22)
    khn, khk = pwl.dense_kernels(G), pwl_k.dense_kernels_k(kt)
    y = pwl_jm.jm_matvec(khn, khk, eps_c, mu_c, x, h, f)
    alpha = -vi.EPS0 / vi.MU0
    yd = pwl_jm.jm_matvec(khn, khk, mu_c, eps_c, np.stack([alpha * x[1], x[0]]), h, f)
    np.testing.assert_allclose(yd[0], alpha * y[1], rtol=1e-12, atol=1e-14 * np.abs(alpha * y[1]).max())
    np.testing.assert_allclose(yd[1], y[0], rtol=1e-12, atol=1e-14 * np.abs(y[0]).max())
    y0 = pwl_jm.jm_matvec(khn, khk, eps_c, mu_c, np.stack([x[0], 0 * x[1]]), h, f)
    assert np.linalg.norm(y0[0] - y[0]) > 1e-6 * np.linalg.norm(y[0])


def test_reduces_to_the_electric_block():
    n, h = (4, 4, 3), 0.005
    f, G, kt, eps_c, _, x = _problem(n, h, 23)
    x[1] = 0
    khn = pwl.dense_kernels(G)
    y = pwl_jm.jm_matvec(khn, pwl_k.dense_kernels_k(kt), eps_c, np.ones_like(eps_c), x, h, f)
    np.testing.assert_allclose(y[0], pwl.matvec(khn, eps_c, x[0], "A"), rtol=0, atol=1e-14 * np.abs(y[0]).max())
    assert not np.any(y[1])


def test_normalised_form():
    n, h = (3, 3, 2), 0.005
    f, G, kt, eps_c, mu_c, x = _problem(n, h, 24)
    khn, khk = pwl.dense_kernels(G), pwl_k.dense_kernels_k(kt)
    S = pwl.SCALE[:, None, None, None, None]
    yn = pwl_jm.to_normalised_jm(lambda w: pwl_jm.jm_matvec(khn, khk, eps_c, mu_c, w, h, f), x)
    ref = pwl_jm.jm_matvec(khn, khk, eps_c, mu_c, np.stack([S * x[0], S * x[1]]), h, f)
    np.testing.assert_allclose(yn, np.stack([S * ref[0], S * ref[1]]), rtol=0, atol=1e-15 * np.abs(ref).max())
