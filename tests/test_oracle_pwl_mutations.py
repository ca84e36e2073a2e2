"""Mistakes planted in the piecewise-linear oracles (on the CPU, through
monkeypatch) must break at least one of their pins: the pins of
test_oracle_pwl.py, test_oracle_pwl_k.py and test_oracle_pwl_jm.py are
re-evaluated here with a wrong pair-swap sign, a wrong parity rule, a lost
antisymmetry sign and swapped coupling constants."""
import numpy as np

import vie_inputs as vi
from oracle import pwl, pwl_jm, pwl_k
from vie_inputs import green_pwl_entry, green_pwl_k_entry, green_pwl_k_tensor, green_pwl_tensor


def _symmetric(M):
    return np.allclose(M, M.T, rtol=0, atol=1e-14)


def _n_signed_entries_match():
    kappa = 0.3
    g = green_pwl_tensor((4, 3, 3), 1.0, kappa, near_order=16)
    for D in [(-1, 0, 1), (2, -1, -2), (-3, -2, 0)]:
        E = green_pwl_entry(D, kappa, 16, method=0)
        for P, (l, lp) in enumerate(pwl.PAIRS):
            for c, (p, q) in enumerate(pwl.COMPONENTS):
                if abs(pwl.signed_entry(g, l, lp, p, q, D) - E[P, c]) > 1e-10:
                    return False
    return True


def _k_signed_entries_match():
    kappa = 0.3
    kt = green_pwl_k_tensor((4, 3, 3), 1.0, kappa, near_order=16)
    for D in [(-1, 0, 1), (2, -1, -2), (-3, -2, 0)]:
        E = green_pwl_k_entry(D, kappa, 16, method=0)
        for P, (l, lp) in enumerate(pwl.PAIRS):
            for c, (p, q) in enumerate(pwl_k.K_COMPONENTS):
                if abs(pwl_k.signed_entry_k(kt, l, lp, p, q, D) - E[P, c]) > 1e-10:
                    return False
    return True


def test_pins_hold_on_the_unmodified_oracles():
    assert _symmetric(pwl.dense_matrix(green_pwl_tensor((3, 2, 2), 1.0, 0.6)))
    assert _symmetric(pwl_k.dense_matrix_k(green_pwl_k_tensor((3, 2, 2), 1.0, 0.6)))
    assert _n_signed_entries_match()
    assert _k_signed_entries_match()


def test_n_without_the_pair_swap_sign_is_caught(monkeypatch):
    monkeypatch.setattr(pwl, "swap_sign", lambda l, lp: 1.0)
    assert not _symmetric(pwl.dense_matrix(green_pwl_tensor((3, 2, 2), 1.0, 0.6)))


def test_n_parity_without_the_linear_functions_is_caught(monkeypatch):
    monkeypatch.setattr(pwl, "odd_axes", lambda l, lp, p, q: tuple(((p == a) + (q == a)) % 2 == 1 for a in range(3)))
    assert not _n_signed_entries_match()


def test_k_without_the_pair_swap_sign_is_caught(monkeypatch):
    monkeypatch.setattr(pwl_k, "swap_sign", lambda l, lp: 1.0)
    assert not _symmetric(pwl_k.dense_matrix_k(green_pwl_k_tensor((3, 2, 2), 1.0, 0.6)))


def test_k_without_the_antisymmetry_sign_is_caught(monkeypatch):
    orig = pwl_k.signed_entry_k
    monkeypatch.setattr(pwl_k, "signed_entry_k",
                        lambda kt, l, lp, p, q, D: orig(kt, l, lp, min(p, q), max(p, q), D))
    assert not _symmetric(pwl_k.dense_matrix_k(green_pwl_k_tensor((3, 2, 2), 1.0, 0.6)))


def test_k_parity_without_the_derivative_axis_is_caught(monkeypatch):
    monkeypatch.setattr(pwl_k, "k_odd_axes", lambda l, lp, c: tuple(((l == a + 1) + (lp == a + 1)) % 2 == 1
                                                                     for a in range(3)))
    assert not _k_signed_entries_match()


def test_jm_with_swapped_coupling_constants_is_caught(monkeypatch):
    n, h, f = (3, 3, 2), 0.004, 298e6
    k0 = vi.wavenumber(f)
    khn = pwl.dense_kernels(green_pwl_tensor(n, h, k0))
    khk = pwl_k.dense_kernels_k(green_pwl_k_tensor(n, h, k0))
    rng = np.random.default_rng(31)
    shape = tuple(reversed(n))
    eps_c = 1 + rng.uniform(0, 50, shape) - 1j * rng.uniform(0, 30, shape)
    mu_c = 1 + rng.uniform(0, 2, shape) - 1j * rng.uniform(0, 0.5, shape)
    x = rng.standard_normal((2, 4, 3) + shape) + 1j * rng.standard_normal((2, 4, 3) + shape)
    alpha = -vi.EPS0 / vi.MU0

    def duality_holds():
        y = pwl_jm.jm_matvec(khn, khk, eps_c, mu_c, x, h, f)
        yd = pwl_jm.jm_matvec(khn, khk, mu_c, eps_c, np.stack([alpha * x[1], x[0]]), h, f)
        return (np.allclose(yd[0], alpha * y[1], rtol=1e-12, atol=1e-14 * np.abs(alpha * y[1]).max()) and
                np.allclose(yd[1], y[0], rtol=1e-12, atol=1e-14 * np.abs(y[0]).max()))

    assert duality_holds()
    monkeypatch.setattr(pwl_jm, "EPS0", vi.MU0)
    monkeypatch.setattr(pwl_jm, "MU0", vi.EPS0)
    assert not duality_holds()
