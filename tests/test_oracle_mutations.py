"""Mistakes planted in the pulse-basis oracles (on the CPU, through
monkeypatch) must break at least one of their pins, re-evaluated here: the
embedding and entry parities, an off-by-one circulant embedding, the
coupling constants of the JM right-hand side and the HOSVD truncation."""
import numpy as np

import vie_inputs as vi
from oracle import circulant, tucker
from oracle import magnetic as mg
from oracle import operator as opm
from vie_inputs.green import green_k_tensor

from test_oracle_magnetic import _grad_g_fd, _jm_problem
from test_oracle_operator import _dyadic_fd


def _n_parity_pin():
    kappa = 0.05
    G = vi.green_tensor((10, 8, 6), 1.0, kappa)
    base = (9, 7, 5)
    for c, (p, q) in enumerate(circulant.COMPONENTS):
        ref = opm.signed_entry(G, c, base) / _dyadic_fd(base, kappa)[p, q]
        for flips in range(1, 8):
            D = tuple(-x if (flips >> a) & 1 else x for a, x in enumerate(base))
            if abs(opm.signed_entry(G, c, D) / _dyadic_fd(D, kappa)[p, q] - ref) >= 2e-3 * abs(ref):
                return False
    return True


def _k_parity_pin():
    kappa = 0.05
    kt = green_k_tensor((10, 8, 6), 1.0, kappa)
    base = (9, 7, 5)
    for c, (p, q) in enumerate(mg.K_COMPONENTS):
        s = mg.K_ODD_AXIS[c]
        ref = mg.k_entry(kt, p, q, base) / _grad_g_fd(base, kappa)[s]
        for flips in range(1, 8):
            D = tuple(-x if (flips >> a) & 1 else x for a, x in enumerate(base))
            if abs(mg.k_entry(kt, p, q, D) / _grad_g_fd(D, kappa)[s] - ref) >= 2e-3 * abs(ref):
                return False
    return True


def _fft_equals_direct_sum():
    n = (4, 3, 5)
    G = vi.random_complex((6, n[2], n[1], n[0]), 3)
    for c in range(6):
        s = circulant.axis_signs(c)
        if s[0] < 0:
            G[c, :, :, 0] = 0
        if s[1] < 0:
            G[c, :, 0, :] = 0
        if s[2] < 0:
            G[c, 0, :, :] = 0
    u = vi.random_field(n, 4)
    y_fft = opm.apply_N(opm.dense_operator(G), u)
    y_dir = opm.brute_force_N(G, u)
    return np.linalg.norm(y_fft - y_dir) <= 1e-13 * np.linalg.norm(y_dir)


def _jm_rhs_duality():
    f, _, _, eps_c, mu_c, _ = _jm_problem((5, 4, 3), 0.004, 15)
    e_inc = vi.random_field((5, 4, 3), 151)
    h_inc = vi.random_field((5, 4, 3), 152)
    b = mg.jm_rhs(eps_c, mu_c, e_inc, h_inc, f)
    alpha = -vi.EPS0 / vi.MU0
    bd = mg.jm_rhs(mu_c, eps_c, -h_inc, (vi.EPS0 / vi.MU0) * e_inc, f)
    return (np.allclose(bd[0], alpha * b[1], rtol=1e-13, atol=1e-15 * np.abs(alpha * b[1]).max()) and
            np.allclose(bd[1], b[0], rtol=1e-13, atol=1e-15 * np.abs(b[0]).max()))


def _hosvd_tails_within_share():
    n = (18, 15, 12)
    A = np.zeros(n, dtype=complex)
    for t in range(12):
        vecs = [vi.random_complex(m, 100 + 3 * t + a) for a, m in enumerate(n)]
        A += 0.3 ** t * np.einsum("i,j,k->ijk", *vecs)
    tol = 1e-4
    G, Us, s = tucker.hosvd(A, tol)
    return all(np.sqrt(np.sum(si[U.shape[1]:] ** 2)) <= tol / np.sqrt(3) * np.linalg.norm(A) * (1 + 1e-12)
               for si, U in zip(s, Us))


def test_pins_hold_on_the_unmodified_oracles():
    assert _n_parity_pin() and _k_parity_pin() and _fft_equals_direct_sum()
    assert _jm_rhs_duality() and _hosvd_tails_within_share()


def test_n_without_entry_parities_is_caught(monkeypatch):
    monkeypatch.setattr(opm, "axis_signs", lambda c: (1, 1, 1))
    assert not _n_parity_pin()


def test_k_without_entry_parities_is_caught(monkeypatch):
    monkeypatch.setattr(mg, "k_axis_signs", lambda c: (1, 1, 1))
    assert not _k_parity_pin()


def test_off_by_one_embedding_is_caught(monkeypatch):
    def shifted(U, s):
        U = np.asarray(U)
        n = U.shape[0]
        E = np.zeros((2 * n,) + U.shape[1:], dtype=np.complex128)
        E[:n] = U
        if n > 1:
            E[n:2 * n - 1] = s * U[1:][::-1]      # the mirror one place early
        return E
    monkeypatch.setattr(circulant, "embed_columns", shifted)
    assert not _fft_equals_direct_sum()


def test_jm_rhs_with_swapped_coupling_constants_is_caught(monkeypatch):
    import vie_inputs.constants as const
    eps0, mu0 = const.EPS0, const.MU0
    monkeypatch.setattr(const, "EPS0", mu0)
    monkeypatch.setattr(mg, "MU0", eps0)
    assert not _jm_rhs_duality()


def test_truncation_one_column_short_is_caught(monkeypatch):
    orig = tucker.truncation_rank
    monkeypatch.setattr(tucker, "truncation_rank", lambda s, tol, rule, fro: max(1, orig(s, tol, rule, fro) - 1))
    assert not _hosvd_tails_within_share()


def _cp_recovers_exact_rank3():
    from oracle import cp
    rng = np.random.default_rng(7)
    Vs = [rng.standard_normal((m, 3)) + 1j * rng.standard_normal((m, 3)) for m in (5, 6, 7)]
    G = cp.cp_reconstruct(Vs)
    W, errs = cp.cp_als(G, 3, iters=300)
    return np.linalg.norm(cp.cp_reconstruct(W) - G) <= 1e-8 * np.linalg.norm(G)


def _gmres_solves_dense():
    from oracle import gmres as gm
    rng = np.random.default_rng(8)
    A = np.eye(40) * 20 + rng.standard_normal((40, 40)) + 1j * rng.standard_normal((40, 40))
    b = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    # one cycle as long as the dimension: exact in exact arithmetic, so the
    # restarts on the true residual cannot mend a wrong least-squares step
    x, info = gm.gmres(lambda v: A @ v, b, tol=1e-12, restart=40, max_outer=1)
    return np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-9 * np.linalg.norm(np.linalg.solve(A, b))


def _passes_equal_fft_convolution():
    from oracle import passes
    n = (4, 3, 5)
    G = vi.green_tensor(n, 0.01, vi.wavenumber(298e6))
    op = opm.dense_operator(G)
    u = vi.random_field(n, 9)
    y = passes.matvec_by_passes(op, None, u, "N")[0]
    y0 = opm.apply_N(op, u)
    return np.linalg.norm(y - y0) <= 1e-12 * np.linalg.norm(y0)


def test_more_pins_hold_on_the_unmodified_oracles():
    assert _cp_recovers_exact_rank3() and _gmres_solves_dense() and _passes_equal_fft_convolution()


def test_khatri_rao_with_swapped_operands_is_caught(monkeypatch):
    from oracle import cp
    orig = cp.khatri_rao
    monkeypatch.setattr(cp, "khatri_rao", lambda X, Y: orig(Y, X))
    assert not _cp_recovers_exact_rank3()


def test_givens_with_a_wrong_sign_is_caught(monkeypatch):
    from oracle import gmres as gm
    orig = gm._givens
    monkeypatch.setattr(gm, "_givens", lambda a, b: (lambda c, s: (c, -s))(*orig(a, b)))
    assert not _gmres_solves_dense()


def test_z_pass_with_the_adjoint_tables_is_caught(monkeypatch):
    # (flipping every DFT direction would not be a mistake here: N is even
    # under reflection of all three axes, so the correlation equals the
    # convolution; using conj(N^) in the forward product is one)
    from oracle import passes
    orig = passes.pass_z
    monkeypatch.setattr(passes, "pass_z", lambda S2, nhat, conj=False: orig(S2, nhat, not conj))
    assert not _passes_equal_fft_convolution()
