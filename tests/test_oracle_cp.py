"""Pins of the oracle's Tucker+CP (Alg. 2, eq. 17): CP by alternating least
squares checked against tensors built from known CP factors, its sweep-wise
monotone fit, the Tucker+CP error bound and the factor algebra."""
import numpy as np

import vie_inputs as vi
from oracle import cp, tucker


def _cplx(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_exact_cp_tensor_is_recovered():
    rng = np.random.default_rng(1)
    R = 3
    Vt = [_cplx(rng, (n, R)) for n in (6, 7, 8)]
    G = cp.cp_reconstruct(Vt)
    Vs, errs = cp.cp_als(G, R, iters=400)
    assert errs[-1] <= 1e-10
    assert np.linalg.norm(cp.cp_reconstruct(Vs) - G) <= 1e-10 * np.linalg.norm(G)


def test_rank_one_is_exact_after_one_sweep():
    rng = np.random.default_rng(2)
    a, b, c = _cplx(rng, (5, 1)), _cplx(rng, (4, 1)), _cplx(rng, (6, 1))
    G = cp.cp_reconstruct([a, b, c])
    Vs, errs = cp.cp_als(G, 1, iters=1)
    assert errs[0] <= 1e-13


def test_fit_never_increases():
    rng = np.random.default_rng(3)
    G = _cplx(rng, (6, 6, 6))          # generic core: not of CP rank 4
    Vs, errs = cp.cp_als(G, 4, iters=60)
    d = np.diff(errs)
    assert np.all(d <= 1e-12 * errs[0])
    assert 0.0 < errs[-1] < errs[0]


def test_khatri_rao_matches_unfolding_convention():
    # G^(mode) = V_mode K^T for a CP tensor, with K the Khatri-Rao product of
    # the other two factors in the unfolding's column order
    rng = np.random.default_rng(4)
    Vt = [_cplx(rng, (n, 2)) for n in (3, 4, 5)]
    G = cp.cp_reconstruct(Vt)
    pairs = {1: (1, 2), 2: (0, 2), 3: (0, 1)}
    for mode, (p, q) in pairs.items():
        K = cp.khatri_rao(Vt[p], Vt[q])
        assert np.allclose(tucker.unfold(G, mode), Vt[mode - 1] @ K.T, atol=1e-13)


def test_tucker_cp_error_bound_and_factor_algebra():
    # a physical defining tensor (xx component at 10^3, 4 mm)
    n = (10, 10, 10)
    G3 = vi.green_tensor(n, 0.004, vi.wavenumber(298e6))
    A = tucker.from_storage(G3[0])
    Ws, G, Us, Vs, errs = cp.tucker_cp(A, 1e-6, iters=300)
    At = tucker.tucker_reconstruct(G, *Us)
    Atcp = cp.cp_reconstruct(Ws)
    e_t = np.linalg.norm(A - At)
    e_cp = np.linalg.norm(G - cp.cp_reconstruct(Vs))
    assert np.linalg.norm(A - Atcp) <= e_t + e_cp + 1e-12 * np.linalg.norm(A)
    # eq. 17 with W = U V equals the CP core multiplied out by the Tucker factors
    assert np.allclose(Atcp, cp.core_times_factors(Vs, Us), atol=1e-12 * np.abs(A).max())
    # the Fourier-domain tensor of the Tucker+CP form equals the FFT of its
    # circulant embedding (Sec. V-A applied to the W factors)
    from oracle import circulant
    s = circulant.axis_signs(0)
    assert np.allclose(cp.fourier_tensor_cp(Ws, s), circulant.fourier_tensor_dense(Atcp, s),
                       atol=1e-11 * np.abs(Atcp).sum())


def test_tucker_cp_operator_exact_on_cp_tensors():
    # defining tensors that are exactly of CP rank 2 (each component with its
    # parity: zero at offset 0 along its odd axes): the Tucker+CP operator of
    # Alg. 2 / eq. 17 reproduces the dense operator's product
    from oracle import circulant, operator as opm
    rng = np.random.default_rng(9)
    n = (6, 5, 4)
    green = np.zeros((6, n[2], n[1], n[0]), complex)
    for c in range(6):
        signs = circulant.axis_signs(c)
        Vs = []
        for a in range(3):
            V = _cplx(rng, (n[a], 2))
            if signs[a] < 0:
                V[0, :] = 0
            Vs.append(V)
        green[c] = tucker.to_storage(cp.cp_reconstruct(Vs))
    dense = opm.dense_operator(green)
    op = opm.tucker_cp_operator(green, 1e-12, R=2, iters=300)
    assert max(op.cp_rel_err) <= 1e-9
    u = vi.random_field(n, 3)
    y = opm.apply_N(op, u)
    yd = opm.apply_N(dense, u)
    assert np.linalg.norm(y - yd) <= 1e-8 * np.linalg.norm(yd)


def test_cp_rank_above_the_core_size_recovers_a_unique_decomposition():
    # a 5 x 6 x 7 tensor of CP rank 7 > 5: Kruskal's condition (k-ranks
    # 5 + 6 + 7 >= 2 R + 2) makes the decomposition unique, and ALS from the
    # padded start reaches it
    rng = np.random.default_rng(4)
    r, R = (5, 6, 7), 7
    Vs = [rng.standard_normal((r[a], R)) + 1j * rng.standard_normal((r[a], R)) for a in range(3)]
    G = cp.cp_reconstruct(Vs)
    _, errs = cp.cp_als(G, R, 3000)
    assert errs[-1] <= 1e-10


def test_start_columns_beyond_the_singular_vectors():
    U = np.linalg.qr(np.random.default_rng(1).standard_normal((4, 4)))[0]
    S = cp.start_columns(U, 6)
    assert np.array_equal(S[:, :4], U)
    g = (np.sqrt(5) - 1) / 2
    for a in range(4):
        for j in (4, 5):
            t = g * (a + 1) * (j + 1)
            assert abs(S[a, j] - np.exp(2j * np.pi * (t - np.floor(t))) / 2.0) <= 1e-15
    assert np.array_equal(cp.start_columns(U, 3), U[:, :3])
