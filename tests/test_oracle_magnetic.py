"""Pins of the K operator's defining tensor (input data) and of the oracle's
K product and b1+ observable (eq. 5, eq. 18):

* parity and antisymmetry of the entries; the far field against the point
  curl kernel with the tent correction and its O(|D|^-4) convergence;
* the near entries, which the generator takes as -int g d_s tau (integrable
  kernel), against an independent quadrature of the other side of the
  integration by parts, int d_s g tau (Duffy-regularised here);
* the FFT product against the explicit Toeplitz sum, the symmetric Galerkin
  matrix, Tucker at a tight tolerance against the dense tensor;
* the plane wave's H against the curl of its E, and b1+ of a field with a
  known value."""
import math

import numpy as np
import pytest

import vie_inputs as vi
from vie_inputs.green import green_k_tensor
from oracle import magnetic as mg


def _ghat(x, kappa):
    r = np.sqrt((x * x).sum(axis=-1))
    return np.exp(-1j * kappa * r) / (4 * math.pi * r), r


def _dg(x, kappa):
    """grad g^(x) for points x (..., 3)."""
    g, r = _ghat(x, kappa)
    f = -g * (1 + 1j * kappa * r) / r ** 2
    return f[..., None] * x


def _gl(q):
    z, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (z + 1), 0.5 * w


def _F_direct(D, kappa, q=28):
    """F_s(D) = int d_s g^(x) tau_D(x) dx over the 8 cells of the support;
    cells with the origin at a corner are split into three pyramids (Duffy),
    whose Jacobian s^2 absorbs the 1/r^2 singularity."""
    x1, w1 = _gl(q)
    F = np.zeros(3, complex)
    for cell in range(8):
        lo = np.array([D[a] + (0.0 if (cell >> a) & 1 else -1.0) for a in range(3)])
        if all(v in (0.0, -1.0) for v in lo):
            sig = np.where(lo == 0.0, 1.0, -1.0)
            for face in range(3):
                a1, a2 = (face + 1) % 3, (face + 2) % 3
                s, u, v = np.meshgrid(x1, x1, x1, indexing="ij")
                W = np.einsum("i,j,k->ijk", w1, w1, w1) * s ** 2
                y = np.zeros(s.shape + (3,))
                y[..., face] = s
                y[..., a1] = s * u
                y[..., a2] = s * v
                x = y * sig
                tau = np.prod(np.maximum(1 - np.abs(x - np.array(D, float)), 0), axis=-1)
                F += np.einsum("ijk,ijka->a", W * tau, _dg(x, kappa))
        else:
            a, b, c = np.meshgrid(lo[0] + x1, lo[1] + x1, lo[2] + x1, indexing="ij")
            x = np.stack([a, b, c], axis=-1)
            W = np.einsum("i,j,k->ijk", w1, w1, w1)
            tau = np.prod(np.maximum(1 - np.abs(x - np.array(D, float)), 0), axis=-1)
            F += np.einsum("ijk,ijka->a", W * tau, _dg(x, kappa))
    return F


def _k_from_F(F):
    """Stored components (xy, xz, yz) from F = (F_x, F_y, F_z)."""
    return np.array([-F[2], F[1], -F[0]])


def test_parity_and_antisymmetry_zeros():
    K = green_k_tensor((5, 4, 3), 0.005, vi.wavenumber(298e6))
    # Kt_xy is odd along z, Kt_xz along y, Kt_yz along x: zero at offset 0 there
    assert np.abs(K[0, 0, :, :]).max() == 0
    assert np.abs(K[1, :, 0, :]).max() == 0
    assert np.abs(K[2, :, :, 0]).max() == 0
    assert np.abs(K).max() > 0
    # axis permutation: Kt_xy(0,0,d) = -Kt_yz(d,0,0) rotated (x->y->z->x)
    K2 = green_k_tensor((4, 4, 4), 1.0, 0.2)
    # F_z(0,0,d) = F_x(d,0,0) by symmetry of g and tau
    np.testing.assert_allclose(K2[0, 2, 0, 0], K2[2, 0, 0, 2], rtol=1e-12)
    np.testing.assert_allclose(-K2[1, 0, 2, 0], K2[2, 0, 0, 2], rtol=1e-12)


def test_far_field_matches_point_curl_kernel():
    # Kt(D) = int eps grad g(D + t) prod(1 - |t_i|) dt; grad g solves the
    # Helmholtz equation away from 0, so Kt = point value (1 - kappa^2/12)
    # + O(|D|^-4) relative
    kappa = 0.05
    K = green_k_tensor((33, 2, 2), 1.0, kappa)
    errs = []
    for d in (4, 8, 16):
        ref = -_dg(np.array([float(d), 0.0, 0.0]), kappa)[0] * (1 - kappa ** 2 / 12)   # Kt_yz = -F_x
        errs.append(abs(K[2, 0, 0, d] - ref) / abs(ref))
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 12) and np.all(ratios < 20), (errs, ratios)


@pytest.mark.parametrize("D", [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (1, 1, 1),
                               (2, 1, 0)])
def test_near_entries_integration_by_parts(D):
    kappa = 0.3
    K = green_k_tensor((3, 2, 2), 1.0, kappa)
    ref = _k_from_F(_F_direct(D, kappa))
    got = K[:, D[2], D[1], D[0]]
    scale = np.abs(K).max()
    assert np.abs(got - ref).max() <= 1e-8 * scale, (D, got, ref)


def test_quadrature_converged_and_kappa_scaling():
    a = green_k_tensor((6, 5, 4), 1.0, 0.3)
    b = green_k_tensor((6, 5, 4), 1.0, 0.3, near_order=28, far_boost=6)
    assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max()
    c = green_k_tensor((6, 5, 4), 0.002, 150.0)
    np.testing.assert_allclose(a, c, rtol=1e-13, atol=1e-15)


def _random_k_tensor(rng, n):
    kt = rng.standard_normal((3,) + tuple(reversed(n))) + 1j * rng.standard_normal((3,) + tuple(reversed(n)))
    kt[0, 0, :, :] = 0
    kt[1, :, 0, :] = 0
    kt[2, :, :, 0] = 0
    return kt


@pytest.mark.parametrize("n", [(3, 2, 4), (4, 3, 2), (1, 1, 1), (2, 3, 3)])
def test_fft_product_matches_toeplitz_sum(n):
    rng = np.random.default_rng(7)
    for kt in (_random_k_tensor(rng, n), green_k_tensor(n, 0.004, vi.wavenumber(298e6))):
        u = vi.random_field(n, 3)
        y = mg.apply_K(mg.dense_k_operator(kt), u)
        yb = mg.brute_force_K(kt, u)
        assert np.abs(y - yb).max() <= 1e-12 * max(np.abs(yb).max(), 1e-30)


def test_galerkin_matrix_is_symmetric():
    # Kt_pq(D) = -Kt_qp(D) and Kt(-D) = -Kt(D): the matrix equals its transpose
    kt = green_k_tensor((3, 2, 2), 0.005, vi.wavenumber(298e6))
    M = mg.dense_matrix_K(kt)
    assert np.abs(M - M.T).max() <= 1e-14 * np.abs(M).max()
    assert np.abs(M - M.conj().T).max() > 1e-6 * np.abs(M).max()   # complex symmetric, not Hermitian
    u = vi.random_field((3, 2, 2), 4)
    np.testing.assert_allclose((M @ u.reshape(-1)).reshape(u.shape), mg.brute_force_K(kt, u), rtol=0,
                               atol=1e-14 * np.abs(M).max() * np.abs(u).max() * M.shape[0])


def test_tucker_tight_tolerance_equals_dense():
    n = (10, 8, 6)
    kt = green_k_tensor(n, 0.004, vi.wavenumber(298e6))
    u = vi.random_field(n, 5)
    yd = mg.apply_K(mg.dense_k_operator(kt), u)
    yt = mg.apply_K(mg.tucker_k_operator(kt, 1e-13), u)
    assert np.linalg.norm(yt - yd) <= 1e-11 * np.linalg.norm(yd)
    # and a loose tolerance moves it by about that tolerance
    y6 = mg.apply_K(mg.tucker_k_operator(kt, 1e-6), u)
    e6 = np.linalg.norm(y6 - yd) / np.linalg.norm(yd)
    assert 1e-10 < e6 <= 1e-5


def test_plane_wave_h_is_the_curl_of_e():
    # exp(+i omega t): curl E = -i omega mu0 H; check along z by central
    # differences of the sampled E on a fine grid
    f = 298e6
    n = (2, 2, 64)
    h = 0.001
    E = vi.plane_wave(n, h, f, pol=0)
    H = vi.plane_wave_h(n, h, f, pol=0)
    dEx_dz = (E[0, 2:] - E[0, :-2]) / (2 * h)
    Hy = dEx_dz / (-1j * vi.omega(f) * vi.MU0)          # (curl E)_y = dEx/dz
    k0h = vi.wavenumber(f) * h
    np.testing.assert_allclose(Hy * (k0h / math.sin(k0h)), H[1, 1:-1], rtol=1e-12)
    assert np.abs(H[0]).max() == 0 and np.abs(H[2]).max() == 0
    # x-polarised plane wave: |b1+| = mu0 |Hy| = 1/c0
    np.testing.assert_allclose(mg.b1_plus(H), 1.0 / vi.C0, rtol=1e-12)


def test_magnetic_field_of_a_single_current_voxel():
    # far from a single current voxel, K J approaches the field of the
    # equivalent Hertzian dipole, H = grad g x (J h^3)
    f = 298e6
    h = 0.004
    n = (24, 1, 1)
    kt = green_k_tensor(n, h, vi.wavenumber(f))
    J = np.zeros((3, 1, 1, 24), complex)
    J[1, 0, 0, 0] = 1.0                                   # y-directed current in voxel 0
    H = mg.magnetic_field(mg.dense_k_operator(kt), J, np.zeros_like(J), h)
    d = 20
    r = np.array([d * h, 0.0, 0.0])
    k0 = vi.wavenumber(f)
    gr = np.linalg.norm(r)
    g = np.exp(-1j * k0 * gr) / (4 * math.pi * gr)
    grad = -g * (1 + 1j * k0 * gr) / gr ** 2 * r
    Hd = np.cross(grad, np.array([0.0, h ** 3, 0.0]))
    np.testing.assert_allclose(H[:, 0, 0, d], Hd, rtol=2e-3, atol=1e-12 * abs(Hd).max())


def _jm_problem(n, h, seed):
    f = 298e6
    G = vi.green_tensor(n, h, vi.wavenumber(f))
    kt = green_k_tensor(n, h, vi.wavenumber(f))
    rng = np.random.default_rng(seed)
    shape = tuple(reversed(n))
    eps_c = 1 + rng.uniform(0, 50, shape) - 1j * rng.uniform(0, 30, shape)
    mu_c = 1 + rng.uniform(0, 2, shape) - 1j * rng.uniform(0, 0.5, shape)
    x = np.stack([vi.random_field(n, seed + 1), vi.random_field(n, seed + 2)])
    return f, G, kt, eps_c, mu_c, x


def test_jm_reduces_to_the_electric_operator():
    # no magnetic contrast and no magnetic current: the first block row is the
    # electric operator of eq. 4 and the second vanishes
    from oracle import operator as opm
    n = (6, 5, 4)
    h = 0.005
    f, G, kt, eps_c, _, x = _jm_problem(n, h, 11)
    x[1] = 0
    opn, opk = opm.dense_operator(G), mg.dense_k_operator(kt)
    y = mg.jm_matvec(opn, opk, eps_c, np.ones_like(eps_c), x, h, f)
    np.testing.assert_allclose(y[0], opm.matvec(opn, eps_c, x[0], "A"), rtol=0, atol=1e-14 * np.abs(y[0]).max())
    assert not np.any(y[1])


def test_jm_duality():
    # Maxwell duality (E, H, eps, mu) -> (H, -E, mu, eps): with
    # alpha = -eps0/mu0, A(mu_c, eps_c) [alpha M; J] = [alpha y_M; y_J]; a wrong
    # sign or coefficient on either coupling block breaks it
    n = (5, 4, 3)
    h = 0.004
    f, G, kt, eps_c, mu_c, x = _jm_problem(n, h, 12)
    from oracle import operator as opm
    opn, opk = opm.dense_operator(G), mg.dense_k_operator(kt)
    y = mg.jm_matvec(opn, opk, eps_c, mu_c, x, h, f)
    alpha = -vi.EPS0 / vi.MU0
    yd = mg.jm_matvec(opn, opk, mu_c, eps_c, np.stack([alpha * x[1], x[0]]), h, f)
    np.testing.assert_allclose(yd[0], alpha * y[1], rtol=1e-12, atol=1e-14 * np.abs(alpha * y[1]).max())
    np.testing.assert_allclose(yd[1], y[0], rtol=1e-12, atol=1e-14 * np.abs(y[0]).max())
    # and the coupling is really exercised: K M moves y_J
    y0 = mg.jm_matvec(opn, opk, eps_c, mu_c, np.stack([x[0], 0 * x[1]]), h, f)
    assert np.linalg.norm(y0[0] - y[0]) > 1e-6 * np.linalg.norm(y[0])


def test_jm_solve_without_magnetic_contrast_is_the_electric_solve():
    # chi_h = 0: M = 0 solves the second block row, and J solves the electric
    # equation of the electric-only path
    from oracle import operator as opm, physics
    n = (6, 5, 4)
    h = 0.005
    f, G, kt, eps_c, _, _ = _jm_problem(n, h, 14)
    mu_c = np.ones_like(eps_c)
    opn, opk = opm.dense_operator(G), mg.dense_k_operator(kt)
    e_inc = vi.plane_wave(n, h, f)
    b = mg.jm_rhs(eps_c, mu_c, e_inc, vi.plane_wave_h(n, h, f), f)
    x, info = mg.solve_jm(opn, opk, eps_c, mu_c, b, h, f, tol=1e-11)
    u, _ = physics.solve_currents(opn, eps_c, e_inc, f, tol=1e-11)
    assert np.linalg.norm(x[1]) <= 1e-9 * np.linalg.norm(x[0])
    assert np.linalg.norm(x[0] - u) <= 1e-8 * np.linalg.norm(u)


def test_jm_rhs_duality():
    # Maxwell duality for the right-hand side of eq. 1: with alpha =
    # -eps0/mu0 the dual problem (eps_c and mu_c exchanged, incident fields
    # E' = -H_inc, H' = (eps0/mu0) E_inc) has the right-hand side
    # [alpha b_M; b_J], the same map that test_jm_duality checks for the
    # operator, so [alpha M; J] solves the dual system.  Exchanging c_e and
    # c_m, dropping the sign of either block or putting chi_e on the magnetic
    # block breaks it.
    n = (5, 4, 3)
    h = 0.004
    f, _, _, eps_c, mu_c, _ = _jm_problem(n, h, 15)
    e_inc = vi.random_field(n, 151)
    h_inc = vi.random_field(n, 152)
    b = mg.jm_rhs(eps_c, mu_c, e_inc, h_inc, f)
    alpha = -vi.EPS0 / vi.MU0
    bd = mg.jm_rhs(mu_c, eps_c, -h_inc, (vi.EPS0 / vi.MU0) * e_inc, f)
    np.testing.assert_allclose(bd[0], alpha * b[1], rtol=1e-13, atol=1e-15 * np.abs(alpha * b[1]).max())
    np.testing.assert_allclose(bd[1], b[0], rtol=1e-13, atol=1e-15 * np.abs(b[0]).max())


def test_single_magnetic_voxel_clausius_mossotti():
    # one non-dielectric voxel (eps_c = 1) of relative permeability mu in an
    # incident field, k0 h -> 0: J = 0, Nt_pp(0) -> 2/3, so the magnetic
    # block row of eq. 4 gives M = c_m H_inc 3 chi_h / (mu + 2), i.e. the
    # internal field H = M / (c_m chi_h) = 3 H_inc / (mu + 2) of a small
    # magnetic sphere (the dual of the electric Clausius-Mossotti limit).
    # This fixes the magnetic block of the right-hand side: c_m = i omega mu0,
    # its sign and the magnetic contrast chi_h = mu_c - 1.
    from oracle import operator as opm
    n = (1, 1, 1)
    h = 1e-6
    f = 298e6
    mu = np.full((1, 1, 1), 2.0 - 0.3j)
    eps_c = np.ones((1, 1, 1), complex)
    e_inc = vi.plane_wave(n, h, f)
    h_inc = vi.plane_wave_h(n, h, f)
    opn = opm.dense_operator(vi.green_tensor(n, h, vi.wavenumber(f)))
    opk = mg.dense_k_operator(green_k_tensor(n, h, vi.wavenumber(f)))
    b = mg.jm_rhs(eps_c, mu, e_inc, h_inc, f)
    x, info = mg.solve_jm(opn, opk, eps_c, mu, b, h, f, tol=1e-14)
    cm = 1j * 2 * np.pi * f * vi.MU0
    chi = mu[0, 0, 0] - 1.0
    expect = cm * h_inc[:, 0, 0, 0] * 3.0 * chi / (mu[0, 0, 0] + 2.0)
    assert np.abs(x[0]).max() <= 1e-12 * np.abs(expect).max()
    np.testing.assert_allclose(x[1][:, 0, 0, 0], expect, rtol=1e-9, atol=1e-12 * np.abs(expect).max())
    assert np.abs(expect).max() > 0


def _grad_g_fd(D, kappa, d=1e-3):
    """grad g(|x|) at the point D by central differences of
    g = exp(-i kappa r) / (4 pi r): no parity rule, no generator code."""
    def g(x):
        r = np.sqrt(np.sum(np.square(x)))
        return np.exp(-1j * kappa * r) / (4 * np.pi * r)
    D = np.asarray(D, float)
    return np.array([(g(D + np.eye(3)[s] * d) - g(D - np.eye(3)[s] * d)) / (2 * d) for s in range(3)])


def test_k_entries_at_negative_offsets_follow_the_point_curl_kernel():
    # far from the source Kt_pq = eps_psq d_s g times one scalar, so the ratio
    # of each stored component (xy ~ d_z, xz ~ d_y, yz ~ d_x) to the matching
    # derivative of g must be the same at every sign combination of the
    # offset: pins k_entry's parity rule independently of the embedding
    kappa = 0.05
    kt = green_k_tensor((10, 8, 6), 1.0, kappa)
    base = (9, 7, 5)
    for c, (p, q) in enumerate(mg.K_COMPONENTS):
        s = mg.K_ODD_AXIS[c]
        ref = mg.k_entry(kt, p, q, base) / _grad_g_fd(base, kappa)[s]
        for flips in range(1, 8):
            D = tuple(-x if (flips >> a) & 1 else x for a, x in enumerate(base))
            ratio = mg.k_entry(kt, p, q, D) / _grad_g_fd(D, kappa)[s]
            assert abs(ratio - ref) < 2e-3 * abs(ref), (c, D, ratio, ref)
