"""Pins of the piecewise-linear Galerkin tensors (eq. 7b, 8a-8b).

The generator reduces each 6-D Galerkin integral to a 3-D integral against
per-axis correlation functions of the basis and handles the singular part
distributionally.  The checks below come from outside that derivation: a
6-D brute-force integral over the test and basis voxels (far offsets), the
static trace identity of curl curl (near offsets), the pulse tensor, the
symmetries of the Galerkin matrix, and quadrature convergence."""
import numpy as np
import pytest

from vie_inputs import PWL_PAIRS, green_pwl_entry, green_pwl_tensor, green_tensor, pwl_pair_index

COMP = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
MASS = (1.0, 1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0)


def _ghat(r, kappa):
    return np.exp(-1j * kappa * r) / (4 * np.pi * r)


def _dyadic(R, kappa):
    """(kappa^2 delta_pq + d_p d_q) g^ at displacements R (..., 3), six
    components, from the derivatives of exp(-i kappa r) / (4 pi r)."""
    r2 = np.sum(R * R, axis=-1)
    r = np.sqrt(r2)
    g = _ghat(r, kappa)
    ikr = 1j * kappa * r
    diag = g * (kappa ** 2 - (1 + ikr) / r2)
    radial = g * (3 + 3 * ikr - kappa ** 2 * r2) / (r2 * r2)
    out = []
    for p, q in COMP:
        v = radial * R[..., p] * R[..., q]
        if p == q:
            v = v + diag
        out.append(v)
    return np.stack(out, axis=-1)


def test_dyadic_helper_by_finite_differences():
    # the helper above against central differences of g^ itself
    kappa, x0, h = 0.7, np.array([1.3, -0.4, 2.1]), 1e-4
    G = _dyadic(x0[None, :], kappa)[0]
    for c, (p, q) in enumerate(COMP):
        ep, eq = np.eye(3)[p] * h, np.eye(3)[q] * h
        f = lambda y: _ghat(np.linalg.norm(y), kappa)
        d2 = (f(x0 + ep + eq) - f(x0 + ep - eq) - f(x0 - ep + eq) + f(x0 - ep - eq)) / (4 * h * h)
        if p == q:
            d2 += kappa ** 2 * f(x0)
        assert abs(d2 - G[c]) < 1e-6 * abs(G[c]) + 1e-9


def _brute6(D, kappa, q=8):
    """<C^l of voxel 0, Gd C^l' of voxel D> for all 16 (l, l') by a tensor
    Gauss rule on both voxels (6-D, smooth when the voxels are apart)."""
    x, w = np.polynomial.legendre.leggauss(q)
    x = 0.5 * x
    w = 0.5 * w
    T = np.stack(np.meshgrid(x, x, x, indexing="ij"), axis=-1).reshape(-1, 3)
    W = np.einsum("i,j,k->ijk", w, w, w).reshape(-1)
    R = (np.asarray(D, float)[None, None, :] + T[None, :, :]) - T[:, None, :]   # r' - r
    Gd = _dyadic(R, kappa)                                                     # (test, basis, 6)
    phi = np.concatenate([np.ones((T.shape[0], 1)), T], axis=1)               # C^0..C^3 at nodes
    out = np.empty((4, 4, 6), complex)
    for l in range(4):
        for lp in range(4):
            wt = (W * phi[:, l])[:, None] * (W * phi[:, lp])[None, :]
            out[l, lp] = np.einsum("ab,abc->c", wt, Gd)
    return out


@pytest.mark.parametrize("D", [(3, 0, 0), (3, 2, 1), (0, 4, 2), (4, 4, 3)])
def test_far_entries_match_six_dim_integral(D):
    kappa = 0.45
    B = _brute6(D, kappa)
    E = green_pwl_entry(D, kappa, 12, method=1)
    for l in range(4):
        for lp in range(4):
            P, sign = pwl_pair_index(l, lp)
            scale = np.abs(B[l, lp]).max()
            np.testing.assert_allclose(sign * E[P], B[l, lp], rtol=0, atol=2e-9 * scale + 1e-15,
                                       err_msg="pair (%d,%d)" % (l, lp))


def test_fill_uses_the_far_form_beyond_the_near_shell():
    G = green_pwl_tensor((5, 4, 3), 1.0, 0.3)
    for D in [(2, 0, 0), (4, 3, 2), (0, 2, 1)]:
        E = green_pwl_entry(D, 0.3, 12, method=1)
        np.testing.assert_allclose(G[:, :, D[2], D[1], D[0]], E, rtol=0, atol=1e-11)


@pytest.mark.parametrize("D", [(2, 0, 0), (2, 1, 1), (3, 2, 0), (-2, 1, 0), (1, 2, -3)])
def test_distributional_form_equals_dyadic_form_where_both_apply(D):
    # the plane (point-mass) terms and regular second derivatives of the
    # correlation functions against the smooth dyadic form
    a = green_pwl_entry(D, 0.35, 16, method=0)
    b = green_pwl_entry(D, 0.35, 16, method=1)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * np.abs(b).max())


def test_static_trace_identity_near_offsets():
    # (lap + kappa^2) g^ = -delta: sum_p Nt^(l,l')_pp(D) = 2 m_l d_ll' d_D0 at
    # kappa = 0 for every near offset, both signs
    for D in [(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)]:
        E = green_pwl_entry(D, 0.0, 16, method=0)
        tr = E[:, 0] + E[:, 1] + E[:, 2]
        expect = np.zeros(10)
        if D == (0, 0, 0):
            for P, (l, lp) in enumerate(PWL_PAIRS):
                expect[P] = 2 * MASS[l] if l == lp else 0.0
        np.testing.assert_allclose(tr, expect, atol=1e-13, err_msg=str(D))


def test_pulse_pair_equals_pulse_tensor():
    G = green_pwl_tensor((6, 5, 4), 1.0, 0.3)
    P0 = green_tensor((6, 5, 4), 1.0, 0.3)
    np.testing.assert_allclose(G[0], P0, rtol=0, atol=1e-13)


def _odd(P, c, a):
    l, lp = PWL_PAIRS[P]
    p, q = COMP[c]
    return ((p == a) + (q == a) + (l == a + 1) + (lp == a + 1)) % 2


def test_parities_and_reciprocity():
    # reflecting axis a flips the sign of x_a, of the a-components of both
    # vectors and of the linear functions along a
    kappa = 0.3
    for D in [(1, 0, 1), (2, 1, 0), (1, 1, 1), (3, 1, 2)]:
        E = green_pwl_entry(D, kappa, 14, method=0)
        for a in range(3):
            Dm = list(D)
            Dm[a] = -Dm[a]
            Em = green_pwl_entry(Dm, kappa, 14, method=0)
            for P in range(10):
                for c in range(6):
                    s = -1.0 if _odd(P, c, a) else 1.0
                    assert abs(Em[P, c] - s * E[P, c]) < 1e-13, (D, a, P, c)
        # reciprocity of the Galerkin matrix: Nt^{(l,l')}(-D) = Nt^{(l',l)}(D)
        En = green_pwl_entry([-d for d in D], kappa, 14, method=0)
        for P, (l, lp) in enumerate(PWL_PAIRS):
            _, sign = pwl_pair_index(lp, l)
            np.testing.assert_allclose(En[P], sign * E[P], rtol=0, atol=1e-13)


def test_odd_components_vanish_on_their_zero_planes():
    G = green_pwl_tensor((4, 4, 3), 1.0, 0.5)
    for P in range(10):
        for c in range(6):
            for a in range(3):
                if not _odd(P, c, a):
                    continue
                sl = [P, c, slice(None), slice(None), slice(None)]
                sl[4 - a] = 0
                assert np.abs(G[tuple(sl)]).max() < 1e-14, (P, c, a)


@pytest.mark.parametrize("D", [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1)])
def test_near_quadrature_converges(D):
    a = green_pwl_entry(D, 0.5, 12, method=0)
    b = green_pwl_entry(D, 0.5, 24, method=0)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-10)


def test_plane_wave_moments_match_closed_forms():
    # x-polarised exp(-i k0 z): pulse moment = sinc(a/2) exp(-i k0 z_m),
    # z-linear moment = i (a cos(a/2) - 2 sin(a/2)) / a^2 exp(-i k0 z_m),
    # a = k0 h; the x- and y-linear moments and the other components vanish
    import vie_inputs as vi
    n, h, f = (4, 3, 5), 0.01, 3e9
    m = vi.plane_wave_pwl(n, h, f)
    k0 = vi.wavenumber(f)
    a = k0 * h
    _, _, z = vi.voxel_centres(n, h)
    ez = np.exp(-1j * k0 * z)
    np.testing.assert_allclose(m[0, 0], np.sin(a / 2) / (a / 2) * ez, rtol=0, atol=1e-14)
    np.testing.assert_allclose(m[3, 0], 1j * (a * np.cos(a / 2) - 2 * np.sin(a / 2)) / a ** 2 * ez, rtol=0,
                               atol=1e-14)
    assert np.abs(m[1:3]).max() < 1e-15 and np.abs(m[:, 1:]).max() == 0.0


# ---------------- the magnetic operator K in the PWL basis ----------------

def _dg(R, kappa):
    """grad g^ at displacements R (..., 3)."""
    r2 = np.sum(R * R, axis=-1)
    r = np.sqrt(r2)
    f = -_ghat(r, kappa) * (1 + 1j * kappa * r) / r2
    return f[..., None] * R


def test_grad_helper_by_finite_differences():
    kappa, x0, h = 0.6, np.array([1.7, 0.4, -2.2]), 1e-5
    g = _dg(x0[None, :], kappa)[0]
    for s in range(3):
        e = np.eye(3)[s] * h
        fd = (_ghat(np.linalg.norm(x0 + e), kappa) - _ghat(np.linalg.norm(x0 - e), kappa)) / (2 * h)
        assert abs(fd - g[s]) < 1e-8 * abs(g[s])


def _brute6_k(D, kappa, q=8):
    """<C^l_D e_p, K C^l'_0 e_q> for the stored components xy, xz, yz of all
    16 (l, l'): test function in the observation voxel D, basis function in
    the source voxel 0, (curl g e_q)_p = eps_psq d_s g, 6-D Gauss rule."""
    x, w = np.polynomial.legendre.leggauss(q)
    x, w = 0.5 * x, 0.5 * w
    T = np.stack(np.meshgrid(x, x, x, indexing="ij"), axis=-1).reshape(-1, 3)
    W = np.einsum("i,j,k->ijk", w, w, w).reshape(-1)
    R = (np.asarray(D, float)[None, None, :] + T[:, None, :]) - T[None, :, :]   # r_obs - r_src
    G = _dg(R, kappa)                                                          # (obs, src, 3)
    comp = np.stack([-G[..., 2], G[..., 1], -G[..., 0]], axis=-1)              # xy, xz, yz
    phi = np.concatenate([np.ones((T.shape[0], 1)), T], axis=1)
    out = np.empty((4, 4, 3), complex)
    for l in range(4):
        for lp in range(4):
            wt = (W * phi[:, l])[:, None] * (W * phi[:, lp])[None, :]
            out[l, lp] = np.einsum("ab,abc->c", wt, comp)
    return out


def test_pwl_k_pulse_pair_equals_the_pulse_k():
    from vie_inputs import green_k_tensor, green_pwl_k_tensor
    K = green_pwl_k_tensor((6, 5, 4), 1.0, 0.3)
    np.testing.assert_allclose(K[0], green_k_tensor((6, 5, 4), 1.0, 0.3), rtol=0, atol=1e-13)


@pytest.mark.parametrize("D", [(3, 0, 0), (3, 2, 1), (0, 4, 2), (-3, 2, 4)])
def test_pwl_k_far_entries_match_six_dim_integral(D):
    from vie_inputs import green_pwl_k_entry
    kappa = 0.45
    B = _brute6_k(D, kappa)
    E = green_pwl_k_entry(D, kappa, 12, method=1)
    for l in range(4):
        for lp in range(4):
            P, sign = pwl_pair_index(l, lp)
            scale = np.abs(B[l, lp]).max()
            np.testing.assert_allclose(sign * E[P], B[l, lp], rtol=0, atol=2e-9 * scale + 1e-15,
                                       err_msg="pair (%d,%d)" % (l, lp))


@pytest.mark.parametrize("D", [(2, 0, 0), (2, 1, 1), (3, -2, 0), (1, 2, -3)])
def test_pwl_k_volume_form_equals_smooth_form(D):
    from vie_inputs import green_pwl_k_entry
    a = green_pwl_k_entry(D, 0.35, 16, method=0)
    b = green_pwl_k_entry(D, 0.35, 16, method=1)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * np.abs(b).max())


def _odd_k(P, c, a):
    l, lp = PWL_PAIRS[P]
    s = 2 - c                      # xy <- F_z, xz <- F_y, yz <- F_x
    return ((s == a) + (l == a + 1) + (lp == a + 1)) % 2


def test_pwl_k_zero_planes_parities_and_entries():
    from vie_inputs import green_pwl_k_entries, green_pwl_k_entry, green_pwl_k_tensor
    kappa, n = 0.5, (5, 4, 3)
    K = green_pwl_k_tensor(n, 1.0, kappa)
    for P in range(10):
        for c in range(3):
            for a in range(3):
                if _odd_k(P, c, a):
                    sl = [P, c, slice(None), slice(None), slice(None)]
                    sl[4 - a] = 0
                    assert np.abs(K[tuple(sl)]).max() == 0.0, (P, c, a)
    for D in [(1, 0, 1), (2, 1, 0), (3, 1, 2)]:
        E = green_pwl_k_entry(D, kappa, 14, method=0)
        for a in range(3):
            Dm = list(D)
            Dm[a] = -Dm[a]
            Em = green_pwl_k_entry(Dm, kappa, 14, method=0)
            for P in range(10):
                for c in range(3):
                    s = -1.0 if _odd_k(P, c, a) else 1.0
                    assert abs(Em[P, c] - s * E[P, c]) < 1e-13, (D, a, P, c)
    idx = np.array([[i, j, k] for k in range(n[2]) for j in range(n[1]) for i in range(n[0])])
    for comp in (0, 7, 17, 29):
        e = green_pwl_k_entries(idx, comp, 1.0, kappa)
        np.testing.assert_allclose(e, K[comp // 3, comp % 3].reshape(-1), rtol=0, atol=1e-15)


@pytest.mark.parametrize("D", [(0, 0, 1), (1, 0, 0), (1, 1, 0), (1, 1, 1)])
def test_pwl_k_near_quadrature_converges(D):
    from vie_inputs import green_pwl_k_entry
    a = green_pwl_k_entry(D, 0.5, 12, method=0)
    b = green_pwl_k_entry(D, 0.5, 24, method=0)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-10)
