"""Pins of the oracle's FFT-VIE operator: FFT convolution against the
explicit Toeplitz sum, commutation of embedding/FFT with the Tucker form
(Sec. V-A), symmetry and the adjoint identity."""
import numpy as np
import pytest

import vie_inputs as vi
from oracle import circulant, operator as opm, tucker

F = 298e6
K0 = vi.wavenumber(F)


@pytest.mark.parametrize("n", [(3, 4, 5), (4, 4, 4), (1, 3, 2)])
def test_fft_convolution_equals_direct_sum(n):
    G = vi.green_tensor(n, 0.01, K0)
    u = vi.random_field(n, 11)
    y_fft = opm.apply_N(opm.dense_operator(G), u)
    y_dir = opm.brute_force_N(G, u)
    assert np.linalg.norm(y_fft - y_dir) <= 1e-13 * np.linalg.norm(y_dir)


def test_fft_convolution_random_tensor():
    # a random (non-physical) defining tensor: the FFT path must still equal
    # the direct sum -- catches embedding-sign and index errors that a smooth
    # physical tensor could hide
    n = (4, 3, 5)
    G = vi.random_complex((6, n[2], n[1], n[0]), 3)
    for c in range(6):                       # respect the component parities
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
    assert np.linalg.norm(y_fft - y_dir) <= 1e-13 * np.linalg.norm(y_dir)


def test_tucker_commutes_with_embedding_and_fft():
    n = (6, 5, 7)
    rng = np.random.default_rng(2)
    Gc = rng.standard_normal((3, 2, 4)) + 1j * rng.standard_normal((3, 2, 4))
    Us = [rng.standard_normal((m, r)) + 1j * rng.standard_normal((m, r))
          for m, r in zip(n, Gc.shape)]
    for c in range(6):
        s = circulant.axis_signs(c)
        Us_c = [U.copy() for U in Us]
        for a in range(3):
            if s[a] < 0:
                Us_c[a][0] = 0           # odd along axis a: zero offset vanishes
        A = tucker.tucker_reconstruct(Gc, *Us_c)
        lhs = circulant.fourier_tensor_dense(A, s)
        rhs = circulant.fourier_tensor_tucker(Gc, Us_c, s)
        assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(lhs)


def test_fourier_tensor_symmetries():
    # N^[L - k] = s N^[k] along each axis; full-offset parity is even
    n = (5, 4, 6)
    G = vi.green_tensor(n, 0.005, K0)
    op = opm.dense_operator(G)
    for c in range(6):
        Nh = op.nhat[c]
        s = circulant.axis_signs(c)
        for a in range(3):
            L = Nh.shape[a]
            flipped = np.take(Nh, [(-k) % L for k in range(L)], axis=a)
            np.testing.assert_allclose(flipped, s[a] * Nh, atol=1e-12 * np.abs(Nh).max())
            # the middle index n carries zero when odd
            if s[a] < 0:
                assert np.abs(np.take(Nh, [n[a]], axis=a)).max() < 1e-12 * np.abs(Nh).max()


def test_matrix_is_complex_symmetric():
    n = (2, 3, 2)
    G = vi.green_tensor(n, 0.01, K0)
    M = opm.dense_matrix(G)
    np.testing.assert_allclose(M, M.T, atol=1e-14)


def test_adjoint_identity_and_dense_matrix():
    n = (3, 3, 4)
    er, sg, _ = vi.sphere_phantom(n, 0.01, 0.012, 40.0, 0.8)
    epsc = vi.complex_permittivity(er, sg, F)
    G = vi.green_tensor(n, 0.01, K0)
    op = opm.dense_operator(G)
    x = vi.random_field(n, 21)
    y = vi.random_field(n, 22)
    Ax = opm.matvec(op, epsc, x, "A")
    AHy = opm.matvec(op, epsc, y, "AH")
    lhs = np.vdot(y, Ax)            # <Ax, y> with the inner product of App. I
    rhs = np.vdot(AHy, x)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    A = opm.dense_matrix(G, epsc, "A")
    np.testing.assert_allclose(Ax.ravel(), A @ x.ravel(), rtol=0, atol=1e-12 * np.abs(Ax).max())
    np.testing.assert_allclose(AHy.ravel(), A.conj().T @ y.ravel(), rtol=0,
                               atol=1e-12 * np.abs(AHy).max())


def test_tucker_operator_error_tracks_tolerance():
    n = (12, 10, 9)
    G = vi.green_tensor(n, 0.005, K0)
    u = vi.random_field(n, 5)
    epsc = vi.complex_permittivity(np.full(n[::-1], 50.0), np.full(n[::-1], 0.6), F)
    ref = opm.matvec(opm.dense_operator(G), epsc, u, "A")
    prev = np.inf
    for tol in (1e-2, 1e-4, 1e-6, 1e-8):
        op = opm.tucker_operator(G, tol)
        err = np.linalg.norm(opm.matvec(op, epsc, u, "A") - ref) / np.linalg.norm(ref)
        assert err < prev
        assert err < 50 * tol
        prev = err


def _dyadic_fd(D, kappa, d=1e-3):
    """(d_p d_q + kappa^2 delta_pq) g(|x|) at the point D by central
    differences of g = exp(-i kappa r) / (4 pi r): the point dyadic written
    from g alone, with no parity rule and no generator code."""
    def g(x):
        r = np.sqrt(np.sum(np.square(x)))
        return np.exp(-1j * kappa * r) / (4 * np.pi * r)
    D = np.asarray(D, float)
    out = np.empty((3, 3), complex)
    for p in range(3):
        for q in range(3):
            ep, eq = np.eye(3)[p] * d, np.eye(3)[q] * d
            out[p, q] = (g(D + ep + eq) - g(D + ep - eq) - g(D - ep + eq) + g(D - ep - eq)) / (4 * d * d)
            if p == q:
                out[p, q] += kappa ** 2 * g(D)
    return out


def test_signed_entries_at_negative_offsets_follow_the_point_dyadic():
    # far from the source the tensor is the point dyadic times one scalar
    # (the tent average, 1 - kappa^2/12, and the generator's sign and
    # normalisation convention), so the ratio of each component to the
    # dyadic must be the same at every sign combination of the offset: this
    # pins the parity rule of signed_entry (and of the embedding, which
    # shares it) against an evaluation that uses no parity at all
    kappa = 0.05
    G = vi.green_tensor((10, 8, 6), 1.0, kappa)
    base = (9, 7, 5)
    for c, (p, q) in enumerate(circulant.COMPONENTS):
        ref = opm.signed_entry(G, c, base) / _dyadic_fd(base, kappa)[p, q]
        for flips in range(1, 8):
            D = tuple(-x if (flips >> a) & 1 else x for a, x in enumerate(base))
            ratio = opm.signed_entry(G, c, D) / _dyadic_fd(D, kappa)[p, q]
            assert abs(ratio - ref) < 2e-3 * abs(ref), (c, D, ratio, ref)
