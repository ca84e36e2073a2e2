"""Pins of the Galerkin Green's tensor (problem data shared by the oracle and
the GPU path).  Each check is an identity of the operator N = curl curl int g
(eq. 5-6) that a plausible mistake (a wrong sign of a derivative term, a
dropped plane integral, a transposed axis) breaks."""
import numpy as np
import pytest

import vie_inputs as vi
from vie_inputs import green_tensor


def _ghat(r, kappa):
    return np.exp(-1j * kappa * r) / (4 * np.pi * r)


def _gl(q):
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def _far_J0(D, kappa, q=12):
    """int g^ tau_D over the support (smooth when max D >= 2), tensor Gauss on
    the 8 kink cells -- an independent numpy quadrature of the volume term."""
    x, w = _gl(q)
    acc = 0j
    for cell in range(8):
        lo = [0.0 if (cell >> a) & 1 else -1.0 for a in range(3)]
        t = [lo[a] + x for a in range(3)]
        T0, T1, T2 = np.meshgrid(t[0], t[1], t[2], indexing="ij")
        W = np.einsum("i,j,k->ijk", w * (1 - np.abs(t[0])), w * (1 - np.abs(t[1])),
                      w * (1 - np.abs(t[2])))
        r = np.sqrt((D[0] + T0) ** 2 + (D[1] + T1) ** 2 + (D[2] + T2) ** 2)
        acc += np.sum(W * _ghat(r, kappa))
    return acc


def test_static_self_term():
    # kappa -> 0: the diagonal self term is 1 - 1/3 = 2/3 (the depolarisation
    # of a cube), off-diagonal self terms vanish by symmetry
    G = green_tensor((2, 2, 2), 1.0, 1e-9)
    np.testing.assert_allclose(G[:3, 0, 0, 0], 2.0 / 3.0, atol=1e-13)
    np.testing.assert_allclose(G[3:, 0, 0, 0], 0.0, atol=1e-13)


def test_static_trace_near_offsets():
    # sum_p Nt_pp(D) = 2 delta_D0 + 2 kappa^2 J0(D); at kappa = 0 the three
    # plane integrals of each near offset must cancel exactly
    G = green_tensor((3, 3, 3), 1.0, 0.0)
    tr = G[0] + G[1] + G[2]
    expect = np.zeros_like(tr)
    expect[0, 0, 0] = 2.0
    np.testing.assert_allclose(tr, expect, atol=1e-12)


@pytest.mark.parametrize("D", [(2, 0, 0), (2, 1, 1), (3, 2, 0), (5, 4, 3)])
def test_trace_identity_far(D):
    kappa = 0.4
    G = green_tensor((6, 6, 6), 1.0, kappa)
    tr = G[0, D[2], D[1], D[0]] + G[1, D[2], D[1], D[0]] + G[2, D[2], D[1], D[0]]
    J0 = _far_J0(D, kappa)
    np.testing.assert_allclose(tr, 2 * kappa ** 2 * J0, rtol=1e-10)


def test_parity_zeros_and_axis_permutation():
    G = green_tensor((5, 5, 5), 1.0, 0.2)
    xx, yy, zz, xy, xz, yz = G
    # odd components vanish on the plane where their odd axis offset is 0
    assert np.abs(xy[:, :, 0]).max() < 1e-13 and np.abs(xy[:, 0, :]).max() < 1e-13
    assert np.abs(xz[:, :, 0]).max() < 1e-13 and np.abs(xz[0, :, :]).max() < 1e-13
    assert np.abs(yz[:, 0, :]).max() < 1e-13 and np.abs(yz[0, :, :]).max() < 1e-13
    # cubic voxels: swapping x and y maps xx <-> yy, xz <-> yz
    np.testing.assert_allclose(yy, np.transpose(xx, (0, 2, 1)), rtol=0, atol=1e-14)
    np.testing.assert_allclose(zz, np.transpose(xx, (2, 1, 0)), rtol=0, atol=1e-14)
    np.testing.assert_allclose(yz, np.transpose(xz, (0, 2, 1)), rtol=0, atol=1e-14)
    np.testing.assert_allclose(xy, np.transpose(xy, (0, 2, 1)), rtol=0, atol=1e-14)


def test_far_field_matches_point_dyadic():
    # Nt(D) = int Gd(D + t) prod(1 - |t_i|) dt.  The tent weights have unit
    # mass and second moment 1/6, and Gd solves the Helmholtz equation away
    # from 0, so Nt(D) = Gd(D) (1 - kappa^2/12) + O(|D|^-4) relative.
    kappa = 0.05
    G = green_tensor((33, 2, 2), 1.0, kappa)
    from vie_inputs import _native
    errs = []
    for d in (4, 8, 16):
        pts = np.array([[float(d), 0.0, 0.0]])
        out = np.empty((1, 6, 2))
        _native.lib().vie_dyadic_points(1, pts.ctypes.data, kappa, out.ctypes.data)
        ref = (out[0, 0, 0] + 1j * out[0, 0, 1]) * (1 - kappa ** 2 / 12)
        errs.append(abs(G[0, 0, 0, d] - ref) / abs(ref))
    errs = np.array(errs)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios > 12) and np.all(ratios < 20), (errs, ratios)


def test_quadrature_converged():
    a = green_tensor((7, 6, 5), 1.0, 0.3)
    b = green_tensor((7, 6, 5), 1.0, 0.3, near_order=28, far_boost=6)
    assert np.abs(a - b).max() <= 1e-11 * np.abs(b).max()


def test_kappa_scaling():
    # entries depend only on kappa = k0 h
    a = green_tensor((4, 3, 2), 0.002, 6.0)
    b = green_tensor((4, 3, 2), 0.004, 3.0)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


def test_dipole_field_far_zone():
    # far from a z-dipole in the equatorial plane E_z ~ -(I l) i omega mu0
    # exp(-i k r) / (4 pi r) (radiation field, exp(+i omega t) convention)
    f = 298e6
    k0 = vi.wavenumber(f)
    n = (1, 1, 1)
    h = 1e-3
    r = 40.0 / k0
    e = vi.dipole_field(n, h, f, (-r, 0.0, 0.0), np.ones((1, 1, 1), bool))
    ref = -1j * vi.omega(f) * vi.MU0 * np.exp(-1j * k0 * r) / (4 * np.pi * r)
    assert abs(e[2, 0, 0, 0] - ref) / abs(ref) < 0.03
