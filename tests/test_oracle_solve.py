"""Pins of the oracle's GMRES, fields and absorbed power: a dense direct
solve, scipy's GMRES, the Clausius-Mossotti limit of one voxel and the Mie
series for a sphere (the paper's own physical reference, Sec. VI-D)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import vie_inputs as vi
from oracle import gmres as gm, operator as opm, physics

F = 298e6
K0 = vi.wavenumber(F)


def _small_problem(n=(4, 3, 5), h=0.01):
    er, sg, _ = vi.sphere_phantom(n, h, 0.02, 52.0, 0.55)
    epsc = vi.complex_permittivity(er, sg, F)
    G = vi.green_tensor(n, h, K0)
    b = vi.rhs_from_field(epsc, vi.plane_wave(n, h, F), F)
    return G, epsc, b


def test_gmres_matches_direct_solve():
    G, epsc, b = _small_problem()
    A = opm.dense_matrix(G, epsc, "A")
    x_ref = np.linalg.solve(A, b.ravel())
    op = opm.dense_operator(G)
    x, info = gm.gmres(lambda v: opm.matvec(op, epsc, v.reshape(b.shape), "A").ravel(), b,
                       tol=1e-12, restart=50)
    assert info.converged
    assert np.linalg.norm(b.ravel() - A @ x) <= 1e-12 * np.linalg.norm(b)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(x - x_ref) <= kappa * 1e-12 * np.linalg.norm(x_ref)


def test_gmres_restarts_and_scipy_cross_check():
    G, epsc, b = _small_problem()
    A = opm.dense_matrix(G, epsc, "A")
    x, info = gm.gmres(lambda v: A @ v, b, tol=1e-9, restart=5, max_outer=400)
    assert info.converged and info.restarts > 0
    xs, code = spla.gmres(A, b.ravel(), rtol=1e-11, restart=50, maxiter=400)
    assert code == 0
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)


def test_gmres_reports_non_convergence():
    G, epsc, b = _small_problem()
    A = opm.dense_matrix(G, epsc, "A")
    x, info = gm.gmres(lambda v: A @ v, b, tol=1e-14, restart=2, max_outer=1)
    assert not info.converged and info.rel_residual > 1e-14
    assert len(info.history) == 2


def test_single_voxel_clausius_mossotti():
    # one voxel, k0 h -> 0: Nt_pp(0) -> 2/3, so u = c_e chi e / (eps - 2 chi/3)
    # = c_e e 3 chi / (eps + 2): the internal field of a small dielectric
    # body, E = 3 e / (eps + 2)
    n = (1, 1, 1)
    h = 1e-6
    epsc = vi.complex_permittivity(np.full((1, 1, 1), 52.0), np.full((1, 1, 1), 0.55), F)
    e = vi.plane_wave(n, h, F)
    op = opm.dense_operator(vi.green_tensor(n, h, K0))
    u, info = physics.solve_currents(op, epsc, e, F, tol=1e-14)
    E = physics.total_field(op, u, e, F)
    cm = 3.0 / (epsc[0, 0, 0] + 2.0)
    assert abs(E[0, 0, 0, 0] - cm) < 1e-9 * abs(cm)
    assert np.abs(E[1:]).max() < 1e-12


def test_mie_limits():
    # Rayleigh limit Q_abs -> 4 x Im((m^2-1)/(m^2+2)) and a lossless sphere
    # absorbs nothing
    f = 1e6
    a = 0.001
    epsc = complex(vi.complex_permittivity(5.0, 0.01, f))
    x = vi.wavenumber(f) * a
    P = physics.mie_absorbed_power(a, epsc, f)
    m2 = np.conj(epsc)
    q_abs = 4 * x * np.imag((m2 - 1) / (m2 + 2))
    eta0 = np.sqrt(vi.MU0 / vi.EPS0)
    P_ray = q_abs * np.pi * a ** 2 / (2 * eta0)
    assert abs(P - P_ray) < 1e-6 * abs(P_ray)
    assert abs(physics.mie_absorbed_power(0.05, 4.0 + 0j, F)) < 1e-15
    assert physics.mie_absorbed_power(0.035, complex(vi.complex_permittivity(52, 0.55, F)), F) > 0


@pytest.mark.slow
def test_sphere_absorbed_power_converges_to_mie():
    # the sphere of the tiny workload (r = 35 mm, eps_r 52, sigma 0.55 S/m,
    # 298 MHz, x-polarised plane wave along z) on 16^3 and 32^3 grids over
    # the same 80 mm box; Mie taken at the equal-volume radius of the
    # staircase sphere.  PWC currents converge at O(h): the error must
    # shrink with h and the O(h)-extrapolated power must be near Mie.
    epsc0 = complex(vi.complex_permittivity(52.0, 0.55, F))
    res = []
    for N in (16, 32):
        h = 0.08 / N
        n = (N, N, N)
        er, sg, mask = vi.sphere_phantom(n, h, 0.035, 52.0, 0.55)
        epsc = vi.complex_permittivity(er, sg, F)
        e = vi.plane_wave(n, h, F)
        op = opm.dense_operator(vi.green_tensor(n, h, K0))
        u, info = physics.solve_currents(op, epsc, e, F, tol=1e-8)
        assert info.converged
        P = physics.absorbed_power(physics.total_field(op, u, e, F), sg, h)
        aeff = (3 * mask.sum() * h ** 3 / (4 * np.pi)) ** (1 / 3)
        res.append((P, physics.mie_absorbed_power(aeff, epsc0, F)))
    e16 = res[0][0] / res[0][1] - 1
    e32 = res[1][0] / res[1][1] - 1
    assert abs(e32) < abs(e16) < 0.5
    extrap = 2 * res[1][0] - res[0][0]
    assert abs(extrap / res[1][1] - 1) < 0.12     # calibrated: 9.3%
