"""GPU GMRES solves through the C ABI, checked against the FP64 oracle:
the true residual of the device solution measured with the oracle's own
operator, and the distance to the oracle's GMRES solution."""
import numpy as np
import pytest
import torch

import vie_inputs as vi
from gpu_common import F, K0, problem, rel, say, to_dev
from oracle import operator as opm, physics
from paper_1811_00484_amd import vie

pytestmark = pytest.mark.gpu


def _sphere16():
    # the tiny workload: 16^3 at 5 mm, sphere r = 35 mm (eps_r 52, sigma
    # 0.55 S/m), x-polarised plane wave along z, HOSVD tol 1e-8
    n = (16, 16, 16)
    h = 0.005
    G = vi.green_tensor(n, h, K0)
    er, sg, _ = vi.sphere_phantom(n, h, 0.035, 52.0, 0.55)
    epsc = vi.complex_permittivity(er, sg, F)
    b = vi.rhs_from_field(epsc, vi.plane_wave(n, h, F), F)
    ref = opm.tucker_operator(G, 1e-8)
    return G, epsc, b, ref


def _oracle_residual(ref, epsc, x, b, mode="A"):
    return rel(opm.matvec(ref, epsc, x, mode), b)


def test_solve_c128_tiny_workload():
    say("solve c128 16^3")
    G, epsc, b, ref = _sphere16()
    op = vie.compress(G, tol=1e-8)
    x, info, st = vie.solve(op, to_dev(b, torch.complex128), to_dev(epsc, torch.complex128), tol=1e-8,
                            restart=50)
    assert st == 0 and info[0]["converged"]
    xh = x.cpu().numpy()
    r = _oracle_residual(ref, epsc, xh, b)
    say("   matvecs", info[0]["matvecs"], "oracle residual", r)
    assert r <= 1.01e-8
    xo, _ = physics.solve_currents(ref, epsc, vi.plane_wave((16, 16, 16), 0.005, F), F, tol=1e-10)
    assert rel(xh, xo) <= 1e-6


def test_solve_c64_plain():
    G, epsc, b, ref = _sphere16()
    op = vie.compress(G, tol=1e-8)
    x, info, st = vie.solve(op, to_dev(b, torch.complex64), to_dev(epsc, torch.complex64), tol=1e-5)
    assert info[0]["converged"]
    r = _oracle_residual(ref, epsc, x.cpu().numpy().astype(np.complex128), b)
    say("   c64 oracle residual", r)
    assert r <= 2e-5


def test_refined_solve_reaches_fp64_tolerance():
    G, epsc, b, ref = _sphere16()
    op = vie.compress(G, tol=1e-8)
    x, info, st = vie.solve(op, to_dev(b, torch.complex128), to_dev(epsc, torch.complex128), tol=1e-9,
                            refine=True, inner_tol=1e-4, max_outer=30)
    say("   refined", info[0])
    assert st == 0 and info[0]["converged"] and info[0]["matvecs_fp64"] >= 2
    assert _oracle_residual(ref, epsc, x.cpu().numpy(), b) <= 1.01e-9


def test_adjoint_solve():
    G, epsc, b, ref = _sphere16()
    op = vie.compress(G, tol=1e-8)
    x, info, st = vie.solve(op, to_dev(b, torch.complex128), to_dev(epsc, torch.complex128), tol=1e-9,
                            adjoint=True)
    assert info[0]["converged"]
    assert _oracle_residual(ref, epsc, x.cpu().numpy(), b, "AH") <= 1.01e-9


def test_batched_solve_equals_single_solves():
    n = (12, 10, 9)
    h = 0.004
    G = vi.green_tensor(n, h, K0)
    er, sg, label = vi.head_phantom(n, h * 10, seed=2)
    epsc = vi.complex_permittivity(er, sg, F)
    mask = label >= 0
    rhs = np.stack([vi.rhs_from_field(epsc, vi.dipole_field(n, h, F, p, mask), F)
                    for p in vi.dipole_ring(4, radius=0.05)])
    op = vie.compress(G, tol=1e-6)
    bb = to_dev(rhs, torch.complex128)
    ee = to_dev(epsc, torch.complex128)
    xb, infos, st = vie.solve(op, bb, ee, tol=1e-9, restart=12)
    assert st == 0 and all(i["converged"] for i in infos)
    ref = opm.tucker_operator(G, 1e-6)
    for s in range(4):
        xs, info_s, _ = vie.solve(op, bb[s].contiguous(), ee, tol=1e-9, restart=12)
        assert info_s[0]["matvecs"] == infos[s]["matvecs"]
        assert rel(xb[s].cpu().numpy(), xs.cpu().numpy()) <= 1e-13
        assert _oracle_residual(ref, epsc, xb[s].cpu().numpy(), rhs[s]) <= 1.01e-9


def test_non_convergence_is_reported():
    G, epsc, b, ref = _sphere16()
    op = vie.compress(G, tol=1e-8)
    with pytest.warns(UserWarning):
        x, info, st = vie.solve(op, to_dev(b, torch.complex128), to_dev(epsc, torch.complex128), tol=1e-12,
                                restart=3, max_outer=2)
    assert st == vie.VIE_NOT_CONVERGED and not info[0]["converged"]
    assert len(info[0]["history"]) == 3 and info[0]["rel_residual"] > 1e-12


def test_nonfinite_and_zero_rhs():
    G, epsc, b, ref = _sphere16()
    op = vie.compress(G, tol=1e-8)
    bad = b.copy()
    bad[0, 3, 3, 3] = np.nan
    with pytest.raises(vie.VieError) as ex:
        vie.solve(op, to_dev(bad, torch.complex128), to_dev(epsc, torch.complex128))
    assert ex.value.status == vie.VIE_E_NONFINITE
    x, info, st = vie.solve(op, to_dev(np.zeros_like(b), torch.complex128), to_dev(epsc, torch.complex128))
    assert st == 0 and info[0]["converged"] and torch.count_nonzero(x).item() == 0
