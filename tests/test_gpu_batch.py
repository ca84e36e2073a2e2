"""Multi-instance batches: several phantoms of different grid size and
several right-hand sides each, every matvec pass as one launch over all
instances.  Checked against the FP64 oracle per instance, against
single-instance calls, and by solving every system."""
import numpy as np
import pytest
import torch

import vie_inputs as vi
from gpu_common import F, K0, rel, say, to_dev
from oracle import operator as opm
from paper_1811_00484_amd import vie

pytestmark = pytest.mark.gpu

GRIDS = [(12, 10, 9), (16, 14, 12), (20, 15, 18), (10, 12, 14)]
H = 0.004


def _instances(nrhs=3):
    out = []
    for i, n in enumerate(GRIDS):
        G = vi.green_tensor(n, H, K0)
        er, sg, label = vi.head_phantom(n, H * 6, seed=100 + i)
        epsc = vi.complex_permittivity(er, sg, F)
        mask = np.ones(er.shape, bool)
        dip = vi.dipole_cylinder(nrhs, 0.06, 0.02, seed=400 + i)
        b = np.stack([vi.rhs_from_field(epsc, vi.dipole_field(n, H, F, p, mask), F) for p in dip])
        out.append((n, G, epsc, b, opm.tucker_operator(G, 1e-6), vie.compress(G, tol=1e-6)))
    return out


@pytest.fixture(params=[0, 1], ids=["per_instance_launches", "one_launch_per_pass"])
def batch_mode(request):
    vie.set_batch_mode(request.param)
    yield request.param
    vie.set_batch_mode(0)


@pytest.mark.parametrize("dt", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("mode", ["A", "AH"])
def test_multi_matvec_matches_oracle_and_single(dt, mode, batch_mode):
    say("multi matvec", dt, mode, "batch mode", batch_mode)
    insts = _instances()
    items = []
    us = []
    for k, (n, G, epsc, b, ref, op) in enumerate(insts):
        u = vi.random_field(n, 30 + k, nrhs=2 + k % 2)
        us.append(u)
        items.append((op, to_dev(u, dt), to_dev(epsc, dt)))
    ys = vie.matvec_multi(items, kind="A", adjoint=(mode == "AH"))
    tol = 1e-5 if dt == torch.complex64 else 1e-12
    for k, (n, G, epsc, b, ref, op) in enumerate(insts):
        y = ys[k].cpu().numpy()
        for s in range(us[k].shape[0]):
            err = rel(y[s].astype(np.complex128), opm.matvec(ref, epsc, us[k][s], mode))
            assert err <= tol, (k, s, err)
        y1 = vie.matvec(op, items[k][1], items[k][2], adjoint=(mode == "AH")).cpu().numpy()
        assert rel(y, y1) <= (1e-6 if dt == torch.complex64 else 1e-13)


def test_multi_solve_all_systems(batch_mode):
    insts = _instances()
    items = [(op, to_dev(b, torch.complex128), to_dev(epsc, torch.complex128))
             for (n, G, epsc, b, ref, op) in insts]
    res, st = vie.solve_multi(items, tol=1e-9, restart=20)
    assert st == 0
    for (x, infos), (n, G, epsc, b, ref, op) in zip(res, insts):
        assert all(i["converged"] for i in infos)
        xh = x.cpu().numpy()
        for s in range(b.shape[0]):
            assert rel(opm.matvec(ref, epsc, xh[s], "A"), b[s]) <= 1.01e-9
    # the lockstep batch gives each system the same iterates as its own solve
    n, G, epsc, b, ref, op = insts[2]
    xs, infos, _ = vie.solve(op, to_dev(b, torch.complex128), to_dev(epsc, torch.complex128), tol=1e-9, restart=20)
    assert rel(res[2][0].cpu().numpy(), xs.cpu().numpy()) <= 1e-10
    assert [i["matvecs"] for i in infos] == [i["matvecs"] for i in res[2][1]]


def test_multi_solve_warm_start_continues():
    # restarted GMRES split over two calls (the second warm-started from the
    # first's iterate) reaches the same tolerance
    insts = _instances(nrhs=2)
    items = [(op, to_dev(b, torch.complex128), to_dev(epsc, torch.complex128))
             for (n, G, epsc, b, ref, op) in insts]
    res1, st1 = vie.solve_multi(items, tol=1e-9, restart=5, max_outer=2)
    res2, st2 = vie.solve_multi(items, tol=1e-9, restart=20, x0=[x for x, _ in res1])
    assert st2 == 0
    for (x, infos), (n, G, epsc, b, ref, op) in zip(res2, insts):
        xh = x.cpu().numpy()
        for s in range(b.shape[0]):
            assert rel(opm.matvec(ref, epsc, xh[s], "A"), b[s]) <= 1.01e-9


# grids whose every FFT length has register-FFT kernels (2n in 128/192/224/256
# on x, y; 128/256 on z): the default batch mode runs them as one launch per
# pass and FFT length, with per-instance descriptors in the kernel arguments
FAST_GRIDS = [(64, 64, 64), (64, 96, 64), (96, 64, 128), (64, 112, 64)]


def _fast_instances(grids, nrhs_of=lambda k: 2 + k % 2, h=0.003):
    out = []
    for k, n in enumerate(grids):
        G = vi.green_tensor(n, h, K0)
        er, sg, label = vi.head_phantom(n, h, seed=200 + k)
        epsc = vi.complex_permittivity(er, sg, F)
        out.append((n, epsc, opm.tucker_operator(G, 1e-6), vie.compress(G, tol=1e-6), nrhs_of(k)))
    return out


@pytest.mark.parametrize("dt", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("mode", ["A", "AH"])
def test_grouped_register_fft_batch_equals_single_calls(dt, mode):
    say("grouped batch", dt, mode)
    insts = _fast_instances(FAST_GRIDS)
    items, us = [], []
    for k, (n, epsc, ref, op, nr) in enumerate(insts):
        u = vi.random_field(n, 60 + k, nrhs=nr)
        us.append(u)
        items.append((op, to_dev(u, dt), to_dev(epsc, dt)))
    ys = vie.matvec_multi(items, kind="A", adjoint=(mode == "AH"))
    for k, (n, epsc, ref, op, nr) in enumerate(insts):
        y1 = vie.matvec(op, items[k][1], items[k][2], adjoint=(mode == "AH"))
        assert torch.equal(ys[k], y1), k          # same kernels and order: bitwise
        y = ys[k].cpu().numpy()
        for s in range(nr):
            err = rel(y[s].astype(np.complex128), opm.matvec(ref, epsc, us[k][s], mode))
            # complex128: the two sides' HOSVDs at tol 1e-6 differ by ~1e-9 on
            # these unfoldings (Gram eigenvectors vs SVD; FP64 parity at a
            # refined 1e-8 operator is in test_gpu_fast.py)
            assert err <= (1e-5 if dt == torch.complex64 else 1e-8), (k, s, err)


def test_grouped_batch_splits_large_groups():
    # ten instances of one grid: more than one z launch is needed per group
    n = (64, 64, 64)
    G = vi.green_tensor(n, 0.003, K0)
    ref = opm.tucker_operator(G, 1e-6)
    op = vie.compress(G, tol=1e-6)
    items, refs = [], []
    for k in range(10):
        er, sg, label = vi.head_phantom(n, 0.003, seed=300 + k)
        epsc = vi.complex_permittivity(er, sg, F)
        u = vi.random_field(n, 90 + k)
        items.append((op, to_dev(u, torch.complex64), to_dev(epsc, torch.complex64)))
        refs.append((epsc, u))
    ys = vie.matvec_multi(items)
    for k, (epsc, u) in enumerate(refs):
        err = rel(ys[k].cpu().numpy().reshape(u.shape).astype(np.complex128), opm.matvec(ref, epsc, u, "A"))
        assert err <= 1e-5, (k, err)


def test_grouped_batch_solve():
    insts = _fast_instances(FAST_GRIDS[:3], nrhs_of=lambda k: 2)
    items, bs = [], []
    for k, (n, epsc, ref, op, nr) in enumerate(insts):
        dip = vi.dipole_cylinder(nr, 0.25, 0.02, seed=500 + k)   # outside every grid
        mask = np.ones(epsc.shape, bool)
        b = np.stack([vi.rhs_from_field(epsc, vi.dipole_field(n, 0.003, F, p, mask), F) for p in dip])
        bs.append(b)
        items.append((op, to_dev(b, torch.complex128), to_dev(epsc, torch.complex128)))
    res, st = vie.solve_multi(items, tol=1e-8, restart=30, refine=True, inner_tol=1e-5)
    assert st == 0
    for (x, infos), (n, epsc, ref, op, nr), b in zip(res, insts, bs):
        xh = x.cpu().numpy()
        for s in range(nr):
            assert rel(opm.matvec(ref, epsc, xh[s], "A"), b[s]) <= 1.05e-8
