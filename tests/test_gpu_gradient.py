"""Adjoint gradients through the torch.autograd.Function against the FP64
oracle's adjoint gradient and against central finite differences of
complex128 device solves (the differentiation workload shrunk to 32^3 at
2 mm: head phantom scale 0.25, x-polarised plane wave, targets drawn from the
tissue voxels)."""
import numpy as np
import pytest
import torch

import vie_inputs as vi
from gpu_common import F, K0, device, rel, say, to_dev
from oracle import gradient as ograd, operator as opm, physics
from paper_1811_00484_amd import vie
from paper_1811_00484_amd.autograd import total_field

pytestmark = pytest.mark.gpu

N = (32, 32, 32)
H = 0.002


def _setup():
    G = vi.green_tensor(N, H, K0)
    er, sg, label = vi.head_phantom(N, H, seed=2)
    e_inc = vi.plane_wave(N, H, F)
    ref = opm.tucker_operator(G, 1e-6)
    rng = np.random.default_rng(50)
    tissue = np.nonzero(label.ravel() >= 0)[0]
    targets = np.sort(rng.choice(tissue, 50, replace=False))
    # target field from the 5%-perturbed phantom (FP64 oracle solve)
    rng2 = np.random.default_rng(51)
    t_mask = label >= 0
    er_t = er * np.where(t_mask, 1 + 0.05 * rng2.uniform(-1, 1, er.shape), 1.0)
    sg_t = sg * np.where(t_mask, 1 + 0.05 * rng2.uniform(-1, 1, sg.shape), 1.0)
    u_t, _ = physics.solve_currents(ref, vi.complex_permittivity(er_t, sg_t, F), e_inc, F, tol=1e-10)
    E_t = physics.total_field(ref, u_t, e_inc, F)[0].ravel()[targets]
    return G, er, sg, label, e_inc, ref, targets, E_t


def _loss_torch(E, targets, E_t):
    ex = E[0].reshape(-1)[targets]
    return torch.sum(torch.abs(ex - E_t) ** 2)


def test_adjoint_gradient_matches_oracle_and_finite_differences():
    G, er, sg, label, e_inc, ref, targets, E_t = _setup()
    op = vie.compress(G, tol=1e-6)
    tg = torch.from_numpy(targets).to(device())
    grads = {}
    # plain complex64 (FP32 everything), refined (FP32-computed operator
    # inside FP64 refinement), plain complex128
    for key, cdt, rdt, tol, refine in (("c64", torch.complex64, torch.float32, 1e-6, False),
                                       ("c64r", torch.complex128, torch.float64, 1e-10, True),
                                       ("c128", torch.complex128, torch.float64, 1e-12, False)):
        e_r = to_dev(er, rdt).requires_grad_(True)
        s_g = to_dev(sg, rdt).requires_grad_(True)
        E = total_field(op, e_r, s_g, to_dev(e_inc, cdt), F, tol=tol, refine=refine)
        L = _loss_torch(E, tg, to_dev(E_t, cdt))
        L.backward()
        grads[key] = (e_r.grad.cpu().numpy().astype(np.float64), s_g.grad.cpu().numpy().astype(np.float64),
                      float(L.item()))
    Lo, go_e, go_s, _ = ograd.adjoint_gradient(ref, vi.complex_permittivity(er, sg, F), e_inc, F, targets, E_t,
                                               tol=1e-12)
    for key, bound in (("c128", 1e-8), ("c64r", 1e-6), ("c64", 1e-3)):
        ge, gs, L = grads[key]
        err = max(rel(ge, go_e), rel(gs, go_s))
        say("   gradient vs oracle", key, err, "loss", L, Lo)
        assert err <= bound

    # central differences, complex128 solves to 1e-13, on 10 target voxels
    ee = to_dev(e_inc, torch.complex128)
    E_t_dev = to_dev(E_t, torch.complex128)

    def loss(er_, sg_):
        eps_c, b = vie.problem_setup(op, to_dev(er_, torch.float64), to_dev(sg_, torch.float64), ee, F)
        u, info, _ = vie.solve(op, b, eps_c, tol=1e-13, restart=60)
        E = vie.total_field(op, ee, u, vie.matvec(op, u, kind="N"), F)
        return _loss_torch(E, tg, E_t_dev).item()

    picks = np.random.default_rng(52).choice(targets, 10, replace=False)
    fd, ad64, ad32, ad32r = [], [], [], []
    for vox in picks:
        idx = np.unravel_index(vox, er.shape)
        for which, base in ((0, er), (1, sg)):
            step = 1e-4 * base[idx]
            p = base.copy()
            p[idx] += step
            m = base.copy()
            m[idx] -= step
            if which == 0:
                fd.append((loss(p, sg) - loss(m, sg)) / (2 * step))
            else:
                fd.append((loss(er, p) - loss(er, m)) / (2 * step))
            ad64.append(grads["c128"][which][idx])
            ad32.append(grads["c64"][which][idx])
            ad32r.append(grads["c64r"][which][idx])
    fd, ad64, ad32, ad32r = map(np.array, (fd, ad64, ad32, ad32r))
    e64, e32, e32r = rel(ad64, fd), rel(ad32, fd), rel(ad32r, fd)
    say("   FD check: complex128 %.2e, FP32 operator with FP64 refinement %.2e, plain complex64 %.2e"
        % (e64, e32r, e32))
    assert e64 <= 1e-5
    assert e32r <= 1e-4
    assert e32 <= 1e-3
