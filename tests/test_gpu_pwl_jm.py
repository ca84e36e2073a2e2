"""GPU parity of the JMVIE operator of eq. 4 in the piecewise-linear basis
(vie_matvec_jm_pwl, vie_solve_jm_pwl) against the FP64 oracle
(oracle/pwl_jm.py) on the same HOSVD tensors, in the mass-normalised basis.
Errors are measured per block row: c_e h = omega eps0 h is ~1e-4 at 5 mm, so
the K M term of y_J is also checked alone (J = 0)."""
import functools

import numpy as np
import pytest
import torch

import vie_inputs as vi
from gpu_common import F, K0, rel, say, to_dev
from oracle import pwl, pwl_jm, pwl_k
from paper_1811_00484_amd import vie

pytestmark = pytest.mark.gpu
H = 0.005


@functools.lru_cache(maxsize=4)
def jm_problem(n, tol=1e-6):
    G = vi.green_pwl_tensor(n, H, K0)
    kt = vi.green_pwl_k_tensor(n, H, K0)
    khn, _ = pwl.tucker_kernels(G, tol)
    khk, _ = pwl_k.tucker_kernels_k(kt, tol)
    r = 0.4 * min(n) * H
    er, sg, inside = vi.sphere_phantom(n, H, r, 52.0, 0.55)
    eps_c = vi.complex_permittivity(er, sg, F)
    mu_c = np.where(inside, 1.6 - 0.3j, 1.0 + 0j)
    return G, kt, khn, khk, eps_c, mu_c


def _x(n, seed):
    rng = np.random.default_rng(seed)
    shape = (2, 4, 3, n[2], n[1], n[0])
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    x[1] *= 377.0     # M ~ eta0 J
    return x


def _oracle(khn, khk, eps_c, mu_c, x):
    return pwl_jm.to_normalised_jm(lambda w: pwl_jm.jm_matvec(khn, khk, eps_c, mu_c, w, H, F), x)


def _device(opn, opk, x, eps_c, mu_c, dtype):
    n = opn.n
    y = vie.matvec_jm_pwl(opn, opk, to_dev(x.reshape(2, 12, n[2], n[1], n[0]), dtype), to_dev(eps_c, dtype),
                          to_dev(mu_c, dtype), H, F)
    return y.cpu().numpy().astype(np.complex128).reshape(x.shape)


@pytest.mark.parametrize("n", [(12, 10, 9), (8, 8, 8), (5, 3, 2)])
def test_pwl_jm_matvec_c64_matches_oracle(n):
    say("pwl JM matvec c64", n)
    G, kt, khn, khk, eps_c, mu_c = jm_problem(n)
    opn, opk = vie.compress_pwl(G, tol=1e-6), vie.compress_pwl_k(kt, tol=1e-6)
    x = _x(n, 500)
    y, ref = _device(opn, opk, x, eps_c, mu_c, torch.complex64), _oracle(khn, khk, eps_c, mu_c, x)
    errs = [rel(y[b], ref[b]) for b in range(2)]
    x[0] = 0                       # y_J = c_e h chi_e K M alone
    y0, ref0 = _device(opn, opk, x, eps_c, mu_c, torch.complex64), _oracle(khn, khk, eps_c, mu_c, x)
    errs.append(rel(y0[0], ref0[0]))
    say("   rel errs (y_J, y_M, y_J from K M)", errs)
    assert max(errs) <= 1e-5


def test_pwl_jm_matvec_c128_matches_oracle():
    n = (12, 10, 9)
    say("pwl JM matvec c128", n)
    G, kt, khn, khk, eps_c, mu_c = jm_problem(n, tol=1e-8)
    opn, opk = vie.compress_pwl(G, tol=1e-8), vie.compress_pwl_k(kt, tol=1e-8)
    x = _x(n, 501)
    y, ref = _device(opn, opk, x, eps_c, mu_c, torch.complex128), _oracle(khn, khk, eps_c, mu_c, x)
    errs = [rel(y[b], ref[b]) for b in range(2)]
    say("   rel errs", errs)
    assert max(errs) <= 1e-11


def test_pwl_jm_pulse_currents_match_the_pulse_jm_operator():
    n = (16, 14, 12)
    say("pwl JM vs pulse JM", n)
    G, kt, _, _, eps_c, mu_c = jm_problem(n)
    opn, opk = vie.compress_pwl(G, tol=1e-6), vie.compress_pwl_k(kt, tol=1e-6)
    opn0, opk0 = vie.compress(G[0], tol=1e-6), vie.compress_k(kt[0], tol=1e-6)
    x = _x(n, 502)
    x[:, 1:] = 0
    y = _device(opn, opk, x, eps_c, mu_c, torch.complex64)
    y0 = vie.matvec_jm(opn0, opk0, to_dev(np.ascontiguousarray(x[:, 0]), torch.complex64),
                       to_dev(eps_c, torch.complex64), to_dev(mu_c, torch.complex64), H, F).cpu().numpy()
    errs = [rel(y[b, 0], y0[b].astype(np.complex128)) for b in range(2)]
    say("   rel errs", errs)
    assert max(errs) <= 1e-6


@pytest.mark.parametrize("dtype,refine,tol", [(torch.complex64, False, 1e-5), (torch.complex128, True, 1e-8)])
def test_pwl_jm_solve_residual_by_the_oracle(dtype, refine, tol):
    n = (10, 9, 8)
    say("pwl JM solve", n, dtype, refine)
    G, kt, khn, khk, eps_c, mu_c = jm_problem(n)
    opn, opk = vie.compress_pwl(G, tol=1e-6), vie.compress_pwl_k(kt, tol=1e-6)
    b = _x(n, 503)
    xd, info, st = vie.solve_jm_pwl(opn, opk, to_dev(b.reshape(2, 12, n[2], n[1], n[0]), dtype),
                                    to_dev(eps_c, dtype), to_dev(mu_c, dtype), H, F, tol=tol, restart=30,
                                    max_outer=100, refine=refine)
    say("   ", {k: v for k, v in info.items() if k != "history"})
    assert st == 0 and info["converged"]
    xs = xd.cpu().numpy().astype(np.complex128).reshape(b.shape)
    r = _oracle(khn, khk, eps_c, mu_c, xs) - b
    rel_res = np.linalg.norm(r) / np.linalg.norm(b)
    say("   oracle residual", rel_res)
    assert rel_res <= (3e-5 if dtype == torch.complex64 else 2 * tol)
