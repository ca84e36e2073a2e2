"""GPU parity of the piecewise-linear magnetic operator (vie_compress_pwl_k,
vie_matvec_pwl with kind N) against the FP64 oracle (oracle/pwl_k.py) on the
same HOSVD tensors, in the mass-normalised basis (S K S).  Tolerances as for
the electric block: relative L2 error 1e-5 for complex64, 1e-11 for
complex128."""
import functools

import numpy as np
import pytest
import torch

import vie_inputs as vi
from gpu_common import K0, device, rel, say, to_dev
from oracle import pwl, pwl_k
from paper_1811_00484_amd import vie

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=8)
def k_problem(n, h=0.005, tol=1e-6):
    kt = vi.green_pwl_k_tensor(n, h, K0)
    kh, ranks = pwl_k.tucker_kernels_k(kt, tol)
    return kt, kh, ranks


def _field(n, seed):
    rng = np.random.default_rng(seed)
    shape = (4, 3, n[2], n[1], n[0])
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _device(op, u, dtype):
    n = op.n
    y = vie.matvec_pwl(op, to_dev(u.reshape(12, n[2], n[1], n[0]), dtype), kind="N")
    return y.cpu().numpy().astype(np.complex128).reshape(u.shape)


SIZES = [(12, 10, 9), (8, 8, 8), (5, 3, 2), (1, 1, 1), (20, 15, 18), (16, 14, 7), (6, 5, 126), (7, 4, 120)]


@pytest.mark.parametrize("n", SIZES)
def test_pwl_k_matvec_c64_matches_oracle(n):
    say("pwl K matvec c64", n)
    kt, kh, ranks = k_problem(n)
    op = vie.compress_pwl_k(kt, tol=1e-6)
    assert op.family == "K"
    assert np.array_equal(op.ranks[:, 3:], ranks)
    u = _field(n, 400)
    err = rel(_device(op, u, torch.complex64), pwl_k.to_normalised_k(kh, u))
    say("   rel err", err)
    assert err <= 1e-5


@pytest.mark.parametrize("n", [(12, 10, 9), (20, 15, 18), (1, 1, 1)])
def test_pwl_k_matvec_c128_matches_oracle(n):
    say("pwl K matvec c128", n)
    kt, kh, ranks = k_problem(n, tol=1e-8)
    op = vie.compress_pwl_k(kt, tol=1e-8)
    assert np.array_equal(op.ranks[:, 3:], ranks)
    u = _field(n, 401)
    err = rel(_device(op, u, torch.complex128), pwl_k.to_normalised_k(kh, u))
    say("   rel err", err)
    assert err <= 1e-11


def test_pwl_k_pulse_rows_match_the_pulse_k():
    # pulse coefficients only: the pulse rows are the pulse-basis K of the
    # (pulse, pulse) tensors, run by the pulse path's K kernels
    n = (16, 16, 16)
    say("pwl K vs pulse K", n)
    kt, _, _ = k_problem(n)
    op = vie.compress_pwl_k(kt, tol=1e-6)
    opk = vie.compress_k(kt[0], tol=1e-6)
    u = np.zeros((4, 3, n[2], n[1], n[0]), complex)
    u[0] = vi.random_field(n, 402)
    y = _device(op, u, torch.complex64)
    y0 = vie.matvec(opk, to_dev(u[0], torch.complex64), kind="N").cpu().numpy()
    err = rel(y[0], y0.astype(np.complex128))
    say("   rel err", err)
    assert err <= 1e-6
    assert np.abs(y[1:]).max() > 1e-3 * np.abs(y[0]).max()


def test_pwl_k_rejects_contrast_and_adjoint():
    n = (5, 3, 2)
    kt, _, _ = k_problem(n)
    op = vie.compress_pwl_k(kt, tol=1e-6)
    x = torch.zeros((12, n[2], n[1], n[0]), dtype=torch.complex64, device=device())
    e = torch.ones((n[2], n[1], n[0]), dtype=torch.complex64, device=device())
    with pytest.raises(vie.VieError):
        vie.matvec_pwl(op, x, e, kind="A")
    with pytest.raises(vie.VieError):
        vie.matvec_pwl(op, x, kind="N", adjoint=True)
    with pytest.raises(vie.VieError):
        vie.solve_pwl(op, x, e)


def test_pwl_k_multi_rhs_equals_single_calls():
    n = (12, 10, 9)
    say("pwl K multi rhs", n)
    kt, kh, _ = k_problem(n)
    op = vie.compress_pwl_k(kt, tol=1e-6)
    rng = np.random.default_rng(403)
    u = rng.standard_normal((3, 12, n[2], n[1], n[0])) + 1j * rng.standard_normal((3, 12, n[2], n[1], n[0]))
    x = to_dev(u, torch.complex64)
    yb = vie.matvec_pwl(op, x, kind="N").cpu().numpy()
    for r in range(3):
        ys = vie.matvec_pwl(op, x[r].contiguous(), kind="N").cpu().numpy()
        assert np.array_equal(yb[r], ys), r
    ref = pwl_k.to_normalised_k(kh, u[2].reshape(4, 3, n[2], n[1], n[0]))
    assert rel(yb[2].astype(np.complex128).reshape(ref.shape), ref) <= 1e-5


def test_pwl_k_fullsize_sampled_outputs():
    # the refinement series' 2.5 mm grid: sampled outputs of the device
    # product against the sums written out over the oracle's HOSVD tensors
    N = 120
    n = (N, N, N)
    say("pwl K full size", n)
    kt = vi.green_pwl_k_tensor(n, 0.3 / N, K0)
    op = vie.compress_pwl_k(kt, tol=1e-6)
    kapprox, ranks = pwl_k.tucker_tensors_k(kt, 1e-6)
    assert np.array_equal(op.ranks[:, 3:], ranks)
    del kt
    rng = np.random.default_rng(410)
    u = rng.standard_normal((4, 3, N, N, N)) + 1j * rng.standard_normal((4, 3, N, N, N))
    y = _device(op, u, torch.complex64)
    S = pwl.SCALE
    samples = [(int(rng.integers(4)), int(rng.integers(3)), int(rng.integers(N)), int(rng.integers(N)),
                int(rng.integers(N))) for _ in range(12)] + [(3, 2, N - 1, N - 1, N - 1), (0, 0, 0, 0, 0)]
    ref = pwl_k.sampled_outputs_k(kapprox, S[:, None, None, None, None] * u, samples)
    ref = np.array([S[s[0]] * r for s, r in zip(samples, ref)])
    got = np.array([y[s] for s in samples])
    err = np.abs(got - ref).max() / np.abs(ref).max()
    say("   max sampled error / max |y|", err)
    assert err <= 1e-5
