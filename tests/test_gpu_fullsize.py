"""Parity at the full workload sizes, in the launch configuration the
benchmark times (register-FFT kernels, complex64, one right-hand side):

* the 96 x 112 x 128 head at 2 mm with 8 ring dipoles: whole-vector matvec
  parity with the FP64 oracle and GMRES to 1e-6, the solution's residual
  checked with the oracle's operator;
* the 256^3 head at 1 mm (512^3 embedding): whole-vector matvec parity with
  the oracle's FFT convolution on the same Tucker operator (its own HOSVD
  at the same tolerance and the same ranks, so the difference is the FP32
  arithmetic alone), then with the oracle's dense-spectrum operator (the
  uncompressed tensor: FP32 rounding plus the 1e-6 truncation).

Plain complex64 GMRES (FP32 Arnoldi and FP32 residual) on the head
workload stops at an FP64 residual near 1.3e-6: it does not reach 1e-6, which
the FP64-refined solve does.  The test states that floor and asserts it."""
import warnings

import numpy as np
import pytest
import torch

import vie_inputs as vi
from gpu_common import F, K0, rel, say, to_dev
from oracle import operator as opm
from paper_1811_00484_amd import vie

pytestmark = pytest.mark.gpu


def test_head_96x112x128_matvec_and_solve():
    n = (96, 112, 128)
    h = 0.002
    G = vi.green_tensor(n, h, K0)
    er, sg, label = vi.head_phantom(n, h, seed=2)
    epsc = vi.complex_permittivity(er, sg, F)
    mask = label >= 0
    dips = vi.dipole_ring(8, 0.15)
    b = np.stack([vi.rhs_from_field(epsc, vi.dipole_field(n, h, F, p, mask), F) for p in dips])
    ref = opm.tucker_operator(G, 1e-6)
    op = vie.compress(G, tol=1e-6)
    assert op.ranks == ref.ranks
    e = to_dev(epsc, torch.complex64)
    u = vi.random_field(n, 77)
    y = vie.matvec(op, to_dev(u, torch.complex64), e).cpu().numpy().astype(np.complex128)
    err = rel(y, opm.matvec(ref, epsc, u, "A"))
    say("   96x112x128 matvec rel err", err)
    assert err <= 1e-5
    # GMRES to 1e-6: the complex64 operator inside FP64 refinement (FP32
    # Arnoldi alone stagnates near 1e-6 on these systems, see below)
    x, infos, st = vie.solve(op, to_dev(b, torch.complex128), to_dev(epsc, torch.complex128), tol=1e-6,
                             restart=50, refine=True, inner_tol=1e-5)
    assert st == 0
    xh = x.cpu().numpy()
    for s in range(8):
        r = rel(opm.matvec(ref, epsc, xh[s], "A"), b[s])
        say("   dipole %d: %d FP32 + %d FP64 matvecs, oracle residual %.3e"
            % (s, infos[s]["matvecs"], infos[s]["matvecs_fp64"], r))
        assert r <= 1.01e-6
    # plain complex64 GMRES (FP32 Arnoldi and residual) to 1e-6: it either
    # converges (status 0, every FP32 residual <= 1e-6) or reports that it did
    # not (status VIE_NOT_CONVERGED) at its FP32 floor; the floor, measured in
    # FP64 with the oracle's operator, is stated and bounded at 1e-5
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        x32, i32, st32 = vie.solve(op, to_dev(b[:2], torch.complex64), e, tol=1e-6, restart=50, max_outer=10)
    assert st32 in (vie.VIE_OK, vie.VIE_NOT_CONVERGED)
    x32 = x32.cpu().numpy().astype(np.complex128)
    floor = 0.0
    for s in range(2):
        r = rel(opm.matvec(ref, epsc, x32[s], "A"), b[s])
        floor = max(floor, r)
        assert i32[s]["converged"] == (i32[s]["rel_residual"] <= 1e-6)
        say("   plain complex64 dipole %d: FP32 residual %.3e, FP64 residual %.3e, converged %s"
            % (s, i32[s]["rel_residual"], r, i32[s]["converged"]))
    if st32 == vie.VIE_NOT_CONVERGED:
        say("   plain complex64 GMRES did not reach 1e-6; FP64 residual floor %.3e" % floor)
    else:
        assert all(i["converged"] for i in i32)
    assert floor <= 1e-5


@pytest.mark.timeout(900)
def test_head_256_matvec_vs_oracle():
    n = (256, 256, 256)
    h = 0.001
    G = vi.green_tensor(n, h, K0)
    er, sg, label = vi.head_phantom(n, h, seed=2)
    epsc = vi.complex_permittivity(er, sg, F)
    b = vi.rhs_from_field(epsc, vi.plane_wave(n, h, F), F)
    op = vie.compress(G, tol=1e-6)
    y = vie.matvec(op, to_dev(b, torch.complex64), to_dev(epsc, torch.complex64)).cpu().numpy()
    # the same Tucker operator: the oracle's HOSVD at the same tolerance
    ref = opm.tucker_operator(G, 1e-6)
    assert op.ranks == ref.ranks
    yt = opm.matvec(ref, epsc, b, "A")
    del ref
    err_t = rel(y.astype(np.complex128), yt)
    say("   256^3 matvec rel err vs the oracle's Tucker operator (FP32 only)", err_t)
    assert err_t <= 1e-5
    del yt
    dense = opm.dense_operator(G)
    yo = opm.matvec(dense, epsc, b, "A")
    del dense
    err = rel(y.astype(np.complex128), yo)
    say("   256^3 matvec rel err vs dense oracle", err)
    assert err <= 1e-5
