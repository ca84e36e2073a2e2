"""BF16 Tucker reconstruction on MFMA (z-factor contraction with BF16 inputs,
FP32 accumulation): its error against the FP64 oracle is stated and bounded
(BF16 keeps 8 significant bits, so about 1e-3 is expected, not 1e-5), and
FP64 iterative refinement around the BF16 operator must still reach the
oracle's solution."""
import numpy as np
import pytest
import torch

import vie_inputs as vi
from gpu_common import library_operator, problem, rel, say, to_dev
from oracle import operator as opm
from paper_1811_00484_amd import vie

pytestmark = pytest.mark.gpu

# z FFT lengths 128, 256, 512 (the MFMA tables exist for these), ragged x/y
BF16_SIZES = [(64, 20, 64), (36, 40, 128), (20, 18, 256)]
BF16_BOUND = 5e-3


@pytest.mark.parametrize("n", BF16_SIZES)
@pytest.mark.parametrize("mode", ["A", "AH", "N"])
def test_bf16_matvec_error_vs_oracle(n, mode):
    say("bf16 matvec", n, mode)
    G, epsc, ref = problem(n, h=0.003, phantom="head")
    op = library_operator(n, h=0.003, phantom="head")
    u = vi.random_field(n, 15)
    x = to_dev(u, torch.complex64)
    e = to_dev(epsc, torch.complex64)
    kind = "N" if mode == "N" else "A"
    y16 = vie.matvec(op, x, e, kind=kind, adjoint=(mode == "AH"), recon="bf16").cpu().numpy()
    y32 = vie.matvec(op, x, e, kind=kind, adjoint=(mode == "AH"), recon="fp32").cpu().numpy()
    yo = opm.matvec(ref, epsc, u, mode)
    e16 = rel(y16.astype(np.complex128), yo)
    e32 = rel(y32.astype(np.complex128), yo)
    say("   rel err vs FP64 oracle: bf16 %.3e, fp32 %.3e" % (e16, e32))
    assert e32 <= 1e-5
    assert e16 <= BF16_BOUND
    # the N-part carries the BF16 error: it must be visibly above FP32 rounding
    # (the MFMA path ran) yet far below O(1) (the tables are right)
    assert e16 > 10 * e32


def test_bf16_refined_solve_reaches_oracle_residual():
    n = (20, 18, 256)
    G, epsc, ref = problem(n, h=0.003, phantom="head")
    op = library_operator(n, h=0.003, phantom="head")
    e_inc = vi.plane_wave(n, 0.003, 298e6)
    b = vi.rhs_from_field(epsc, e_inc, 298e6)
    bb = to_dev(b, torch.complex128)
    ee = to_dev(epsc, torch.complex128)
    res = {}
    for rc in ("fp32", "bf16"):
        x, info, st = vie.solve(op, bb, ee, tol=1e-9, restart=30, max_outer=30, refine=True, inner_tol=1e-3,
                                inner_recon=rc)
        assert st == 0 and info[0]["converged"]
        xh = x.cpu().numpy()
        r = rel(opm.matvec(ref, epsc, xh, "A"), b)
        say("   refined solve inner %s: %s, oracle residual %.3e" % (rc, info[0], r))
        assert r <= 1.05e-9
        res[rc] = xh
    assert rel(res["bf16"], res["fp32"]) <= 1e-7


def test_bf16_unsupported_lengths_raise():
    n = (12, 10, 9)   # 2 n3 = 18: no MFMA table kernel for this length
    G, epsc, ref = problem(n)
    op = library_operator(n)
    x = to_dev(vi.random_field(n, 3), torch.complex64)
    with pytest.raises(RuntimeError):
        vie.matvec(op, x, to_dev(epsc, torch.complex64), recon="bf16")
    with pytest.raises(RuntimeError):
        vie.matvec(op, x.to(torch.complex128), to_dev(epsc, torch.complex128), recon="bf16")
