"""Register-FFT kernels (FFT lengths 128, 256, 512) against the FP64 oracle
and against the mixed-radix LDS kernels, including grids that mix the two
(one axis on each path) and partial tiles."""
import numpy as np
import pytest
import torch

import vie_inputs as vi
from gpu_common import library_operator, problem, rel, say, to_dev
from oracle import operator as opm
from paper_1811_00484_amd import vie

pytestmark = pytest.mark.gpu

# register-FFT lengths on each axis: 128, 256, 512 everywhere, 192 (8 8 3) and
# 224 (7 4 4 2) on x and y; partial tiles, and axes that fall back to the
# mixed-radix kernels (e.g. 2 n2 = 40, 2 n3 = 32)
FAST_SIZES = [(64, 64, 64), (64, 20, 64), (64, 48, 128), (128, 40, 64), (36, 64, 256), (96, 112, 16),
              (40, 112, 64), (96, 20, 64)]


@pytest.mark.parametrize("n", FAST_SIZES)
@pytest.mark.parametrize("mode", ["A", "AH", "N"])
def test_fast_c64_matches_oracle(n, mode):
    say("fast c64", n, mode)
    G, epsc, ref = problem(n, h=0.003)
    op = library_operator(n, h=0.003)
    assert op.ranks == ref.ranks
    u = vi.random_field(n, 5)
    y = vie.matvec(op, to_dev(u, torch.complex64), to_dev(epsc, torch.complex64),
                   kind="N" if mode == "N" else "A", adjoint=(mode == "AH")).cpu().numpy()
    err = rel(y.astype(np.complex128), opm.matvec(ref, epsc, u, mode))
    say("   rel err", err)
    assert err <= 1e-5


@pytest.mark.parametrize("n", [(64, 64, 64), (64, 48, 128)])
def test_fast_c128_matches_oracle(n):
    # tol 1e-8: the library's HOSVD then always runs its Jacobi refinement,
    # so both sides hold the same Tucker operator to ~1e-14 (at tol >= 1e-7
    # on large unfoldings the library keeps the Gram-matrix eigenvectors,
    # whose subspaces differ from the SVD's by ~1e-10: irrelevant for FP32,
    # but visible at FP64)
    G, epsc, ref = problem(n, h=0.003, tol=1e-8)
    op = library_operator(n, h=0.003, tol=1e-8)
    u = vi.random_field(n, 6)
    y = vie.matvec(op, to_dev(u, torch.complex128), to_dev(epsc, torch.complex128)).cpu().numpy()
    err = rel(y, opm.matvec(ref, epsc, u, "A"))
    say("   c128 rel err", err)
    assert err <= 1e-11


def test_fast_equals_generic_kernels():
    n = (64, 48, 128)
    G, epsc, ref = problem(n, h=0.003)
    op = library_operator(n, h=0.003)
    x = to_dev(vi.random_field(n, 8, nrhs=2), torch.complex128)
    e = to_dev(epsc, torch.complex128)
    y_fast = vie.matvec(op, x, e).cpu().numpy()
    vie.set_kernel_path(1)
    try:
        y_gen = vie.matvec(op, x, e).cpu().numpy()
    finally:
        vie.set_kernel_path(0)
    assert rel(y_fast, y_gen) <= 1e-13


def test_fast_dense_spectrum_path():
    n = (64, 64, 64)
    G, epsc, ref = problem(n, h=0.003)
    op = library_operator(n, h=0.003)
    x = to_dev(vi.random_field(n, 9), torch.complex64)
    e = to_dev(epsc, torch.complex64)
    y_t = vie.matvec(op, x, e).cpu().numpy()
    vie.densify(op)
    vie.set_nhat(op, "dense")
    try:
        y_d = vie.matvec(op, x, e).cpu().numpy()
    finally:
        vie.set_nhat(op, "tucker")
    assert rel(y_d, y_t) <= 1e-6
