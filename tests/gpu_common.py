"""Shared helpers of the GPU parity tests (no test functions here)."""
import functools
import sys

import numpy as np
import torch

import vie_inputs as vi
from oracle import operator as opm

F = 298e6
K0 = vi.wavenumber(F)


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def device():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch.device("cuda:0")


@functools.lru_cache(maxsize=16)
def problem(n, h=0.005, tol=1e-6, phantom="sphere", seed=2):
    """Green's tensor, contrast and the oracle's Tucker operator (FP64)."""
    G = vi.green_tensor(n, h, K0)
    if phantom == "sphere":
        r = 0.4 * min(n) * h
        er, sg, _ = vi.sphere_phantom(n, h, r, 52.0, 0.55)
    else:
        er, sg, _ = vi.head_phantom(n, h, seed)
    epsc = vi.complex_permittivity(er, sg, F)
    ref = opm.tucker_operator(G, tol)
    return G, epsc, ref


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=device(), dtype=dtype)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@functools.lru_cache(maxsize=8)
def library_operator(n, h=0.005, tol=1e-6, phantom="sphere", seed=2):
    from paper_1811_00484_amd import vie
    G, _, _ = problem(n, h, tol, phantom, seed)
    return vie.compress(G, tol=tol)
