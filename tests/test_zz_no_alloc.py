"""vie_matvec_noalloc (the matvec that allocates nothing, for callers that
cannot call hipMalloc) against vie_matvec / vie_matvec_adjoint with a caller
workspace: both run the same five passes, so the results must agree bit for
bit.  Two calls in a row on the shared scratch, the second with a smaller
input, then the first workload again after the scratch holds stale data."""
import ctypes

import numpy as np
import pytest
import torch

import vie_inputs as vi
from gpu_common import device, library_operator, problem, say

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1811_00484_amd import vie
    return vie, vie.load()


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _case(n, nrhs, dtype, kind, adjoint, seed):
    vie, lib = _lib()
    _, epsc, _ = problem(n)
    op = library_operator(n)
    u = np.stack([vi.random_field(n, seed + r) for r in range(nrhs)])
    x = torch.from_numpy(u).to(device=device(), dtype=dtype).contiguous()
    e = torch.from_numpy(epsc).to(device=device(), dtype=dtype).contiguous()
    dt = vie.VIE_C128 if dtype == torch.complex128 else vie.VIE_C64
    k = vie.VIE_OP_A if kind == "A" else vie.VIE_OP_N
    eps_arg = _p(e) if kind == "A" else None
    # reference: the existing entry point with its own workspace
    y_ref = torch.empty_like(x)
    nbytes = lib.vie_workspace_bytes(op.handle, dt, nrhs)
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=device())
    fn = lib.vie_matvec_adjoint if adjoint else lib.vie_matvec
    st = fn(op.handle, k, dt, vie.VIE_RECON_AUTO, eps_arg, _p(x), _p(y_ref), nrhs, _p(ws), nbytes, _stream())
    assert st == 0, lib.vie_last_error()
    # the entry point under test
    y = torch.full_like(x, float("nan"))
    say("noalloc: n=%s nrhs=%d %s kind=%s adjoint=%d" % (n, nrhs, dtype, kind, adjoint))
    st = lib.vie_matvec_noalloc(op.handle, k, adjoint, dt, vie.VIE_RECON_AUTO, eps_arg, _p(x), _p(y), nrhs,
                                _stream())
    assert st == 0, lib.vie_last_error()
    torch.cuda.synchronize()
    assert torch.isfinite(torch.view_as_real(y)).all()
    assert torch.equal(y, y_ref), "noalloc result differs from vie_matvec's"
    return nbytes


def test_noalloc_matches_workspace_matvec_on_successive_calls():
    vie, lib = _lib()
    cap = lib.vie_noalloc_scratch_bytes()
    assert cap == 256 << 20
    # register-FFT path (FFT length 128 on every axis), two right-hand sides
    b1 = _case((64, 64, 64), 2, torch.complex64, "A", 0, 11)
    # a smaller input right after, mixed-radix lengths, FP64, adjoint
    b2 = _case((12, 10, 9), 1, torch.complex128, "A", 1, 21)
    assert b2 < b1 <= cap
    # the bare operator on the first grid again, over the stale scratch
    _case((64, 64, 64), 1, torch.complex64, "N", 0, 31)
    _case((64, 64, 64), 1, torch.complex64, "N", 1, 41)


def test_noalloc_rejects_requests_beyond_the_scratch():
    vie, lib = _lib()
    n = (64, 64, 64)
    op = library_operator(n)
    cap = lib.vie_noalloc_scratch_bytes()
    nrhs = 1
    while lib.vie_workspace_bytes(op.handle, vie.VIE_C64, nrhs) <= cap:
        nrhs += 1
    x = torch.zeros((1, 3, 64, 64, 64), dtype=torch.complex64, device=device())
    # the size check comes before any launch, so the short buffers are never touched
    st = lib.vie_matvec_noalloc(op.handle, vie.VIE_OP_N, 0, vie.VIE_C64, vie.VIE_RECON_AUTO, None, _p(x), _p(x),
                                nrhs, _stream())
    assert st == vie.VIE_E_ARG
    assert b"scratch" in lib.vie_last_error()
