"""Differentiable forward model: total field E as a function of the per-voxel
relative permittivity and conductivity, with an adjoint backward pass.

Forward (eq. 1-4, electric block): eps_c = eps_r - i sigma/(omega eps0),
b = c_e chi e_inc, solve A(chi) u = b with GMRES, E = e_inc + (N u - u)/c_e.
Backward: given G = dL/dRe(E) + i dL/dIm(E) (PyTorch's complex gradient of a
real loss), solve A^H z = N^H G - G and return
dL/d eps_r = Re sum_q conj(z_q) E_q and dL/d sigma = Im(...) / (omega eps0).
Nothing of the forward Krylov process is stored: the backward pass runs its
own (adjoint) GMRES solve, so memory stays at a few vectors per voxel grid.
Every step runs in the HIP library (vie.*).
"""
import torch

from . import vie


class VIEFieldFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eps_r, sigma, op, e_inc, freq_hz, tol, restart, max_outer, adj_tol, refine):
        eps_c, b = vie.problem_setup(op, eps_r, sigma, e_inc, freq_hz)
        u, info, _ = vie.solve(op, b, eps_c, tol=tol, restart=restart, max_outer=max_outer, refine=refine)
        Nu = vie.matvec(op, u, kind="N")
        E = vie.total_field(op, e_inc, u, Nu, freq_hz)
        ctx.op = op
        ctx.freq = freq_hz
        ctx.solver = (adj_tol, restart, max_outer, refine)
        ctx.forward_info = info[0]
        ctx.save_for_backward(eps_c, E)
        return E

    @staticmethod
    def backward(ctx, gE):
        eps_c, E = ctx.saved_tensors
        op = ctx.op
        adj_tol, restart, max_outer, refine = ctx.solver
        g = gE.contiguous()
        NHg = vie.matvec(op, g, kind="N", adjoint=True)
        t = vie.adjoint_source(op, g, NHg)
        z, info, _ = vie.solve(op, t, eps_c, tol=adj_tol, restart=restart, max_outer=max_outer, adjoint=True,
                               refine=refine)
        g_eps, g_sig = vie.field_gradient(op, z, E, ctx.freq)
        return g_eps, g_sig, None, None, None, None, None, None, None, None


def total_field(op, eps_r, sigma, e_inc, freq_hz, tol=1e-6, restart=50, max_outer=200, adj_tol=None,
                refine=False):
    """E(eps_r, sigma): differentiable with respect to eps_r and sigma.

    complex64 e_inc: FP32 vectors and operator throughout.  complex128 e_inc
    with ``refine``: the solves run iterative refinement (FP64 residual and
    Arnoldi around the FP32-computed operator), so the FP32 operator sets the
    cost and FP64 the accuracy."""
    return VIEFieldFn.apply(eps_r, sigma, op, e_inc, freq_hz, tol, restart, max_outer,
                            tol if adj_tol is None else adj_tol, bool(refine))
