"""Adjoint gradient of a field objective (FP64).  Test infrastructure only.

Objective L = sum_{t in targets} |E_x(t) - E*_x(t)|^2 with E the total field
of ``physics.total_field``.  Differentiating A(chi) u = c_e chi e_inc with
E = u / (c_e chi) = e_inc + K u / c_e (K = N - I) gives, for a real
parameter theta_n of voxel n,

    dL/dtheta_n = Re[ (d chi_n / d theta) sum_q conj(z_q(n)) E_q(n) ]

where z solves A^H z = K^H G and G = dL/dRe(E) + i dL/dIm(E) is 2 (E_x - E*_x)
on the x-component of the target voxels and zero elsewhere.  With
chi = eps_r - 1 - i sigma / (omega eps0): d chi/d eps_r = 1 and
d chi / d sigma = -i / (omega eps0).  (The inverse problem is only mentioned
as an application in the paper's conclusion; this is the standard adjoint
derivation for the operator of eq. 4.)
"""
import numpy as np

from vie_inputs.constants import EPS0, omega

from .gmres import gmres
from .operator import apply_N, matvec
from .physics import solve_currents, total_field


def objective(E, targets, E_target):
    """``targets``: flat voxel indices; ``E_target``: target x-field there."""
    ex = E[0].ravel()[targets]
    return float(np.sum(np.abs(ex - E_target) ** 2))


def adjoint_gradient(op, eps_c, e_inc, freq_hz, targets, E_target, tol=1e-10):
    """Returns (L, dL/d eps_r, dL/d sigma, E); gradients have shape (n3, n2, n1)."""
    u, _ = solve_currents(op, eps_c, e_inc, freq_hz, tol=tol)
    E = total_field(op, u, e_inc, freq_hz)
    L = objective(E, targets, E_target)
    G = np.zeros_like(E)
    gx = G[0].reshape(-1)
    gx[targets] = 2.0 * (E[0].ravel()[targets] - E_target)
    rhs = apply_N(op, G, conj=True) - G            # K^H G
    shape = rhs.shape

    def AH(v):
        return matvec(op, eps_c, v.reshape(shape), "AH").ravel()

    z, _ = gmres(AH, rhs, tol=tol)
    z = z.reshape(shape)
    X = np.sum(np.conj(z) * E, axis=0)
    g_eps = np.real(X)
    g_sig = np.real(-1j / (omega(freq_hz) * EPS0) * X)
    return L, g_eps, g_sig, E
