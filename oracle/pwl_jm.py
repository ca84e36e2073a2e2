"""The full JMVIE operator of eq. 4 in the piecewise-linear basis (FP64).
Test infrastructure only.

On x = [J; M], the electric and magnetic polarisation currents, each with
the twelve coefficients per voxel of eq. 7b ((4, 3, n3, n2, n1) in the
paper's basis), with the contrasts constant in each voxel so that they
multiply whole Galerkin rows:

    y_J = eps_c m_l J - chi_e (N J) + c_e h chi_e (K M)
    y_M = mu_c m_l M  - chi_h (N M) - c_m h chi_h (K J)

m_l = (1, 1/12, 1/12, 1/12) the self products of the basis, chi_e = eps_c - 1,
chi_h = mu_c - 1, c_e = i omega eps0, c_m = i omega mu0 (eq. 2), N the
Galerkin sum of ``oracle.pwl`` and K that of ``oracle.pwl_k`` (dimensionless:
the physical K is h times it, h the voxel edge).  In the mass-normalised
basis the operator is S A S with S = diag(1, sqrt 12, sqrt 12, sqrt 12) over
l on both currents (``to_normalised_jm``).
"""
import numpy as np

from vie_inputs.constants import EPS0, MU0, omega

from .pwl import MASS, SCALE, apply


def jm_matvec(khat_n, khat_k, eps_c, mu_c, x, h, freq_hz):
    """The operator above on x of shape (2, 4, 3, n3, n2, n1); khat_n and
    khat_k are the Fourier-domain kernels of ``pwl.dense_kernels`` /
    ``pwl.tucker_kernels`` and ``pwl_k.dense_kernels_k`` /
    ``pwl_k.tucker_kernels_k``."""
    ce = 1j * omega(freq_hz) * EPS0
    cm = 1j * omega(freq_hz) * MU0
    eps_c = np.asarray(eps_c)
    mu_c = np.asarray(mu_c)
    chi_e = (eps_c - 1.0)[None, None]
    chi_h = (mu_c - 1.0)[None, None]
    m = MASS[:, None, None, None, None]
    J, M = x[0], x[1]
    yJ = eps_c[None, None] * m * J - chi_e * apply(khat_n, J) + ce * h * chi_e * apply(khat_k, M)
    yM = mu_c[None, None] * m * M - chi_h * apply(khat_n, M) - cm * h * chi_h * apply(khat_k, J)
    return np.stack([yJ, yM])


def to_normalised_jm(op, x):
    """Apply ``op`` (a function of paper-basis [J; M]) in the mass-normalised
    basis: S op(S x) on both currents."""
    S = SCALE[None, :, None, None, None, None]
    return S * op(S * x)
