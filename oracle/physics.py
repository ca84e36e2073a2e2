"""Fields, absorbed power and the Mie series (FP64).  Test infrastructure only.

Time convention exp(+i omega t) (the kernel exp(-i k0 R)/(4 pi R)), so a
lossy medium has eps_c = eps_r - i sigma/(omega eps0).
"""
import numpy as np
import scipy.special as ssp

from vie_inputs.constants import EPS0, MU0, omega, wavenumber

from .gmres import gmres
from .operator import apply_N, matvec


def c_e(freq_hz):
    """c_e = i omega eps0 (eq. 2)."""
    return 1j * omega(freq_hz) * EPS0


def total_field(op, u, e_inc, freq_hz):
    """E = e_inc + (N u - u) / c_e: the scattered field of the polarisation
    current u = c_e chi E (eq. 3) through the operator N of eq. 5."""
    return e_inc + (apply_N(op, u) - u) / c_e(freq_hz)


def solve_currents(op, eps_c, e_inc, freq_hz, tol=1e-8, restart=50, max_outer=200, x0=None):
    """Solve (M_eps - M_chi N) u = c_e chi e_inc (eq. 1, electric block)."""
    chi = np.asarray(eps_c) - 1.0
    b = c_e(freq_hz) * chi[None] * e_inc
    shape = b.shape

    def A(v):
        return matvec(op, eps_c, v.reshape(shape), "A").ravel()

    x, info = gmres(A, b, x0=x0, tol=tol, restart=restart, max_outer=max_outer)
    return x.reshape(shape), info


def absorbed_power(E, sigma, h):
    """p_abs = 1/2 sigma |E|^2 (eq. 18) summed over voxels of volume h^3."""
    return 0.5 * float(np.sum(np.asarray(sigma)[None] * np.abs(E) ** 2)) * float(h) ** 3


def mie_absorbed_power(radius, eps_c, freq_hz, e0=1.0, nmax=None):
    """Power absorbed by a homogeneous sphere in a plane wave of amplitude
    ``e0`` (Bohren & Huffman Mie coefficients).  Their exp(-i omega t)
    convention needs m = sqrt(conj(eps_c))."""
    k0 = wavenumber(freq_hz)
    x = k0 * radius
    m = np.sqrt(np.conj(complex(eps_c)))
    if nmax is None:
        nmax = int(np.ceil(x + 4.0 * x ** (1.0 / 3.0) + 12))
    n = np.arange(1, nmax + 1)
    mx = m * x

    def psi(z):
        return z * ssp.spherical_jn(n, z)

    def dpsi(z):
        return ssp.spherical_jn(n, z) + z * ssp.spherical_jn(n, z, derivative=True)

    def xi(z):
        return z * (ssp.spherical_jn(n, z) + 1j * ssp.spherical_yn(n, z))

    def dxi(z):
        h = ssp.spherical_jn(n, z) + 1j * ssp.spherical_yn(n, z)
        dh = ssp.spherical_jn(n, z, derivative=True) + 1j * ssp.spherical_yn(n, z, derivative=True)
        return h + z * dh

    a_n = (m * psi(mx) * dpsi(x) - psi(x) * dpsi(mx)) / (m * psi(mx) * dxi(x) - xi(x) * dpsi(mx))
    b_n = (psi(mx) * dpsi(x) - m * psi(x) * dpsi(mx)) / (psi(mx) * dxi(x) - m * xi(x) * dpsi(mx))
    q_ext = 2.0 / x ** 2 * np.sum((2 * n + 1) * np.real(a_n + b_n))
    q_sca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (np.abs(a_n) ** 2 + np.abs(b_n) ** 2))
    eta0 = np.sqrt(MU0 / EPS0)
    intensity = abs(e0) ** 2 / (2.0 * eta0)
    return float((q_ext - q_sca) * np.pi * radius ** 2 * intensity)
