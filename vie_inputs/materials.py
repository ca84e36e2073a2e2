"""Material parameters of the synthetic phantoms."""
import numpy as np

from .constants import EPS0, omega

# relative permittivity and conductivity (S/m) near 298 MHz (7 T proton
# Larmor frequency), the tissue set of the nested-ellipsoid head phantom,
# ordered from the outermost layer inwards
TISSUES_298MHZ = (
    ("skin", 50.0, 0.6),
    ("skull", 15.0, 0.1),
    ("csf", 72.0, 2.2),
    ("grey", 60.0, 0.7),
    ("white", 44.0, 0.4),
)


def complex_permittivity(eps_r, sigma, freq_hz):
    """eps_c = eps_r - i sigma / (omega eps0).

    Time convention exp(+i omega t), the one implied by the kernel
    exp(-i k0 R) / (4 pi R) of the Green's function; with it a lossy medium
    has a negative imaginary part.
    """
    return np.asarray(eps_r, dtype=np.float64) - 1j * np.asarray(sigma, dtype=np.float64) / (
        omega(freq_hz) * EPS0)
