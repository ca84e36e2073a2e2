"""Physical constants and the component ordering of the Green's tensor."""
import math

C0 = 299792458.0                 # speed of light in vacuum, m/s
EPS0 = 8.8541878128e-12          # vacuum permittivity, F/m
MU0 = 1.0 / (EPS0 * C0 * C0)     # vacuum permeability, H/m

# unique components of the symmetric 3x3 Green's tensor (PWC basis)
COMPONENTS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def omega(freq_hz):
    return 2.0 * math.pi * freq_hz


def wavenumber(freq_hz):
    """Free-space wavenumber k0 = omega / c0 (m^-1)."""
    return omega(freq_hz) / C0
