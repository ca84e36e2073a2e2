"""Seeded synthetic problem data for the FFT-VIE matvec and solver.

This package holds the *problem* only -- voxel grids, material maps of the
synthetic phantoms, incident fields, right-hand sides, the Galerkin Green's
tensor of the volume operator and seeded random vectors.  It holds none of
the compressed-matvec method (compression, circulant embedding, FFTs,
Hadamard products, Krylov solves): the oracle and the GPU library implement
those independently and both consume the arrays built here.

Array conventions (numpy, C order): a vector field is (3, n3, n2, n1)
complex with x fastest; a scalar map is (n3, n2, n1); the Green's tensor is
(6, n3, n2, n1) complex128, components xx, yy, zz, xy, xz, yz, entry
[c, k, j, i] = Nt_c(offset (i, j, k)); the K tensor is (3, n3, n2, n1),
components xy, xz, yz; the piecewise-linear tensors are (10, 6, n3, n2, n1),
one block of six components per basis pair of ``PWL_PAIRS``.
"""
from .constants import C0, EPS0, MU0, COMPONENTS, omega, wavenumber
from .grid import voxel_centres
from .materials import complex_permittivity, TISSUES_298MHZ
from .phantoms import sphere_phantom, head_phantom, head_semi_axes
from .fields import plane_wave, plane_wave_h, plane_wave_pwl, pwl_moments, dipole_field, dipole_ring, \
    dipole_cylinder, rhs_from_field
from .green import GreenEntryCallback, GreenPwlEntryCallback, PWL_PAIRS, green_entries, green_pwl_entries, green_k_tensor, green_pwl_entry, \
    green_pwl_k_entries, green_pwl_k_entry, green_pwl_k_tensor, green_pwl_tensor, green_tensor, pwl_pair_index
from .random import random_field, random_complex

__all__ = [
    "C0", "EPS0", "MU0", "COMPONENTS", "omega", "wavenumber", "voxel_centres",
    "complex_permittivity", "TISSUES_298MHZ", "sphere_phantom", "head_phantom",
    "head_semi_axes", "plane_wave", "plane_wave_h", "plane_wave_pwl", "pwl_moments", "dipole_field", "dipole_ring", "dipole_cylinder",
    "rhs_from_field", "green_tensor", "green_pwl_tensor", "green_pwl_entry", "PWL_PAIRS",
    "pwl_pair_index", "green_pwl_entries", "green_pwl_k_tensor", "green_pwl_k_entry", "green_pwl_k_entries", "GreenPwlEntryCallback", "green_k_tensor", "green_entries", "GreenEntryCallback", "random_field", "random_complex",
]
