"""Incident fields and right-hand sides.

Incident fields are sampled at voxel centres.  The right-hand side of the
electric current equation is b = c_e chi e_inc with c_e = i omega eps0 and
chi = eps_c - 1 (eq. 1-2 of the paper, electric block).
"""
import math

import numpy as np

from . import _native
from .constants import C0, EPS0, MU0, omega, wavenumber
from .grid import voxel_centres


def plane_wave(n, h, freq_hz, pol=0, amplitude=1.0):
    """Unit plane wave pol-hat * exp(-i k0 z) travelling along +z
    (exp(+i omega t) convention).  Shape (3, n3, n2, n1) complex128."""
    _, _, z = voxel_centres(n, h)
    e = np.zeros((3,) + z.shape, dtype=np.complex128)
    e[pol] = amplitude * np.exp(-1j * wavenumber(freq_hz) * z)
    return e


def plane_wave_h(n, h, freq_hz, pol=0, amplitude=1.0):
    """Magnetic field of ``plane_wave``: H = z-hat x E / eta0 with
    eta0 = mu0 c0 (exp(+i omega t), travelling along +z).  Shape (3, n3, n2, n1)."""
    e = plane_wave(n, h, freq_hz, pol, amplitude)
    eta0 = MU0 * C0
    hf = np.zeros_like(e)
    hf[0] = -e[1] / eta0
    hf[1] = e[0] / eta0
    return hf


def _dyadic(points, k0):
    """(k0^2 I + grad grad) exp(-i k0 R)/(4 pi R) at the given points
    (N x 3, metres), six components per point."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    out = np.empty((pts.shape[0], 6, 2), dtype=np.float64)
    _native.lib().vie_dyadic_points(pts.shape[0], pts.ctypes.data, float(k0), out.ctypes.data)
    return out[..., 0] + 1j * out[..., 1]


def dipole_field(n, h, freq_hz, r_d, mask, moment=1.0):
    """Field of a z-directed Hertzian dipole of moment I*l = ``moment`` A m at
    ``r_d`` (metres): E = (I l / (i omega eps0)) [(k0^2 I + grad grad) g] z-hat,
    evaluated at the centres of voxels where ``mask`` is true and set to zero
    elsewhere (the dipole may sit inside the grid's bounding box)."""
    x, y, z = voxel_centres(n, h)
    sel = np.nonzero(mask.ravel())[0]
    pts = np.stack([x.ravel()[sel] - r_d[0], y.ravel()[sel] - r_d[1], z.ravel()[sel] - r_d[2]], axis=1)
    G = _dyadic(pts, wavenumber(freq_hz))
    pref = moment / (1j * omega(freq_hz) * EPS0)
    e = np.zeros((3, x.size), dtype=np.complex128)
    # components (x,z), (y,z), (z,z) are indices 4, 5, 2 of xx,yy,zz,xy,xz,yz
    e[0, sel] = pref * G[:, 4]
    e[1, sel] = pref * G[:, 5]
    e[2, sel] = pref * G[:, 2]
    return e.reshape((3,) + x.shape)


def dipole_ring(count=8, radius=0.15, z=0.0):
    """Dipole positions (count x 3) on a ring in the z = ``z`` plane,
    angles 2 pi k / count."""
    phi = 2.0 * math.pi * np.arange(count) / count
    return np.stack([radius * np.cos(phi), radius * np.sin(phi), np.full(count, z)], axis=1)


def dipole_cylinder(count, radius, half_height, seed):
    """Seeded dipole positions on a cylinder: phi ~ U(0, 2 pi) then
    z ~ U(-half_height, half_height), both from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0 * math.pi, count)
    zz = rng.uniform(-half_height, half_height, count)
    return np.stack([radius * np.cos(phi), radius * np.sin(phi), zz], axis=1)


def rhs_from_field(eps_c, e_inc, freq_hz):
    """b = c_e chi e_inc with c_e = i omega eps0, chi = eps_c - 1."""
    ce = 1j * omega(freq_hz) * EPS0
    chi = np.asarray(eps_c) - 1.0
    return ce * chi[None] * e_inc


def pwl_moments(n, h, field, order=6):
    """Voxel moments of a vector field against the piecewise-linear basis
    (eq. 7b): out[l, p, k, j, i] = (1/h^3) int_voxel C^l(r) E_p(r) dr with
    C^0 = 1 and C^l = (r_a - r_a,m)/h (a = l - 1) inside the voxel, by a
    tensor Gauss-Legendre rule of ``order`` points per axis.  ``field(x, y,
    z)`` returns the (3, ...) complex field at points of the broadcast
    shape.  Shape (4, 3, n3, n2, n1) complex128."""
    x, y, z = voxel_centres(n, h)
    t, w = np.polynomial.legendre.leggauss(order)
    t, w = 0.5 * t, 0.5 * w
    out = np.zeros((4, 3) + z.shape, dtype=np.complex128)
    for a, ta in enumerate(t):
        for b, tb in enumerate(t):
            for c, tc in enumerate(t):
                e = np.asarray(field(x + h * ta, y + h * tb, z + h * tc))
                wt = w[a] * w[b] * w[c]
                out[0] += wt * e
                out[1] += (wt * ta) * e
                out[2] += (wt * tb) * e
                out[3] += (wt * tc) * e
    return out


def plane_wave_pwl(n, h, freq_hz, pol=0, amplitude=1.0):
    """``plane_wave`` as piecewise-linear voxel moments (``pwl_moments``),
    shape (4, 3, n3, n2, n1)."""
    k0 = wavenumber(freq_hz)

    def field(x, y, z):
        e = np.zeros((3,) + np.broadcast(x, y, z).shape, dtype=np.complex128)
        e[pol] = amplitude * np.exp(-1j * k0 * z)
        return e
    return pwl_moments(n, h, field)
