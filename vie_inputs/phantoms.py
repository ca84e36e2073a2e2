"""Synthetic phantoms: a homogeneous sphere and a nested-ellipsoid head.

Head recipe (the tissue set of the 7 T head-model workloads, synthetic
geometry): reference skin semi-axes A_ref = (76.8, 89.6, 102.4) mm, i.e.
0.8 x the half extents of a 192 x 224 x 256 mm box; scale
s = min_i(n_i h / L_ref_i) with L_ref = (192, 224, 256) mm; layer fractions
f = (skin 1.00, skull 0.92, CSF 0.86, grey 0.82, white 0.66); jitter
J = rng.uniform(-0.1, 0.1, (5, 3)) with rng = numpy.random.default_rng(seed);
semi-axes a_{l,i} = s f_l A_ref_i (1 + J_{l,i}).  A voxel takes the tissue of
the innermost layer whose ellipsoid contains its centre, otherwise air.
"""
import numpy as np

from .grid import voxel_centres
from .materials import TISSUES_298MHZ

A_REF_MM = np.array([76.8, 89.6, 102.4])
L_REF_MM = np.array([192.0, 224.0, 256.0])
LAYER_FRACTIONS = np.array([1.00, 0.92, 0.86, 0.82, 0.66])


def sphere_phantom(n, h, radius, eps_r, sigma, centre=(0.0, 0.0, 0.0)):
    """Homogeneous sphere in vacuum: a voxel belongs to the sphere iff its
    centre lies within ``radius`` of ``centre``.  Returns (eps_r, sigma, mask)
    maps of shape (n3, n2, n1)."""
    x, y, z = voxel_centres(n, h)
    d2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    mask = d2 <= radius * radius * (1.0 + 1e-12)
    er = np.where(mask, float(eps_r), 1.0)
    sg = np.where(mask, float(sigma), 0.0)
    return er, sg, mask


def head_semi_axes(n, h, seed):
    """Semi-axes (metres), shape (5, 3), of the five nested ellipsoids."""
    n = np.asarray(n, dtype=np.float64)
    h_mm = float(h) * 1e3
    s = float(np.min(n * h_mm / L_REF_MM))
    rng = np.random.default_rng(seed)
    J = rng.uniform(-0.1, 0.1, (5, 3))
    a_mm = s * LAYER_FRACTIONS[:, None] * A_REF_MM[None, :] * (1.0 + J)
    return a_mm * 1e-3


def head_phantom(n, h, seed):
    """Nested-ellipsoid head in air.  Returns (eps_r, sigma, label) maps of
    shape (n3, n2, n1); label is -1 for air, else the index into
    ``TISSUES_298MHZ``."""
    a = head_semi_axes(n, h, seed)
    x, y, z = voxel_centres(n, h)
    label = np.full(x.shape, -1, dtype=np.int8)
    for l in range(5):
        inside = (x / a[l, 0]) ** 2 + (y / a[l, 1]) ** 2 + (z / a[l, 2]) ** 2 <= 1.0
        label[inside] = l
    er = np.ones(x.shape)
    sg = np.zeros(x.shape)
    for l, (_, e, s) in enumerate(TISSUES_298MHZ):
        er[label == l] = e
        sg[label == l] = s
    return er, sg, label
