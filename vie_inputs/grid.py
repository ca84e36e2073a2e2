"""Uniform voxel grid centred on the origin."""
import numpy as np


def voxel_centres(n, h):
    """Voxel-centre coordinates (x, y, z), each of shape (n3, n2, n1).

    Centre of voxel m along axis i is (m + 1/2 - n_i/2) * h_i, so the grid is
    centred on the origin.  ``h`` may be a scalar or a 3-sequence (metres).
    """
    n1, n2, n3 = (int(v) for v in n)
    hh = np.broadcast_to(np.asarray(h, dtype=np.float64), (3,))
    cx = (np.arange(n1) + 0.5 - n1 / 2.0) * hh[0]
    cy = (np.arange(n2) + 0.5 - n2 / 2.0) * hh[1]
    cz = (np.arange(n3) + 0.5 - n3 / 2.0) * hh[2]
    z, y, x = np.meshgrid(cz, cy, cx, indexing="ij")
    return x, y, z
