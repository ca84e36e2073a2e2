"""Seeded random complex arrays (numpy.random.default_rng)."""
import numpy as np


def random_complex(shape, seed):
    """Complex normal entries, real then imaginary parts drawn in that order."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return re + 1j * im


def random_field(n, seed, nrhs=None):
    """Random current-like field of shape (3, n3, n2, n1), or
    (nrhs, 3, n3, n2, n1) when ``nrhs`` is given."""
    n1, n2, n3 = (int(v) for v in n)
    shape = (3, n3, n2, n1) if nrhs is None else (int(nrhs), 3, n3, n2, n1)
    return random_complex(shape, seed)
