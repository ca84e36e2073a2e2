"""MI355X (gfx950) Tucker-compressed FFT-VIE matvec and GMRES solver.

The product path is ``libvie.so`` (HIP kernels + C ABI, ``include/vie.h``);
``vie`` is its thin ctypes binding and ``autograd`` the adjoint-gradient
``torch.autograd.Function`` built on it.
"""
from . import vie  # noqa: F401
from .vie import (MatvecGraph, Operator, VieError, autotune, compress, debug_nhat, densify,  # noqa: F401
                  field_gradient, from_tucker, matvec, set_nhat, solve)
