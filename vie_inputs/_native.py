"""Loader for the input generator's small C helper (Galerkin Green's tensor,
dyadic point samples).  Built with gcc into this directory; ``build()`` in
the repository root compiles it every time, and this loader compiles it on
first use if the shared object is missing."""
import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "green.c")
_LIB = os.path.join(_HERE, "libvie_inputs.so")
_lib = None


def build_native(force=True):
    """Compile csrc/green.c into libvie_inputs.so (gcc, OpenMP)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_native(force=True)
        L = ctypes.CDLL(_LIB)
        L.vie_green_fill.restype = ctypes.c_int
        L.vie_green_fill.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_long, ctypes.c_long]
        L.vie_green_k_fill.restype = ctypes.c_int
        L.vie_green_k_fill.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_long, ctypes.c_long]
        L.vie_green_entries.restype = ctypes.c_int
        L.vie_green_entries.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_long,
                                        ctypes.c_void_p, ctypes.c_void_p]
        L.vie_green_pwl_fill.restype = ctypes.c_int
        L.vie_green_pwl_fill.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                         ctypes.c_long, ctypes.c_long]
        L.vie_green_pwl_entry.restype = ctypes.c_int
        L.vie_green_pwl_entry.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p]
        L.vie_green_pwl_entries.restype = ctypes.c_int
        L.vie_green_pwl_entries.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p]
        L.vie_green_pwl_k_fill.restype = ctypes.c_int
        L.vie_green_pwl_k_fill.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_long, ctypes.c_long]
        L.vie_green_pwl_k_entry.restype = ctypes.c_int
        L.vie_green_pwl_k_entry.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_void_p]
        L.vie_green_pwl_k_entries.restype = ctypes.c_int
        L.vie_green_pwl_k_entries.argtypes = [ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p]
        L.vie_dyadic_points.restype = None
        L.vie_dyadic_points.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_double,
                                        ctypes.c_void_p]
        _lib = L
    return _lib
