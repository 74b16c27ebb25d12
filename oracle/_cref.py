"""Loader for the oracle's plain-C hopping term (``csrc/hop_ref.c``).

Test infrastructure only.  ``build_oracle_c()`` compiles the shared object
with gcc; ``hop_c`` calls it through ctypes on canonical complex128 arrays.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "hop_ref.c")
_LIB = os.path.join(_HERE, "csrc", "liboracle_hop.so")
_lib = None


def build_oracle_c(force=True):
    """Compile the oracle's C code (gcc, OpenMP over sites)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fcx-limited-range", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle_c(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_hop.restype = None
        lib.oracle_hop.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int] * 7
        _lib = lib
    return _lib


def hop_c(U, psi, gammas, antiperiodic_t=True, dagger=False):
    """Hopping term on a field ``psi[..., t, z, y, x, s, a]`` (any leading batch)."""
    lib = _load()
    U = np.ascontiguousarray(U, dtype=np.complex128)
    lt, lz, ly, lx = U.shape[:4]
    batch = psi.shape[:-6]
    p = np.ascontiguousarray(psi, dtype=np.complex128).reshape((-1,) + psi.shape[-6:])
    out = np.empty_like(p)
    g = np.ascontiguousarray(gammas, dtype=np.complex128)
    lib.oracle_hop(U.ctypes.data, p.ctypes.data, out.ctypes.data, g.ctypes.data,
                   lx, ly, lz, lt, p.shape[0], int(bool(antiperiodic_t)), int(bool(dagger)))
    return out.reshape(batch + psi.shape[-6:])
