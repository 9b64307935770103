"""Build and load the oracle's C library (``oracle/liborc.so``).

Test infrastructure: compiled with plain gcc, no GPU code."""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "bem_oracle.c")
LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle library with gcc -O2 -fopenmp (no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        d = ctypes.c_double
        L.orc_radial.argtypes = [d, d, d, ctypes.c_int, P]
        L.orc_kernel.argtypes = [d, d, P, P, P, P, ctypes.c_int, P, P]
        L.orc_radon7.argtypes = [P, P]
        L.orc_gauss_legendre.argtypes = [ctypes.c_int, P, P]
        L.orc_geometry.argtypes = [P, i64, P, P]
        L.orc_blocks.argtypes = [P, i64, P, d, d, P, P, i64, P, P, P]
        L.orc_assemble_rows.argtypes = [P, i64, P, P, P, d, d, P, P, i64, P, P, P]
        L.orc_rowsum_H_static.argtypes = [P, i64, P, P, P, P]
        L.orc_gauss6.argtypes = [P, P]
        L.orc_lagrange6.argtypes = [P]
        L.orc_q6_map.argtypes = [P, i64, P, P]
        L.orc_nys_nodes.argtypes = [P, i64, P, P]
        L.orc_nys_element.argtypes = [P, P, ctypes.c_int, d, d, P, P, P, P]
        L.orc_nys_assemble_rows.argtypes = [P, i64, P, P, P, d, d, P, P, i64, P, P, P]
        L.orc_nys_rowsum_H_static.argtypes = [P, i64, P, P, P, P]
        _lib = L
    return _lib
