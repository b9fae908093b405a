"""Loader for the oracle's C part (test infrastructure only).

``build()`` compiles ``bandchol.c`` with gcc into ``liboracle_band.so`` next
to it; ``lib()`` loads it, building it first when no library is present.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bandchol.c")
_LIB = os.path.join(_HERE, "liboracle_band.so")
_handle = None


def build() -> str:
    """Compile the oracle C sources (always recompiles)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-Wextra", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _handle
    if _handle is None:
        if not os.path.exists(_LIB):
            build()
        h = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        h.oracle_band_solve.argtypes = [ctypes.c_int64, ctypes.c_int, dp, dp, ctypes.c_int,
                                        dp, dp, dp, ctypes.c_int]
        h.oracle_band_solve.restype = ctypes.c_int
        h.oracle_band_residual_dd.argtypes = [ctypes.c_int64, ctypes.c_int, dp, dp,
                                              ctypes.c_int, dp, dp, dp, dp]
        h.oracle_band_residual_dd.restype = None
        h.oracle_shift_dd.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, dp, dp]
        h.oracle_shift_dd.restype = None
        h.oracle_cband_solve.argtypes = [ctypes.c_int64, ctypes.c_int, dp, dp, dp, dp,
                                         ctypes.c_int, dp, dp, dp, dp, dp, dp, ctypes.c_int]
        h.oracle_cband_solve.restype = ctypes.c_int
        h.oracle_shift_cdd.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, dp, dp, dp, dp]
        h.oracle_shift_cdd.restype = None
        _handle = h
    return _handle


def dptr(a):
    """ctypes double* for a C-contiguous float64 numpy array (or None)."""
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
