"""Oracle -- test infrastructure only.  Builds and loads the plain-C ladder oracle.

``build()`` compiles ``ppl_oracle.c`` with gcc (-O3, OpenMP, portable x86-64-v3
code so the library also runs on another host CPU).  ``lib()`` loads it and
builds it first when it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ppl_oracle.c")
_SO = os.path.join(_HERE, "libppl_oracle.so")
_lib = None


def build() -> str:
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.oracle_ppl.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.oracle_ppl.restype = ctypes.c_int
        L.oracle_ppl_pairs.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip,
                                       ctypes.c_int, dp]
        L.oracle_ppl_pairs.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def _dp(x):
    return x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def ppl(B_vv: np.ndarray, tau: np.ndarray, R: np.ndarray | None = None) -> np.ndarray:
    """R += sum_cd (ac|bd) tau^{cd}_{ij}; returns R (a new zero array when None)."""
    naux, v, v2 = B_vv.shape
    o = tau.shape[0]
    assert v == v2 and tau.shape == (o, o, v, v)
    B_vv = np.ascontiguousarray(B_vv, dtype=np.float64)
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    if R is None:
        R = np.zeros((o, o, v, v))
    assert R.flags.c_contiguous and R.dtype == np.float64 and R.shape == tau.shape
    rc = lib().oracle_ppl(_dp(B_vv), _dp(tau), o, v, naux, _dp(R))
    if rc != 0:
        raise RuntimeError(f"oracle_ppl failed ({rc})")
    return R


def ppl_pairs(B_vv: np.ndarray, tau: np.ndarray, pairs) -> np.ndarray:
    """[p][i][j] = L^{a_p b_p}_{ij} for the given (a, b) pairs."""
    naux, v, _ = B_vv.shape
    o = tau.shape[0]
    B_vv = np.ascontiguousarray(B_vv, dtype=np.float64)
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    ab = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    out = np.zeros((ab.shape[0], o, o))
    rc = lib().oracle_ppl_pairs(_dp(B_vv), _dp(tau), o, v, naux,
                                ab.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ab.shape[0], _dp(out))
    if rc != 0:
        raise RuntimeError(f"oracle_ppl_pairs failed ({rc})")
    return out


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    lib().oracle_set_num_threads(int(n))
