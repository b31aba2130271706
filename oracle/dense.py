"""ctypes wrapper of the FP64 dense oracle in ``dense.c`` (test
infrastructure only).

``potential(src, q, k, tgt=None)`` and ``field(src, q, k, tgt=None)`` follow
the pair-potential definition of the paper's problem statement (Sec. 2,
Eq. for Phi(r)) with G(r) = exp(ikr)/r; pairs of bit-identical points are
skipped (no self term).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dense.c")
_LIB = os.path.join(_HERE, "_dense.so")
_lib = None


def build(force=False):
    """Compile dense.c into _dense.so with gcc (FP64, IEEE, OpenMP)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC,
             "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        args = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                ctypes.c_double, ctypes.c_void_p]
        for name in ("oracle_dense_potential", "oracle_dense_field"):
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = None
        _lib = lib
    return _lib


def _prep(src, q, tgt):
    src = np.ascontiguousarray(src, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q)
    squeeze = q.ndim == 1
    q = np.ascontiguousarray(q.reshape(src.shape[0], -1), dtype=np.complex128)
    tgt = src if tgt is None else np.ascontiguousarray(
        tgt, dtype=np.float64).reshape(-1, 3)
    return src, q, tgt, squeeze


def potential(src, q, k, tgt=None):
    """phi[t, c] = sum_{s != t} exp(ik|r_t - r_s|)/|r_t - r_s| q[s, c]."""
    src, q, tgt, squeeze = _prep(src, q, tgt)
    nrhs = q.shape[1]
    out = np.empty((tgt.shape[0], nrhs), dtype=np.complex128)
    _load().oracle_dense_potential(
        src.shape[0], src.ctypes.data, q.ctypes.data, tgt.shape[0],
        tgt.ctypes.data, nrhs, float(k), out.ctypes.data)
    return out[:, 0] if squeeze else out


def field(src, q, k, tgt=None):
    """grad[t, c, :] = sum_{s != t} grad_r G(r_t - r_s) q[s, c]."""
    src, q, tgt, squeeze = _prep(src, q, tgt)
    nrhs = q.shape[1]
    out = np.empty((tgt.shape[0], nrhs, 3), dtype=np.complex128)
    _load().oracle_dense_field(
        src.shape[0], src.ctypes.data, q.ctypes.data, tgt.shape[0],
        tgt.ctypes.data, nrhs, float(k), out.ctypes.data)
    return out[:, 0, :] if squeeze else out
