"""Builds the dense S x S windows of G from per-axis tap vectors (+ DDE kernel).

The heavy loop lives in ``_windows.c`` (built on first use with gcc); a plain
NumPy path (``windows_numpy``) exists for tiny inputs and for cross-checks.
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "_windows.c")
_LIB = os.path.join(_HERE, "_windows.so")
_lock = threading.Lock()
_lib = None

SKW_MAX = 32
SD_MAX = 7


def build(force=False):
    """Compile the window builder (gcc -O3 -fopenmp)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            lib.synth_windows.restype = ctypes.c_int
            lib.synth_windows.argtypes = [
                ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
            _lib = lib
    return _lib


def window_offsets(S):
    """Element offset of each visibility's window in the flat array (+ total)."""
    sq = np.asarray(S, dtype=np.int64) ** 2
    off = np.zeros(len(sq) + 1, dtype=np.int64)
    np.cumsum(sq, out=off[1:])
    return off


def windows_c(skw, uy, ux, pair_id=None, pairs=None, pair_sd=None, dtype=np.complex128):
    """Flat windows (row-major S x S per visibility) and their offsets."""
    lib = _load()
    skw = np.ascontiguousarray(skw, dtype=np.int32)
    uy = np.ascontiguousarray(uy, dtype=np.complex128)
    ux = np.ascontiguousarray(ux, dtype=np.complex128)
    M = len(skw)
    if pair_id is not None:
        pair_id = np.ascontiguousarray(pair_id, dtype=np.int32)
        pairs = np.ascontiguousarray(pairs, dtype=np.complex128)
        pair_sd = np.ascontiguousarray(pair_sd, dtype=np.int32)
        assert pairs.shape[1:] == (SD_MAX, SD_MAX)
        sd = np.where(pair_id >= 0, pair_sd[np.maximum(pair_id, 0)], 1)
    else:
        sd = np.ones(M, dtype=np.int32)
    S = skw + sd - 1
    off = window_offsets(S)
    out = np.empty(int(off[-1]), dtype=dtype)
    kind = 0 if dtype == np.complex128 else 1
    if dtype not in (np.complex128, np.complex64):
        raise ValueError("dtype must be complex128 or complex64")
    rc = lib.synth_windows(
        M, skw.ctypes.data, uy.ctypes.data, ux.ctypes.data, uy.shape[1],
        pair_id.ctypes.data if pair_id is not None else None,
        pairs.ctypes.data if pair_id is not None else None,
        pair_sd.ctypes.data if pair_id is not None else None,
        off.ctypes.data, out.ctypes.data, kind)
    if rc != 0:
        raise ValueError("synth_windows: bad sizes")
    return out, off, S.astype(np.int32)


def windows_numpy(skw, uy, ux, pair_id=None, pairs=None, pair_sd=None):
    """Reference path with scipy.signal.convolve2d (tiny inputs only)."""
    from scipy.signal import convolve2d
    wins = []
    S = []
    for m in range(len(skw)):
        k = int(skw[m])
        w = np.outer(uy[m, :k], ux[m, :k])
        if pair_id is not None and pair_id[m] >= 0:
            sd = int(pair_sd[pair_id[m]])
            w = convolve2d(w, pairs[pair_id[m], :sd, :sd], mode="full")
        wins.append(w.ravel())
        S.append(w.shape[0])
    S = np.asarray(S, dtype=np.int32)
    return np.concatenate(wins), window_offsets(S), S
