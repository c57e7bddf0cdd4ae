"""ctypes front end of the FP64 ISM oracle (ism_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by ``__graft_entry__.smoke()`` and
by the CPU-baseline leg of ``bench.py``. The GPU library never imports it.

Every function takes plain numbers / numpy arrays and returns numpy float64
arrays. Positions are promoted from float32 exactly, so the oracle and the GPU
library solve the same problem instance.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_DIR, "ism_oracle.c")
_LIB = os.path.join(_DIR, "libism_oracle.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no fast-math) into oracle/libism_oracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
             _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Room(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3), ("beta", ctypes.c_double * 6), ("n", ctypes.c_int * 3),
                ("c", ctypes.c_double), ("fs", ctypes.c_double), ("t_max", ctypes.c_double),
                ("t_w", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_n_samples.restype = ctypes.c_int64
        L.oracle_n_samples.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_beta_from_t60.restype = ctypes.c_int
        L.oracle_beta_from_t60.argtypes = [dp, ctypes.c_double, dp]
        L.oracle_n_img_for_time.restype = None
        L.oracle_n_img_for_time.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
        L.oracle_time_for_attenuation.restype = ctypes.c_double
        L.oracle_time_for_attenuation.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_rir_window.restype = ctypes.c_int
        L.oracle_rir_window.argtypes = [ctypes.POINTER(_Room), dp, dp, ctypes.c_int64, ctypes.c_int64, dp]
        L.oracle_rir_batch.restype = ctypes.c_int
        L.oracle_rir_batch.argtypes = [ctypes.POINTER(_Room), dp, ctypes.c_int, dp, ctypes.c_int,
                                       ctypes.c_int64, ctypes.c_int64, ctypes.c_int, dp]
        L.oracle_image_list.restype = ctypes.c_int64
        L.oracle_image_list.argtypes = [ctypes.POINTER(_Room), dp, dp, ctypes.POINTER(ctypes.c_int32), dp,
                                        ctypes.c_int64]
        L.oracle_count_taps.restype = ctypes.c_int64
        L.oracle_count_taps.argtypes = [ctypes.POINTER(_Room), dp, dp]
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _room(L, beta, n_img, c, fs, t_max, t_w) -> _Room:
    r = _Room()
    for i in range(3):
        r.L[i] = float(L[i])
        r.n[i] = int(n_img[i])
    for i in range(6):
        r.beta[i] = float(beta[i])
    r.c, r.fs, r.t_max, r.t_w = float(c), float(fs), float(t_max), float(t_w)
    return r


def _pos(p) -> np.ndarray:
    """Positions as float64, promoted from float32 so both sides see the same values."""
    return np.ascontiguousarray(np.asarray(p, dtype=np.float32).astype(np.float64).reshape(-1, 3))


def n_samples(t_max: float, fs: float) -> int:
    return int(lib().oracle_n_samples(float(t_max), float(fs)))


def beta_from_t60(L, t60: float) -> np.ndarray:
    Lv = np.ascontiguousarray(L, dtype=np.float64)
    out = np.zeros(6)
    st = lib().oracle_beta_from_t60(_dptr(Lv), float(t60), _dptr(out))
    if st != 0:
        raise ValueError(f"infeasible T60 {t60} for room {list(L)} (status {st})")
    return out


def n_img_for_time(L, c: float, t: float) -> tuple:
    Lv = np.ascontiguousarray(L, dtype=np.float64)
    n = (ctypes.c_int * 3)()
    lib().oracle_n_img_for_time(_dptr(Lv), float(c), float(t), n)
    return (n[0], n[1], n[2])


def time_for_attenuation(t60: float, att_db: float) -> float:
    return float(lib().oracle_time_for_attenuation(float(t60), float(att_db)))


def rir(L, beta, n_img, c, fs, t_max, t_w, src, rcv, k_begin: int = 0, k_end: int | None = None,
        n_threads: int | None = None) -> np.ndarray:
    """RIRs [n_src, n_rcv, k_end - k_begin] in float64 (default: the whole RIR)."""
    room = _room(L, beta, n_img, c, fs, t_max, t_w)
    nS = n_samples(t_max, fs)
    if k_end is None:
        k_end = nS
    s = _pos(src)
    r = _pos(rcv)
    out = np.zeros((s.shape[0], r.shape[0], k_end - k_begin))
    nt = n_threads or max(1, min(os.cpu_count() or 1, s.shape[0] * r.shape[0]))
    st = lib().oracle_rir_batch(ctypes.byref(room), _dptr(s), s.shape[0], _dptr(r), r.shape[0],
                                int(k_begin), int(k_end), int(nt), _dptr(out))
    if st != 0:
        raise ValueError(f"oracle_rir_batch failed with status {st}")
    return out


def image_list(L, beta, n_img, c, fs, t_max, t_w, src, rcv):
    """(idx [n,3] int32, vals [n,4] float64 = gain, d, x, A) for every lattice image."""
    room = _room(L, beta, n_img, c, fs, t_max, t_w)
    s = _pos(src)[0]
    r = _pos(rcv)[0]
    n = int(lib().oracle_image_list(ctypes.byref(room), _dptr(s), _dptr(r), None, None, 0))
    idx = np.zeros((n, 3), dtype=np.int32)
    vals = np.zeros((n, 4))
    lib().oracle_image_list(ctypes.byref(room), _dptr(s), _dptr(r),
                            idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dptr(vals), n)
    return idx, vals


def count_taps(L, beta, n_img, c, fs, t_max, t_w, src, rcv) -> int:
    """Exact tap count summed over all (src, rcv) pairs."""
    room = _room(L, beta, n_img, c, fs, t_max, t_w)
    total = 0
    for s in _pos(src):
        sv = np.ascontiguousarray(s)
        for r in _pos(rcv):
            rv = np.ascontiguousarray(r)
            total += int(lib().oracle_count_taps(ctypes.byref(room), _dptr(sv), _dptr(rv)))
    return total
