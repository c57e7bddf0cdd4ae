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
        L.oracle_rir_batch_lut.restype = ctypes.c_int
        L.oracle_rir_batch_lut.argtypes = [ctypes.POINTER(_Room), dp, ctypes.c_int, dp, ctypes.c_int,
                                           ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int, dp]
        L.oracle_rir_batch_polar.restype = ctypes.c_int
        L.oracle_rir_batch_polar.argtypes = [ctypes.POINTER(_Room), dp, ctypes.c_int, dp, ctypes.c_int, dp,
                                             ctypes.c_double, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                             ctypes.c_int, dp]
        L.oracle_lut_taps.restype = ctypes.c_int
        L.oracle_lut_taps.argtypes = [dp, ctypes.c_int64, ctypes.c_double, ctypes.c_int, dp]
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
        n_threads: int | None = None, lut_q: int = 0) -> np.ndarray:
    """RIRs [n_src, n_rcv, k_end - k_begin] in float64 (default: the whole RIR).

    lut_q > 0: every tap from the table of Eq. (9) at lut_q points per sample
    with linear interpolation (Sec. 3.5) instead of Eq. (6) itself."""
    room = _room(L, beta, n_img, c, fs, t_max, t_w)
    nS = n_samples(t_max, fs)
    if k_end is None:
        k_end = nS
    s = _pos(src)
    r = _pos(rcv)
    out = np.zeros((s.shape[0], r.shape[0], k_end - k_begin))
    nt = n_threads or max(1, min(os.cpu_count() or 1, s.shape[0] * r.shape[0]))
    st = lib().oracle_rir_batch_lut(ctypes.byref(room), _dptr(s), s.shape[0], _dptr(r), r.shape[0],
                                    int(k_begin), int(k_end), int(lut_q), int(nt), _dptr(out))
    if st != 0:
        raise ValueError(f"oracle_rir_batch failed with status {st}")
    return out


def rir_polar(L, beta, n_img, c, fs, t_max, t_w, src, rcv, orient, pattern_a: float, k_begin: int = 0,
              k_end: int | None = None, n_threads: int | None = None, lut_q: int = 0) -> np.ndarray:
    """RIRs [n_src, n_rcv, k_end - k_begin] with directional receivers: each image's
    amplitude times a + (1 - a) cos(theta), theta between orient[r] and the
    direction from the receiver to the image (first-order pattern family).
    lut_q > 0: table taps as in ``rir``."""
    room = _room(L, beta, n_img, c, fs, t_max, t_w)
    if k_end is None:
        k_end = n_samples(t_max, fs)
    s, r, o = _pos(src), _pos(rcv), _pos(orient)
    if o.shape != r.shape:
        raise ValueError("orient must be [n_rcv, 3]")
    out = np.zeros((s.shape[0], r.shape[0], k_end - k_begin))
    nt = n_threads or max(1, min(os.cpu_count() or 1, s.shape[0] * r.shape[0]))
    st = lib().oracle_rir_batch_polar(ctypes.byref(room), _dptr(s), s.shape[0], _dptr(r), r.shape[0], _dptr(o),
                                      float(pattern_a), int(k_begin), int(k_end), int(lut_q), int(nt), _dptr(out))
    if st != 0:
        raise ValueError(f"oracle_rir_batch_polar failed with status {st}")
    return out


def lut_taps(v, W: float, q: int = 16) -> np.ndarray:
    """Table taps of Sec. 3.5 (Eq. (9) table, q points per sample, linear
    interpolation) at offsets v = k - x in samples; 0 where |v| >= W/2."""
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float64).ravel())
    out = np.zeros_like(v)
    if lib().oracle_lut_taps(_dptr(v), v.size, float(W), int(q), _dptr(out)) != 0:
        raise ValueError("q W / 2 must be an integer")
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


# ---------------------------------------------------------------------------
# Diffuse reverberation (Sec. 2.2, Eq. (8); Sec. 3.3): the RIR after t_diff is
# logistic noise times the square root of an exponential power envelope whose
# level A is estimated from the ISM part. Plain float64 numpy, written from the
# definitions; the random bits come from the Philox4x32-10 counter-based
# generator of Salmon et al. (SC'11), implemented from its published
# definition (the GPU library implements the same definition independently).
# ---------------------------------------------------------------------------
_PHILOX_M = (0xD2511F53, 0xCD9E8D57)  # round multipliers
_PHILOX_W = (0x9E3779B9, 0xBB67AE85)  # key increments between rounds
_MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds. ctr: four uint32 arrays (broadcastable),
    key: two uint32 scalars. Returns four uint32 arrays.

    One round maps (c0, c1, c2, c3) with key (k0, k1) to
    (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)), where hi
    and lo are the upper and lower 32 bits of the 64-bit product; the key is
    advanced by the two Weyl increments before every round but the first."""
    c = [np.asarray(x, dtype=np.uint64) & _MASK32 for x in ctr]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    m0, m1 = np.uint64(_PHILOX_M[0]), np.uint64(_PHILOX_M[1])
    for r in range(10):
        if r > 0:
            k0 = (k0 + _PHILOX_W[0]) & 0xFFFFFFFF
            k1 = (k1 + _PHILOX_W[1]) & 0xFFFFFFFF
        p0 = m0 * c[0]
        p1 = m1 * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ np.uint64(k0), p1 & _MASK32,
             (p0 >> np.uint64(32)) ^ c[3] ^ np.uint64(k1), p0 & _MASK32]
    return [x.astype(np.uint32) for x in c]


def noise_bits(seed: int, rir_index: int, k: np.ndarray) -> np.ndarray:
    """Random word of sample k of RIR rir_index: Philox4x32-10 with counter
    (k // 4, rir_index, 0, 0) and key (low, high 32 bits of seed), word k % 4."""
    k = np.asarray(k, dtype=np.int64)
    blk = (k // 4).astype(np.uint64)
    zero = np.zeros_like(blk)
    out = philox4x32_10([blk, zero + np.uint64(rir_index), zero, zero], (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    words = np.stack(out, axis=-1)
    return np.take_along_axis(words, (k % 4)[..., None], axis=-1)[..., 0]


def logistic_from_bits(x: np.ndarray) -> np.ndarray:
    """Unit-variance logistic variate from a uint32 word: the logistic quantile
    function log(u / (1 - u)) at u = (x + 1/2) / 2^32, scaled by sqrt(3)/pi
    (a logistic law of scale s has variance s^2 pi^2 / 3)."""
    x = np.asarray(x, dtype=np.float64)
    return np.log((x + 0.5) / (4294967296.0 - 0.5 - x)) * (np.sqrt(3.0) / np.pi)


def envelope(k: np.ndarray, fs: float, t_diff: float, t60: float) -> np.ndarray:
    """Power envelope shape 10^(-6 (t - t_diff) / T60) at t = k / fs: the power
    falls by 60 dB in T60 (Sabine), normalised to 1 at t_diff."""
    t = np.asarray(k, dtype=np.float64) / fs
    return 10.0 ** (-6.0 * (t - t_diff) / t60)


def diffuse_window(k_diff: int) -> tuple:
    """Samples [k_w, k_diff) of the ISM part that set the envelope level: the
    last fifth of the ISM part (at least one sample)."""
    return k_diff - max(1, k_diff // 5), k_diff


def envelope_level(h_ism: np.ndarray, fs: float, t_diff: float, t60: float) -> np.ndarray:
    """A per RIR: the mean of h[k]^2 / envelope(k) over the window of the ISM
    part h_ism [..., k_diff] (least-squares level of the exponential envelope
    fitted to the ISM energy there)."""
    k_diff = h_ism.shape[-1]
    k0, k1 = diffuse_window(k_diff)
    k = np.arange(k0, k1)
    return np.mean(h_ism[..., k0:k1] ** 2 / envelope(k, fs, t_diff, t60), axis=-1)


def diffuse_rir(L, beta, n_img, c, fs, t_max, t_w, t_diff, t60, seed, src, rcv) -> np.ndarray:
    """Full RIRs [n_src, n_rcv, nS(t_max)]: the ISM part (lattice n_img, up to
    k_diff = nS(t_diff) samples), then for k >= k_diff logistic noise times
    sqrt(A envelope(k)). RIR index i = source * n_rcv + receiver selects the
    noise stream."""
    nS = n_samples(t_max, fs)
    k_diff = n_samples(t_diff, fs)
    h_ism = rir(L, beta, n_img, c, fs, t_diff, t_w, src, rcv)
    n_src, n_rcv = h_ism.shape[:2]
    A = envelope_level(h_ism, fs, t_diff, t60)
    out = np.zeros((n_src, n_rcv, nS))
    out[..., :k_diff] = h_ism
    k = np.arange(k_diff, nS)
    env = envelope(k, fs, t_diff, t60)
    for i in range(n_src * n_rcv):
        s, r = divmod(i, n_rcv)
        z = logistic_from_bits(noise_bits(seed, i, k))
        out[s, r, k_diff:] = z * np.sqrt(A[s, r] * env)
    return out


# ---------------------------------------------------------------------------
# Moving source (Sec. 3.4): overlap-add of the source signal's segments, each
# convolved (numpy's direct convolution, float64) with the RIR of its
# trajectory point.
# ---------------------------------------------------------------------------
def filter_trajectory(x, rirs) -> np.ndarray:
    """x [n_x], rirs [n_pos, n_mic, n_rir] -> y [n_mic, n_x + n_rir - 1]:
    segment p = x[p L : (p + 1) L] with L = ceil(n_x / n_pos) is convolved with
    rirs[p, m] and added at offset p L."""
    x = np.asarray(x, dtype=np.float64)
    rirs = np.asarray(rirs, dtype=np.float64)
    n_pos, n_mic, n_rir = rirs.shape
    n_x = x.shape[0]
    seg = -(-n_x // n_pos)
    y = np.zeros((n_mic, n_x + n_rir - 1))
    for p in range(n_pos):
        xs = x[p * seg:(p + 1) * seg]
        if xs.size == 0:
            continue
        for m in range(n_mic):
            y[m, p * seg:p * seg + xs.size + n_rir - 1] += np.convolve(xs, rirs[p, m])
    return y


def filter_samples(x, rirs, m: int, n_idx) -> np.ndarray:
    """Selected outputs of the moving-source filter, one by one from the
    definition: y_m[n] = sum_k x[n - k] rirs[p(n - k), m, k] over the k with
    0 <= n - k < n_x, p(i) = floor(i / L), L = ceil(n_x / n_pos) (float64).
    Equal to filter_trajectory(x, rirs)[m, n_idx]."""
    x = np.asarray(x, dtype=np.float64)
    n_pos, n_mic, n_rir = np.asarray(rirs).shape
    n_x = x.shape[0]
    seg = -(-n_x // n_pos)
    out = np.zeros(len(n_idx))
    for t, n in enumerate(n_idx):
        k = np.arange(max(0, n - n_x + 1), min(n_rir, n + 1))
        i = n - k
        h = np.asarray(rirs[i // seg, m, k], dtype=np.float64)
        out[t] = float(np.sum(x[i] * h))
    return out
