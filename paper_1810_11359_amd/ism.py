"""Thin ctypes binding of libism.so (include/ism.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels of the library. PyTorch provides device memory and the stream. The
library must be built (``python -m paper_1810_11359_amd.build`` or
``__graft_entry__.build()``); importing the binding without it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libism.so")

ISM_OK = 0
ISM_E_INVALID_ARG = -1
ISM_E_INFEASIBLE_T60 = -2
ISM_E_OUT_OF_ROOM = -3
ISM_E_WORKSPACE = -4
ISM_E_DEVICE = -5
ISM_E_TOO_LARGE = -6
ISM_E_UNSUPPORTED = -7
# Limits of the library (ISM_E_TOO_LARGE beyond them), as in include/ism.h.
ISM_MAX_SAMPLES = 256 * 1024
ISM_MAX_N_IMG = 2048
ISM_MAX_PAIRS = 1 << 22

PRECISIONS = {"fp32": 0, "fp16": 1, "bf16": 2, "lut": 3}

# Every symbol include/ism.h declares.
EXPORTS = (
    "ism_status_string", "ism_abi_version", "ism_beta_from_t60", "ism_n_img_for_time",
    "ism_time_for_attenuation", "ism_n_samples", "ism_check_room", "ism_check_positions",
    "ism_count_taps", "ism_workspace_size", "ism_simulate", "ism_simulate_timed", "ism_simulate_polar",
    "ism_simulate_diffuse_polar",
    "ism_batch_workspace_size", "ism_batch_prepare", "ism_batch_run", "ism_batch_run_timed",
    "ism_diffuse_workspace_size", "ism_simulate_diffuse", "ism_simulate_diffuse_timed",
    "ism_filter_trajectory", "ism_workspace_size_ex", "ism_simulate_ex", "ism_simulate_host",
    "ism_batch_workspace_size_ex", "ism_batch_prepare_ex", "ism_simulate_batch", "ism_debug_enumerate",
    "ism_simulate_noalloc", "ism_filter_workspace_size", "ism_filter_trajectory_ex",
)


class IsmError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_string(status)} (status {status})")
        self.status = status


class _Room(ctypes.Structure):
    _fields_ = [("room", ctypes.c_double * 3), ("beta", ctypes.c_double * 6), ("n_img", ctypes.c_int * 3),
                ("c", ctypes.c_double), ("fs", ctypes.c_double), ("t_max", ctypes.c_double),
                ("t_w", ctypes.c_double)]


class _Job(ctypes.Structure):
    _fields_ = [("room", _Room), ("src", ctypes.c_void_p), ("n_src", ctypes.c_int), ("rcv", ctypes.c_void_p),
                ("n_rcv", ctypes.c_int), ("out", ctypes.c_void_p), ("orient", ctypes.c_void_p),
                ("pattern", ctypes.c_double)]


class _Batch(ctypes.Structure):
    _fields_ = [("opaque", ctypes.c_uint64 * 40)]


class _Schedule(ctypes.Structure):
    _fields_ = [("item_taps", ctypes.c_double), ("min_item_taps", ctypes.c_double),
                ("balance_items", ctypes.c_double), ("tail_rounds", ctypes.c_double),
                ("batch_waves", ctypes.c_double)]


@dataclass
class Schedule:
    """Work split of a call (``ism_schedule``): 0 keeps a field's default
    (tail_rounds: a negative value does)."""
    item_taps: float = 0.0
    min_item_taps: float = 0.0
    balance_items: float = 0.0
    tail_rounds: float = -1.0
    batch_waves: float = 0.0

    def _c(self) -> _Schedule:
        return _Schedule(float(self.item_taps), float(self.min_item_taps), float(self.balance_items),
                         float(self.tail_rounds), float(self.batch_waves))


def _sched(schedule):
    """ctypes pointer argument for an optional Schedule (None -> NULL)."""
    return None if schedule is None else ctypes.byref(schedule._c())


# One record of ism_debug_enumerate (include/ism_debug.h).
IMAGE_RECORD = np.dtype([("rir", "<i4"), ("n", "<i4", (3,)), ("k0", "<i4"), ("fq", "<u4"), ("amp", "<f4"),
                         ("pad", "<u4")])


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libism.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python -m paper_1810_11359_amd.build)")
        # torch first: its HIP runtime is then the one the library binds to, so
        # both share one runtime (devices, streams, memory). Loaded the other
        # way round, the process can end up with two runtimes, and the
        # library's sees no device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        dp, ip, fp = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.c_void_p
        rp = ctypes.POINTER(_Room)
        L.ism_status_string.restype = ctypes.c_char_p
        L.ism_status_string.argtypes = [ctypes.c_int]
        L.ism_abi_version.restype = ctypes.c_int
        L.ism_abi_version.argtypes = []
        L.ism_beta_from_t60.restype = ctypes.c_int
        L.ism_beta_from_t60.argtypes = [dp, ctypes.c_double, dp]
        L.ism_n_img_for_time.restype = ctypes.c_int
        L.ism_n_img_for_time.argtypes = [dp, ctypes.c_double, ctypes.c_double, ip]
        L.ism_time_for_attenuation.restype = ctypes.c_int
        L.ism_time_for_attenuation.argtypes = [ctypes.c_double, ctypes.c_double, dp]
        L.ism_n_samples.restype = ctypes.c_int64
        L.ism_n_samples.argtypes = [ctypes.c_double, ctypes.c_double]
        L.ism_check_room.restype = ctypes.c_int
        L.ism_check_room.argtypes = [rp]
        L.ism_check_positions.restype = ctypes.c_int
        L.ism_check_positions.argtypes = [rp, fp, ctypes.c_int, fp, ctypes.c_int]
        L.ism_count_taps.restype = ctypes.c_int
        L.ism_count_taps.argtypes = [rp, fp, ctypes.c_int, fp, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)]
        L.ism_workspace_size.restype = ctypes.c_int
        L.ism_workspace_size.argtypes = [rp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.ism_simulate.restype = ctypes.c_int
        L.ism_simulate.argtypes = [rp, fp, ctypes.c_int, fp, ctypes.c_int, ctypes.c_int, fp, fp, ctypes.c_size_t, fp]
        jp = ctypes.POINTER(_Job)
        L.ism_batch_workspace_size.restype = ctypes.c_int
        L.ism_batch_workspace_size.argtypes = [jp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.ism_batch_prepare.restype = ctypes.c_int
        L.ism_batch_prepare.argtypes = [jp, ctypes.c_int, ctypes.c_int, fp, ctypes.c_size_t, fp, ctypes.POINTER(_Batch)]
        L.ism_batch_run.restype = ctypes.c_int
        L.ism_batch_run.argtypes = [ctypes.POINTER(_Batch), fp]
        L.ism_batch_run_timed.restype = ctypes.c_int
        L.ism_batch_run_timed.argtypes = [ctypes.POINTER(_Batch), fp, fp, fp]
        L.ism_simulate_timed.restype = ctypes.c_int
        L.ism_simulate_timed.argtypes = [rp, fp, ctypes.c_int, fp, ctypes.c_int, ctypes.c_int, fp, fp, ctypes.c_size_t,
                                         fp, fp, fp]
        L.ism_simulate_polar.restype = ctypes.c_int
        L.ism_simulate_polar.argtypes = [rp, fp, ctypes.c_int, fp, ctypes.c_int, fp, ctypes.c_double, ctypes.c_int,
                                         fp, fp, ctypes.c_size_t, fp]
        L.ism_simulate_diffuse_polar.restype = ctypes.c_int
        L.ism_simulate_diffuse_polar.argtypes = [rp, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, fp, ctypes.c_int,
                                                 fp, ctypes.c_int, fp, ctypes.c_double, ctypes.c_int, fp, fp,
                                                 ctypes.c_size_t, fp]
        L.ism_diffuse_workspace_size.restype = ctypes.c_int
        L.ism_diffuse_workspace_size.argtypes = [rp, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
        L.ism_simulate_diffuse.restype = ctypes.c_int
        L.ism_simulate_diffuse.argtypes = [rp, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, fp, ctypes.c_int, fp,
                                           ctypes.c_int, ctypes.c_int, fp, fp, ctypes.c_size_t, fp]
        L.ism_filter_trajectory.restype = ctypes.c_int
        L.ism_filter_trajectory.argtypes = [fp, ctypes.c_int, fp, ctypes.c_int, ctypes.c_int, ctypes.c_int, fp, fp]
        sp = ctypes.POINTER(_Schedule)
        L.ism_workspace_size_ex.restype = ctypes.c_int
        L.ism_workspace_size_ex.argtypes = [rp, ctypes.c_int, ctypes.c_int, ctypes.c_int, sp,
                                            ctypes.POINTER(ctypes.c_size_t)]
        L.ism_simulate_ex.restype = ctypes.c_int
        L.ism_simulate_ex.argtypes = [rp, fp, ctypes.c_int, fp, ctypes.c_int, ctypes.c_int, sp, fp, fp,
                                      ctypes.c_size_t, fp, fp, fp]
        L.ism_simulate_host.restype = ctypes.c_int
        L.ism_simulate_host.argtypes = [rp, fp, ctypes.c_int, fp, ctypes.c_int, ctypes.c_int, fp, fp,
                                        ctypes.c_size_t, fp]
        L.ism_batch_workspace_size_ex.restype = ctypes.c_int
        L.ism_batch_workspace_size_ex.argtypes = [jp, ctypes.c_int, ctypes.c_int, sp, ctypes.POINTER(ctypes.c_size_t)]
        L.ism_batch_prepare_ex.restype = ctypes.c_int
        L.ism_batch_prepare_ex.argtypes = [jp, ctypes.c_int, ctypes.c_int, sp, fp, ctypes.c_size_t, fp,
                                           ctypes.POINTER(_Batch)]
        L.ism_simulate_batch.restype = ctypes.c_int
        L.ism_simulate_batch.argtypes = [jp, ctypes.c_int, ctypes.c_int, fp, ctypes.c_size_t, fp]
        L.ism_debug_enumerate.restype = ctypes.c_int
        L.ism_debug_enumerate.argtypes = [rp, fp, ctypes.c_int, fp, ctypes.c_int, sp, fp, ctypes.c_uint32, fp, fp,
                                          ctypes.c_size_t, fp]
        L.ism_filter_workspace_size.restype = ctypes.c_int
        L.ism_filter_workspace_size.argtypes = [ctypes.c_int] * 5 + [ctypes.POINTER(ctypes.c_size_t)]
        L.ism_filter_trajectory_ex.restype = ctypes.c_int
        L.ism_filter_trajectory_ex.argtypes = [fp, ctypes.c_int, fp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, fp, fp, ctypes.c_size_t, fp]
        L.ism_simulate_noalloc.restype = ctypes.c_int
        L.ism_simulate_noalloc.argtypes = [rp, fp, ctypes.c_int, fp, ctypes.c_int, ctypes.c_int, fp, fp]
        L.ism_simulate_diffuse_timed.restype = ctypes.c_int
        L.ism_simulate_diffuse_timed.argtypes = [rp, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, fp,
                                                 ctypes.c_int, fp, ctypes.c_int, ctypes.c_int, fp, fp, ctypes.c_size_t,
                                                 fp, fp, fp]
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().ism_status_string(int(status)).decode()


def _check(status: int, where: str) -> None:
    if status != ISM_OK:
        raise IsmError(status, where)


@dataclass
class Room:
    """One shoebox room (fields as in ``ism_room`` of include/ism.h)."""
    room: Sequence[float]
    beta: Sequence[float]
    n_img: Sequence[int]
    c: float = 343.0
    fs: float = 16000.0
    t_max: float = 0.5
    t_w: float = 0.004

    def _c(self) -> _Room:
        r = _Room()
        for i in range(3):
            r.room[i] = float(self.room[i])
            r.n_img[i] = int(self.n_img[i])
        for i in range(6):
            r.beta[i] = float(self.beta[i])
        r.c, r.fs, r.t_max, r.t_w = float(self.c), float(self.fs), float(self.t_max), float(self.t_w)
        return r

    @property
    def n_samples(self) -> int:
        return n_samples(self.t_max, self.fs)


def beta_from_t60(room: Sequence[float], t60: float) -> np.ndarray:
    L = (ctypes.c_double * 3)(*[float(v) for v in room])
    out = (ctypes.c_double * 6)()
    _check(lib().ism_beta_from_t60(L, float(t60), out), "ism_beta_from_t60")
    return np.array(out[:])


def n_img_for_time(room: Sequence[float], c: float, t: float) -> tuple:
    L = (ctypes.c_double * 3)(*[float(v) for v in room])
    n = (ctypes.c_int * 3)()
    _check(lib().ism_n_img_for_time(L, float(c), float(t), n), "ism_n_img_for_time")
    return (n[0], n[1], n[2])


def time_for_attenuation(t60: float, att_db: float) -> float:
    t = ctypes.c_double()
    _check(lib().ism_time_for_attenuation(float(t60), float(att_db), ctypes.byref(t)), "ism_time_for_attenuation")
    return t.value


def n_samples(t_max: float, fs: float) -> int:
    v = int(lib().ism_n_samples(float(t_max), float(fs)))
    if v < 0:
        raise IsmError(ISM_E_INVALID_ARG, "ism_n_samples")
    return v


def _host_pos(p) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(p, dtype=np.float32).reshape(-1, 3))


def check_positions(room: Room, src, rcv) -> None:
    s, r = _host_pos(src), _host_pos(rcv)
    rc = room._c()
    _check(lib().ism_check_positions(ctypes.byref(rc), s.ctypes.data, s.shape[0], r.ctypes.data, r.shape[0]),
           "ism_check_positions")


def count_taps(room: Room, src, rcv) -> int:
    s, r = _host_pos(src), _host_pos(rcv)
    rc = room._c()
    out = ctypes.c_int64()
    _check(lib().ism_count_taps(ctypes.byref(rc), s.ctypes.data, s.shape[0], r.ctypes.data, r.shape[0],
                                ctypes.byref(out)), "ism_count_taps")
    return out.value


def workspace_size(room: Room, n_src: int, n_rcv: int, precision: str = "fp32", schedule: Schedule = None) -> int:
    rc = room._c()
    out = ctypes.c_size_t()
    _check(lib().ism_workspace_size_ex(ctypes.byref(rc), int(n_src), int(n_rcv), PRECISIONS[precision],
                                       _sched(schedule), ctypes.byref(out)), "ism_workspace_size_ex")
    return out.value


class Simulator:
    """Reusable device state for repeated ``ism_simulate`` calls on one room shape.

    Holds the device positions, output tensor and workspace so a timed loop
    launches kernels only.
    """

    def __init__(self, room: Room, src, rcv, precision: str = "fp32", device: str = "cuda", check: bool = True,
                 schedule: Schedule = None):
        import torch

        self.torch = torch
        self.room = room
        self._room_c = room._c()
        self.schedule = schedule
        self._sched_c = None if schedule is None else schedule._c()
        s, r = _host_pos(src), _host_pos(rcv)
        if check:
            check_positions(room, s, r)
        self.precision = PRECISIONS[precision]
        self.src = torch.from_numpy(s).to(device)
        self.rcv = torch.from_numpy(r).to(device)
        self.n_src, self.n_rcv = s.shape[0], r.shape[0]
        self.out = torch.empty((self.n_src, self.n_rcv, room.n_samples), dtype=torch.float32, device=device)
        nbytes = workspace_size(room, self.n_src, self.n_rcv, precision, schedule)
        self.ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
        self.ws_bytes = nbytes

    def run(self, stream=None, ev_start=None, ev_stop=None):
        """Launch one simulation on ``stream`` (default: torch's current stream); returns the output tensor.

        ``ev_start``/``ev_stop`` are optional raw hipEvent_t handles recorded around the tap kernel."""
        st = stream if stream is not None else self.torch.cuda.current_stream()
        sc = None if self._sched_c is None else ctypes.byref(self._sched_c)
        _check(lib().ism_simulate_ex(ctypes.byref(self._room_c), self.src.data_ptr(), self.n_src,
                                     self.rcv.data_ptr(), self.n_rcv, self.precision, sc, self.out.data_ptr(),
                                     self.ws.data_ptr(), self.ws_bytes, st.cuda_stream, ev_start, ev_stop),
               "ism_simulate_ex")
        return self.out


def simulate(room: Room, src, rcv, precision: str = "fp32", device: str = "cuda", schedule: Schedule = None):
    """RIRs [n_src, n_rcv, nS] (float32, on ``device``) of every source/receiver pair."""
    return Simulator(room, src, rcv, precision, device, schedule=schedule).run()


def simulate_host(room: Room, src, rcv, precision: str = "fp32", out=None, device: str = "cuda"):
    """``ism_simulate_host``: positions passed from host memory and checked by
    the library before any launch. ``out`` (optional) is a float32 device
    tensor [n_src, n_rcv, nS] to overwrite; returns it."""
    import torch

    s, r = _host_pos(src), _host_pos(rcv)
    if out is None:
        out = torch.empty((s.shape[0], r.shape[0], room.n_samples), dtype=torch.float32, device=device)
    rc = room._c()
    nbytes = workspace_size(room, s.shape[0], r.shape[0], precision)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=out.device)
    st = torch.cuda.current_stream(out.device)
    _check(lib().ism_simulate_host(ctypes.byref(rc), s.ctypes.data, s.shape[0], r.ctypes.data, r.shape[0],
                                   PRECISIONS[precision], out.data_ptr(), ws.data_ptr(), nbytes, st.cuda_stream),
           "ism_simulate_host")
    return out


def debug_enumerate(room: Room, src, rcv, schedule: Schedule = None, cap: int = None, device: str = "cuda"):
    """``ism_debug_enumerate``: every image the work items of ``ism_simulate_ex``
    own, as a numpy array of IMAGE_RECORD (unordered). ``cap`` bounds the
    records fetched (default: the lattice size of all pairs)."""
    import torch

    s, r = _host_pos(src), _host_pos(rcv)
    n_rir = s.shape[0] * r.shape[0]
    if cap is None:
        cap = n_rir * int(np.prod(room.n_img))
    rc = room._c()
    nbytes = workspace_size(room, s.shape[0], r.shape[0], "fp32", schedule)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
    rec = torch.empty(max(cap, 1) * IMAGE_RECORD.itemsize, dtype=torch.uint8, device=device)
    cnt = torch.zeros(1, dtype=torch.int32, device=device)
    src_d, rcv_d = torch.from_numpy(s).to(device), torch.from_numpy(r).to(device)
    st = torch.cuda.current_stream()
    _check(lib().ism_debug_enumerate(ctypes.byref(rc), src_d.data_ptr(), s.shape[0], rcv_d.data_ptr(), r.shape[0],
                                     _sched(schedule), rec.data_ptr(), int(cap), cnt.data_ptr(), ws.data_ptr(),
                                     nbytes, st.cuda_stream), "ism_debug_enumerate")
    n = int(cnt.item()) & 0xFFFFFFFF
    if n > cap:
        raise IsmError(ISM_E_TOO_LARGE, f"ism_debug_enumerate: {n} images, cap {cap}")
    return np.frombuffer(rec[:n * IMAGE_RECORD.itemsize].cpu().numpy().tobytes(), dtype=IMAGE_RECORD)


# First-order receiver patterns a + (1 - a) cos(theta) (ism_simulate_polar).
PATTERNS = {"omni": 1.0, "subcardioid": 0.75, "cardioid": 0.5, "hypercardioid": 0.25, "bidirectional": 0.0}


def simulate_polar(room: Room, src, rcv, orient, pattern="cardioid", precision: str = "fp32", device: str = "cuda",
                   check: bool = True):
    """RIRs [n_src, n_rcv, nS] with directional receivers: ``orient`` [n_rcv, 3]
    orientations (normalised by the library), ``pattern`` a name of PATTERNS
    or the coefficient a in [0, 1]; ``precision`` as for ``simulate``."""
    import torch

    a = PATTERNS[pattern] if isinstance(pattern, str) else float(pattern)
    s, r = _host_pos(src), _host_pos(rcv)
    o = _host_pos(orient)
    if o.shape != r.shape:
        raise ValueError(f"orient must be [n_rcv, 3] = {r.shape}, got {o.shape}")
    if check:
        check_positions(room, s, r)
    rc = room._c()
    nbytes = workspace_size(room, s.shape[0], r.shape[0], precision)
    src_d, rcv_d, o_d = (torch.from_numpy(x).to(device) for x in (s, r, o))
    out = torch.empty((s.shape[0], r.shape[0], room.n_samples), dtype=torch.float32, device=device)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
    st = torch.cuda.current_stream()
    _check(lib().ism_simulate_polar(ctypes.byref(rc), src_d.data_ptr(), s.shape[0], rcv_d.data_ptr(), r.shape[0],
                                    o_d.data_ptr(), a, PRECISIONS[precision], out.data_ptr(), ws.data_ptr(), nbytes,
                                    st.cuda_stream), "ism_simulate_polar")
    return out


def diffuse_workspace_size(room: Room, t_diff: float, t60: float, n_src: int, n_rcv: int,
                           precision: str = "fp32") -> int:
    rc = room._c()
    out = ctypes.c_size_t()
    _check(lib().ism_diffuse_workspace_size(ctypes.byref(rc), float(t_diff), float(t60), int(n_src), int(n_rcv),
                                            PRECISIONS[precision], ctypes.byref(out)), "ism_diffuse_workspace_size")
    return out.value


class DiffuseSimulator:
    """Reusable device state for ``ism_simulate_diffuse``: RIRs [n_src, n_rcv, nS(t_max)]
    with the ISM part up to ``t_diff`` and a logistic-noise tail after it
    (Sec. 2.2, Eq. (8); Sec. 3.3)."""

    def __init__(self, room: Room, src, rcv, t_diff: float, t60: float, seed: int = 0, precision: str = "fp32",
                 device: str = "cuda", check: bool = True):
        import torch

        self.torch = torch
        self.room = room
        self._room_c = room._c()
        s, r = _host_pos(src), _host_pos(rcv)
        if check:
            check_positions(room, s, r)
        self.t_diff, self.t60, self.seed = float(t_diff), float(t60), int(seed)
        self.precision = PRECISIONS[precision]
        self.src = torch.from_numpy(s).to(device)
        self.rcv = torch.from_numpy(r).to(device)
        self.n_src, self.n_rcv = s.shape[0], r.shape[0]
        self.out = torch.empty((self.n_src, self.n_rcv, room.n_samples), dtype=torch.float32, device=device)
        nbytes = diffuse_workspace_size(room, t_diff, t60, self.n_src, self.n_rcv, precision)
        self.ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
        self.ws_bytes = nbytes

    def run(self, stream=None, ev_start=None, ev_stop=None):
        """Launch on ``stream`` (default: torch's current stream); ``ev_start``/``ev_stop``
        are optional raw hipEvent_t handles recorded around the tap kernel of the ISM part."""
        st = stream if stream is not None else self.torch.cuda.current_stream()
        _check(lib().ism_simulate_diffuse_timed(ctypes.byref(self._room_c), self.t_diff, self.t60, self.seed,
                                                self.src.data_ptr(), self.n_src, self.rcv.data_ptr(), self.n_rcv,
                                                self.precision, self.out.data_ptr(), self.ws.data_ptr(),
                                                self.ws_bytes, st.cuda_stream, ev_start, ev_stop),
               "ism_simulate_diffuse_timed")
        return self.out


def simulate_diffuse(room: Room, src, rcv, t_diff: float, t60: float, seed: int = 0, precision: str = "fp32",
                     device: str = "cuda"):
    """RIRs [n_src, n_rcv, nS] with the ISM up to t_diff and the diffuse tail after it."""
    return DiffuseSimulator(room, src, rcv, t_diff, t60, seed, precision, device).run()


def simulate_diffuse_polar(room: Room, src, rcv, orient, t_diff: float, t60: float, seed: int = 0,
                           pattern="cardioid", precision: str = "fp32", device: str = "cuda", check: bool = True):
    """``simulate_diffuse`` with directional receivers (``orient`` and
    ``pattern`` as for ``simulate_polar``): directional ISM part, tail at the
    level of that part."""
    import torch

    a = PATTERNS[pattern] if isinstance(pattern, str) else float(pattern)
    s, r, o = _host_pos(src), _host_pos(rcv), _host_pos(orient)
    if o.shape != r.shape:
        raise ValueError(f"orient must be [n_rcv, 3] = {r.shape}, got {o.shape}")
    if check:
        check_positions(room, s, r)
    rc = room._c()
    nbytes = diffuse_workspace_size(room, t_diff, t60, s.shape[0], r.shape[0], precision)
    src_d, rcv_d, o_d = (torch.from_numpy(x).to(device) for x in (s, r, o))
    out = torch.empty((s.shape[0], r.shape[0], room.n_samples), dtype=torch.float32, device=device)
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
    st = torch.cuda.current_stream()
    _check(lib().ism_simulate_diffuse_polar(ctypes.byref(rc), float(t_diff), float(t60), int(seed), src_d.data_ptr(),
                                            s.shape[0], rcv_d.data_ptr(), r.shape[0], o_d.data_ptr(), a,
                                            PRECISIONS[precision], out.data_ptr(), ws.data_ptr(), nbytes,
                                            st.cuda_stream), "ism_simulate_diffuse_polar")
    return out


FILTER_METHODS = {"auto": 0, "direct": 1, "fft": 2}


def filter_workspace_size(n_x: int, n_pos: int, n_mic: int, n_rir: int, method: str = "auto") -> int:
    out = ctypes.c_size_t()
    _check(lib().ism_filter_workspace_size(int(n_x), int(n_pos), int(n_mic), int(n_rir), FILTER_METHODS[method],
                                           ctypes.byref(out)), "ism_filter_workspace_size")
    return out.value


def filter_trajectory(x, rirs, stream=None, method: str = "auto", ws=None):
    """Moving source (Sec. 3.4): x [n_x] float32 device tensor, rirs [n_pos, n_mic,
    n_rir] float32 device tensor (ism_simulate output with the trajectory points as
    sources). Returns y [n_mic, n_x + n_rir - 1] on the same device.
    method: "direct" (direct sum), "fft" (partitioned FFT convolution) or
    "auto"; ws: optional uint8 device tensor of at least filter_workspace_size bytes."""
    import torch

    if x.dtype != torch.float32 or rirs.dtype != torch.float32 or x.dim() != 1 or rirs.dim() != 3:
        raise IsmError(ISM_E_INVALID_ARG, "filter_trajectory")
    x = x.contiguous()
    rirs = rirs.contiguous()
    n_pos, n_mic, n_rir = rirs.shape
    nbytes = filter_workspace_size(x.shape[0], n_pos, n_mic, n_rir, method)
    if nbytes and (ws is None or ws.numel() < nbytes):
        ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    y = torch.empty((n_mic, x.shape[0] + n_rir - 1), dtype=torch.float32, device=x.device)
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().ism_filter_trajectory_ex(x.data_ptr(), int(x.shape[0]), rirs.data_ptr(), int(n_pos), int(n_mic),
                                          int(n_rir), FILTER_METHODS[method], y.data_ptr(),
                                          ws.data_ptr() if nbytes else None, nbytes, st.cuda_stream),
           "ism_filter_trajectory_ex")
    return y


def room_for(w) -> Room:
    """Room of a ``workloads.Workload`` built with this library's helpers: Sabine
    beta for the workload's T60 (times its per-wall jitter, capped at 0.999) and
    the lattice that keeps every image closer than c * T_max (c * t_diff for a
    workload with a diffuse tail, whose ISM part ends there)."""
    beta = beta_from_t60(w.room, w.t60)
    if w.beta_jitter is not None:
        beta = np.minimum(beta * np.asarray(w.beta_jitter), 0.999)
    n = n_img_for_time(w.room, w.c, w.t_diff if getattr(w, "t_diff", 0.0) > 0.0 else w.t_max)
    return Room(list(map(float, w.room)), list(map(float, beta)), n, w.c, w.fs, w.t_max, w.t_w)


class BatchSimulator:
    """Many rooms in one prepared batch (``ism_batch_prepare`` once, ``ism_batch_run`` per call).

    ``jobs`` is a list of (Room, src, rcv), or (Room, src, rcv, orient, pattern)
    for directional receivers (as for ``simulate_polar``); outputs are
    ``self.outs[i]`` with shape [n_src, n_rcv, nS] on ``device``.
    """

    def __init__(self, jobs, precision: str = "fp32", device: str = "cuda", check: bool = True, stream=None,
                 schedule: Schedule = None):
        import torch

        self.torch = torch
        self.precision = PRECISIONS[precision]
        self._keep = []
        self.outs = []
        arr = (_Job * len(jobs))()
        host = [(_host_pos(j[1]), _host_pos(j[2])) for j in jobs]
        if check:
            for j, (s, r) in zip(jobs, host):
                check_positions(j[0], s, r)
        # all positions of the batch in one device buffer (one host-to-device copy)
        pos = torch.from_numpy(np.concatenate([a for sr in host for a in sr], axis=0)).to(device)
        self._keep.append(pos)
        row = 0
        for i, (job, (s, r)) in enumerate(zip(jobs, host)):
            room = job[0]
            out = torch.empty((s.shape[0], r.shape[0], room.n_samples), dtype=torch.float32, device=device)
            if len(job) == 5:
                o = _host_pos(job[3])
                if o.shape != r.shape:
                    raise ValueError(f"orient must be [n_rcv, 3] = {r.shape}, got {o.shape}")
                o_d = torch.from_numpy(o).to(device)
                self._keep.append(o_d)
                arr[i].orient = o_d.data_ptr()
                arr[i].pattern = PATTERNS[job[4]] if isinstance(job[4], str) else float(job[4])
            self.outs.append(out)
            arr[i].room = room._c()
            arr[i].src, arr[i].n_src = pos[row:].data_ptr(), s.shape[0]
            row += s.shape[0]
            arr[i].rcv, arr[i].n_rcv = pos[row:].data_ptr(), r.shape[0]
            row += r.shape[0]
            arr[i].out = out.data_ptr()
        self.n_rirs = sum(int(o.shape[0] * o.shape[1]) for o in self.outs)
        nbytes = ctypes.c_size_t()
        _check(lib().ism_batch_workspace_size_ex(arr, len(jobs), self.precision, _sched(schedule),
                                                 ctypes.byref(nbytes)), "ism_batch_workspace_size_ex")
        self.ws = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=device)
        self.ws_bytes = nbytes.value
        self.batch = _Batch()
        st = stream if stream is not None else torch.cuda.current_stream()
        _check(lib().ism_batch_prepare_ex(arr, len(jobs), self.precision, _sched(schedule), self.ws.data_ptr(),
                                          self.ws_bytes, st.cuda_stream, ctypes.byref(self.batch)),
               "ism_batch_prepare_ex")

    def run(self, stream=None, ev_start=None, ev_stop=None):
        st = stream if stream is not None else self.torch.cuda.current_stream()
        if ev_start is None and ev_stop is None:
            _check(lib().ism_batch_run(ctypes.byref(self.batch), st.cuda_stream), "ism_batch_run")
        else:
            _check(lib().ism_batch_run_timed(ctypes.byref(self.batch), st.cuda_stream, ev_start, ev_stop),
                   "ism_batch_run_timed")
        return self.outs


def batch_workspace_size(jobs, precision: str = "fp32", schedule: Schedule = None) -> int:
    """``ism_batch_workspace_size_ex`` of jobs given as (Room, n_src, n_rcv) or
    (Room, n_src, n_rcv, directional) tuples (no positions are needed to size it)."""
    arr = (_Job * len(jobs))()
    dummy = ctypes.c_float(0.0)
    for i, j in enumerate(jobs):
        arr[i].room = j[0]._c()
        arr[i].n_src, arr[i].n_rcv = int(j[1]), int(j[2])
        arr[i].src = arr[i].rcv = arr[i].out = ctypes.addressof(dummy)
        if len(j) > 3 and j[3]:
            arr[i].orient, arr[i].pattern = ctypes.addressof(dummy), 1.0
    out = ctypes.c_size_t()
    _check(lib().ism_batch_workspace_size_ex(arr, len(jobs), PRECISIONS[precision], _sched(schedule),
                                             ctypes.byref(out)), "ism_batch_workspace_size_ex")
    return out.value


def simulate_batch(jobs, precision: str = "fp32", outs=None, device: str = "cuda"):
    """``ism_simulate_batch``: jobs as (Room, src, rcv) or (Room, src, rcv, orient,
    pattern) with HOST positions, checked by the library before any launch and
    uploaded with the batch tables. ``outs`` (optional): float32 device tensors
    [n_src, n_rcv, nS] per job to overwrite. Returns the list of outputs."""
    import torch

    arr = (_Job * len(jobs))()
    keep = []
    if outs is None:
        outs = []
        for j in jobs:
            s, r = _host_pos(j[1]), _host_pos(j[2])
            outs.append(torch.empty((s.shape[0], r.shape[0], j[0].n_samples), dtype=torch.float32, device=device))
    for i, j in enumerate(jobs):
        s, r = _host_pos(j[1]), _host_pos(j[2])
        keep += [s, r]
        arr[i].room = j[0]._c()
        arr[i].src, arr[i].n_src = s.ctypes.data, s.shape[0]
        arr[i].rcv, arr[i].n_rcv = r.ctypes.data, r.shape[0]
        arr[i].out = outs[i].data_ptr()
        if len(j) == 5:
            o = _host_pos(j[3])
            keep.append(o)
            arr[i].orient = o.ctypes.data
            arr[i].pattern = PATTERNS[j[4]] if isinstance(j[4], str) else float(j[4])
    nbytes = ctypes.c_size_t()
    _check(lib().ism_batch_workspace_size(arr, len(jobs), PRECISIONS[precision], ctypes.byref(nbytes)),
           "ism_batch_workspace_size")
    ws = torch.empty(max(nbytes.value, 1), dtype=torch.uint8, device=outs[0].device)
    st = torch.cuda.current_stream(outs[0].device)
    _check(lib().ism_simulate_batch(arr, len(jobs), PRECISIONS[precision], ws.data_ptr(), nbytes.value,
                                    st.cuda_stream), "ism_simulate_batch")
    return outs
