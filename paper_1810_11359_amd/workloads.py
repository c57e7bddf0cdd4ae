"""Seeded synthetic workloads (rooms, reverberation times and positions).

This module only draws inputs; it holds none of the method's arithmetic. The
reflection coefficients (Sabine) and the lattice size are computed by whoever
consumes a workload: the GPU library's helpers on the product side, the
oracle's on the reference side. Positions are float32 so both sides see the
same numbers. Draws use numpy's PCG64 (``default_rng(seed)``).

The paper times synthetic rooms too (a 3 x 4 x 2.5 m room, T60 0.3-1.9 s); these
generators stand in for its workloads with the shapes named below.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


@dataclass
class Workload:
    name: str
    room: np.ndarray          # [3] metres (float64)
    t60: float                # target reverberation time [s]
    src: np.ndarray           # [n_src, 3] float32
    rcv: np.ndarray           # [n_rcv, 3] float32
    c: float = 343.0
    fs: float = 16000.0
    t_max: float = 0.0        # RIR length [s]
    t_w: float = 0.004        # window length [s]
    beta_jitter: Optional[np.ndarray] = None  # [6] multiplicative factors, or None for uniform beta
    t_diff: float = 0.0       # > 0: ISM up to t_diff, diffuse tail after it (Sec. 2.2, Eq. (8))


def _uniform_positions(rng, room, n, margin=0.5) -> np.ndarray:
    lo = np.full(3, margin)
    hi = np.asarray(room) - margin
    return rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)


def single_rir(seed: int = 0) -> Workload:
    """One source and one receiver >= 0.5 m from the walls of a 3 x 4 x 2.5 m room,
    T60 = T_max = 0.3 s, fs = 16 kHz, T_w = 4 ms."""
    rng = np.random.default_rng(seed)
    room = np.array([3.0, 4.0, 2.5])
    src = _uniform_positions(rng, room, 1)
    rcv = _uniform_positions(rng, room, 1)
    return Workload("single_rir_3x4x2.5_t60_0.3", room, 0.3, src, rcv, t_max=0.3)


def room_32_receivers(seed: int = 0) -> Workload:
    """One 4 x 5 x 3 m room, T60 = T_max = 0.7 s, fs = 16 kHz, T_w = 4 ms,
    1 source and 32 receivers (uniform, >= 0.5 m from the walls)."""
    rng = np.random.default_rng(seed)
    room = np.array([4.0, 5.0, 3.0])
    src = _uniform_positions(rng, room, 1)
    rcv = _uniform_positions(rng, room, 32)
    return Workload("room_4x5x3_t60_0.7_32rcv", room, 0.7, src, rcv, t_max=0.7)


def large_room_uca(seed: int = 0) -> Workload:
    """6 x 9 x 3.5 m room, T60 = T_max = 2 s, fs = 48 kHz, T_w = 2 ms, one seeded
    source and a 64-microphone circular array of radius 0.1 m centred at
    (3, 4.5, 1.5) in the horizontal plane."""
    rng = np.random.default_rng(seed)
    room = np.array([6.0, 9.0, 3.5])
    src = _uniform_positions(rng, room, 1)
    ang = 2.0 * np.pi * np.arange(64) / 64.0
    rcv = np.stack([3.0 + 0.1 * np.cos(ang), 4.5 + 0.1 * np.sin(ang), np.full(64, 1.5)], axis=1).astype(np.float32)
    return Workload("room_6x9x3.5_t60_2.0_uca64_48k", room, 2.0, src, rcv, fs=48000.0, t_max=2.0, t_w=0.002)


def batch_rooms(n_rooms: int = 1024, seed: int = 0,
                feasible: Optional[Callable[[np.ndarray, float], bool]] = None) -> List[Workload]:
    """Independent rooms: sides U(3, 10) m, T60 U(0.2, 1.0) s (redrawn from the
    same stream while ``feasible(room, t60)`` is False), per-wall jitter factors
    1 + U(-0.1, 0.1) on the reflection coefficient, 1-8 receivers, fs = 16 kHz,
    T_max = T60, T_w = 4 ms."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_rooms):
        room = rng.uniform(3.0, 10.0, 3)
        t60 = float(rng.uniform(0.2, 1.0))
        while feasible is not None and not feasible(room, t60):
            t60 = float(rng.uniform(0.2, 1.0))
        jitter = 1.0 + rng.uniform(-0.1, 0.1, 6)
        n_rcv = int(rng.integers(1, 9))
        src = _uniform_positions(rng, room, 1)
        rcv = _uniform_positions(rng, room, n_rcv)
        out.append(Workload(f"batch_room_{i}", room, t60, src, rcv, t_max=t60, beta_jitter=jitter))
    return out


def paper_room_128rir(seed: int = 0) -> Workload:
    """The full-ISM case of the paper's Table 4 and Fig. 4: a 3 x 4 x 2.5 m room,
    T60 = T_max = 0.7 s, 128 RIRs (1 source, 128 receivers, uniform >= 0.5 m from
    the walls). The paper does not state fs, T_w or positions: 16 kHz and 4 ms here."""
    rng = np.random.default_rng(seed)
    room = np.array([3.0, 4.0, 2.5])
    return Workload("room_3x4x2.5_t60_0.7_128rcv", room, 0.7, _uniform_positions(rng, room, 1),
                    _uniform_positions(rng, room, 128), t_max=0.7)


def paper_table_room(t60: float, n_rcv: int, seed: int = 0) -> Workload:
    """The full-ISM cases of the paper's Tables 4 and 5: the 3 x 4 x 2.5 m room
    at T60 = T_max = t60 with 1 source and n_rcv receivers (the first n_rcv of
    the 128 positions of paper_room_128rir, so the cases are nested)."""
    w = paper_room_128rir(seed)
    return Workload(f"room_3x4x2.5_t60_{t60:g}_{n_rcv}rcv", w.room, t60, w.src, w.rcv[:n_rcv], t_max=t60)


def paper_room_diffuse_1024rir(seed: int = 0) -> Workload:
    """The diffuse-model case of the paper's Table 4 (1024 RIRs, T60 0.7 s, same
    room): ISM up to the 13 dB attenuation time (T60 13/60, the switch the paper
    compares with in Sec. 5), diffuse tail to T_max = T60. 1 source, 1024 receivers."""
    rng = np.random.default_rng(seed)
    room = np.array([3.0, 4.0, 2.5])
    return Workload("room_3x4x2.5_t60_0.7_1024rcv_diffuse", room, 0.7, _uniform_positions(rng, room, 1),
                    _uniform_positions(rng, room, 1024), t_max=0.7, t_diff=0.7 * 13.0 / 60.0)


WORKLOADS = {
    "single_rir": single_rir,
    "room_32_receivers": room_32_receivers,
    "large_room_uca": large_room_uca,
    "paper_room_128rir": paper_room_128rir,
    "paper_room_diffuse_1024rir": paper_room_diffuse_1024rir,
}


@dataclass
class ServingRequest:
    arrival: float            # seconds from the start of the stream
    workload: Workload


def serving_stream(rate: float, n_jobs: int, seed: int = 0,
                   feasible: Optional[Callable[[np.ndarray, float], bool]] = None) -> List[ServingRequest]:
    """Poisson arrivals at ``rate`` jobs/s. Each job: a room with sides U(3, 10) m,
    T60 U(0.1, 1.5) s (redrawn while ``feasible`` is False), T_max = T60,
    fs 16 kHz (T_w 4 ms) or 48 kHz (T_w 2 ms) with equal probability. 80% of
    jobs are one source with U{1..64} receivers; 20% are a moving source: 100
    positions evenly spaced on a segment between two seeded interior points,
    one receiver."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_jobs):
        t += float(rng.exponential(1.0 / rate))
        room = rng.uniform(3.0, 10.0, 3)
        t60 = float(rng.uniform(0.1, 1.5))
        while feasible is not None and not feasible(room, t60):
            t60 = float(rng.uniform(0.1, 1.5))
        fs, t_w = (16000.0, 0.004) if rng.random() < 0.5 else (48000.0, 0.002)
        if rng.random() < 0.8:
            src = _uniform_positions(rng, room, 1)
            rcv = _uniform_positions(rng, room, int(rng.integers(1, 65)))
            kind = "static"
        else:
            a, b = _uniform_positions(rng, room, 2)
            s = np.linspace(0.0, 1.0, 100)[:, None]
            src = (a[None, :] * (1.0 - s) + b[None, :] * s).astype(np.float32)
            rcv = _uniform_positions(rng, room, 1)
            kind = "trajectory"
        w = Workload(f"serving_{kind}_{i}", room, t60, src, rcv, fs=fs, t_max=t60, t_w=t_w)
        out.append(ServingRequest(t, w))
    return out
