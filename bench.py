#!/usr/bin/env python3
"""Throughput benchmark of the ISM hot path on one MI355X.

Default run: the batch of 1024 independent rooms (sides U(3, 10) m, T60
U(0.2, 1.0) s, per-wall jittered Sabine beta, 1-8 receivers, 16 kHz, T_w 4 ms),
all RIRs in one prepared batch. One step = one ``ism_batch_run`` (axis tables,
shell enumeration + windowed-sinc accumulation, ordered completion of the
tiles) with positions, outputs and workspace already resident in HBM.

The JSON line carries:
  value / rirs_per_s   FP32 taps: image-source sinc taps/s (G/s) and RIRs/s;
  roofline             the tap-accumulation kernel, timed live with HIP events
                       around each of its launches, against the FP32 vector peak;
  fp16                 the same batch with packed-FP16 taps: rate, speedup over
                       FP32 on this GPU, max error against the FP64 oracle;
  serving              a Poisson stream through the continuous-batching loop:
                       RIRs/s with p50/p99 latency;
  cpu_baseline         the FP64 oracle on a bounded sample of the same batch, on
                       all usable host cores and on one core.
Other workloads (``--workload``) print the single-leg line of that workload.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "image-source sinc taps/s (G/s) + RIRs/s, FP32 vs FP16; p50/p99 serving latency"
# frozen accounting of one windowed-sinc tap: 1 sub, 1 mul, 1 mul, 5 FMA,
# 1 mul, 1 reciprocal, 2 mul, 1 add, an FMA counting 2
FLOP_PER_TAP = 18
FP32_VECTOR_PEAK = 157.3   # TFLOP/s, MI355X FP32 vector peak (256 CUs x 2.4 GHz x 256 FLOP/clk)
# Host threads the oracle may use: the host CPU share of one GPU on a shared node.
CPU_THREADS_MAX = 16
# rocprofv3 summaries holding the calibrated HBM traffic of the timed kernel,
# valid while the library bench.py loads hashes to the value recorded beside
# it (compiling is deterministic: edits that leave the code unchanged keep it)
TRAFFIC_PROFILES = {"room_32_receivers": "profiles/accumulate_kernel_room_4x5x3_32rcv.md",
                    "batch_rooms": "profiles/accumulate_batch_kernel_1024_rooms.md",
                    "moving_source_10s": "profiles/filter_moving_source_16k_8000_taps.md",
                    "moving_source_48k_96000": "profiles/filter_moving_source_48k_96000_taps.md"}
HBM_PEAK = 8000.0  # GB/s, MI355X HBM3E


class _HipEvents:
    """hipEvent_t handles from the HIP runtime torch already loaded."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        ev = ctypes.c_void_p()
        if self.hip.hipEventCreate(ctypes.byref(ev)) != 0:
            raise RuntimeError("hipEventCreate failed")
        return ev.value

    def elapsed_ms(self, a, b) -> float:
        ms = ctypes.c_float()
        if self.hip.hipEventElapsedTime(ctypes.byref(ms), ctypes.c_void_p(a), ctypes.c_void_p(b)) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return ms.value

    def destroy(self, ev):
        self.hip.hipEventDestroy(ctypes.c_void_p(ev))


def ism_lib_path() -> str:
    from paper_1810_11359_amd import ism

    return ism.LIB_PATH


def library_sha256() -> str:
    """sha256 of the libism.so that the package loads (kernels, planner and
    tuning table compiled in)."""
    from paper_1810_11359_amd import ism

    with open(ism.LIB_PATH, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(workload: str, precision: str, key: str = "traffic_bytes_per_launch"):
    """HBM bytes per launch of the timed kernel (or per call, for the keys of a
    whole call) from the committed counter summary (FETCH_SIZE + WRITE_SIZE,
    copy-calibrated), or None when there is none for this workload or the
    library changed since it was taken."""
    rel = TRAFFIC_PROFILES.get(workload) if precision == "fp32" else None
    if rel is None or not os.path.exists(os.path.join(ROOT, rel)):
        return None
    vals = {}
    with open(os.path.join(ROOT, rel)) as fh:
        for line in fh:
            if ":" in line and line.split(":", 1)[0] in (key, "library_sha256"):
                k, v = line.split(":", 1)
                vals[k] = v.strip()
    if key not in vals or not os.path.exists(ism_lib_path()):
        return None
    if vals.get("library_sha256") != library_sha256():
        return None
    return int(vals[key])


def host_cpu():
    """(usable threads for the oracle, nproc, CPU model name) of this host."""
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return max(1, min(usable, CPU_THREADS_MAX)), os.cpu_count() or 1, model


def _oracle_args(orc, w):
    beta = orc.beta_from_t60(w.room, w.t60)
    if w.beta_jitter is not None:
        beta = np.minimum(beta * np.asarray(w.beta_jitter), 0.999)
    n = orc.n_img_for_time(w.room, w.c, w.t_max)
    return (w.room, beta, n, w.c, w.fs, w.t_max, w.t_w)


def _sample_jobs(ws, n_rir: int):
    """The first n_rir RIRs of the workloads: [(workload, receivers)] (one source each)."""
    jobs, left = [], n_rir
    for w in ws:
        if left <= 0:
            break
        k = min(left, w.rcv.shape[0])
        jobs.append((w, w.rcv[:k]))
        left -= k
    return jobs


def _max_err(jobs, refs, outs):
    """Largest per-RIR max|h_gpu - h_oracle| / max|h_oracle| over the sample."""
    err = 0.0
    for (w, r), ref, got in zip(jobs, refs, outs):
        g = np.asarray(got, dtype=np.float64)[:, :r.shape[0], :]
        peak = np.max(np.abs(ref), axis=-1)
        err = max(err, float(np.max(np.max(np.abs(g - ref), axis=-1) / peak)))
    return err


def cpu_baseline(ws, n_rcv_sample: int, gpu_outs=None, lut_q: int = 0, one_core_taps: float = 1.5e8):
    """FP64 oracle on a bounded sample: the first ``n_rcv_sample`` RIRs of the
    workload(s), on all usable host threads (at most CPU_THREADS_MAX), then the
    first RIRs of that sample holding at least ``one_core_taps`` taps on one
    thread. ``gpu_outs``: {label: [host arrays [n_src, n_rcv, nS] per workload]};
    for each label it reports the largest max|h_gpu - h_oracle| / max|h_oracle|
    over the sample. lut_q > 0: the oracle's table taps (Eq. (9))."""
    from oracle import oracle as orc

    orc.build()
    threads, nproc, model = host_cpu()
    jobs = _sample_jobs(ws, n_rcv_sample)
    n_rir = sum(r.shape[0] for _, r in jobs)
    threads = min(threads, n_rir)
    taps_per = [orc.count_taps(*_oracle_args(orc, w), w.src, r) for w, r in jobs]
    taps = sum(taps_per)
    # every RIR of the sample on its own oracle thread, `threads` at a time
    # (the oracle's C code runs outside the interpreter lock)
    from concurrent.futures import ThreadPoolExecutor

    tasks = [(j, i) for j, (w, r) in enumerate(jobs) for i in range(r.shape[0])]

    def one(t):
        w, r = jobs[t[0]]
        return orc.rir(*_oracle_args(orc, w), w.src, r[t[1]:t[1] + 1], n_threads=1, lut_q=lut_q)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as pool:
        parts = list(pool.map(one, tasks))
    dt = time.perf_counter() - t0
    refs = [np.concatenate([parts[k] for k, t in enumerate(tasks) if t[0] == j], axis=1) for j in range(len(jobs))]
    # one core: whole RIRs from the front of the sample
    one_jobs, one_taps = [], 0
    for (w, r) in jobs:
        for i in range(r.shape[0]):
            if one_taps >= one_core_taps:
                break
            t_i = orc.count_taps(*_oracle_args(orc, w), w.src, r[i:i + 1])
            one_jobs.append((w, r[i:i + 1]))
            one_taps += t_i
    t1 = time.perf_counter()
    for w, r in one_jobs:
        orc.rir(*_oracle_args(orc, w), w.src, r, n_threads=1, lut_q=lut_q)
    dt1 = time.perf_counter() - t1
    out = {"value": taps / dt / 1e9, "unit": "G taps/s", "cores": threads, "kind": "oracle",
           "sample": f"first {n_rir} full RIRs of the workload ({len(jobs)} room(s); {taps} taps, {dt:.2f} s wall "
                     f"on {threads} threads); one core: first {len(one_jobs)} of them ({one_taps} taps, {dt1:.2f} s)",
           "rirs_per_s": n_rir / dt, "value_1core": one_taps / dt1 / 1e9, "rirs_per_s_1core": len(one_jobs) / dt1,
           "nproc": nproc, "cpu_model": model}
    errs = {}
    for label, outs in (gpu_outs or {}).items():
        errs[label] = _max_err(jobs, refs, outs)
    return out, errs


# Untimed seconds of back-to-back steps after the warm-up steps: the GPU's
# clocks take longer than a few short steps to reach their level under load
# (the 32-receiver room measured 0.53 ms per kernel after 3 warm-up steps,
# 0.45 ms after a second of steps), so short steps are timed only from then.
PREWARM_S = 1.0


def _prewarm(step, seconds: float) -> None:
    """Runs ``step`` back to back (synchronising after each) for ``seconds``."""
    import torch

    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        step()
        torch.cuda.synchronize()


def _time_runs(sim, steps: int, warmup: int, prewarm_s: float = PREWARM_S):
    """Warm-up steps, ``prewarm_s`` seconds of untimed steps, then ``steps``
    timed runs: (ms per whole step, per-run kernel ms list)."""
    import torch

    hip = _HipEvents()
    ev_a = [hip.create() for _ in range(steps)]
    ev_b = [hip.create() for _ in range(steps)]
    for _ in range(warmup):
        sim.run()
    torch.cuda.synchronize()
    _prewarm(sim.run, prewarm_s)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps):
        sim.run(ev_start=ev_a[i], ev_stop=ev_b[i])
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    kern_ms = [hip.elapsed_ms(a, b) for a, b in zip(ev_a, ev_b)]
    for ev in ev_a + ev_b:
        hip.destroy(ev)
    return ms_total / steps, kern_ms


def _feasible(ism):
    def feasible(room, t60):
        try:
            ism.beta_from_t60(room, t60)
            return True
        except ism.IsmError:
            return False

    return feasible


def serving_leg(rate: float, n_jobs: int, count_taps: bool = False, n_slots: int = 4, budget: int = 64 << 30):
    """Continuous-batching serving of a Poisson stream (mixed rooms, 16/48 kHz,
    static arrays and moving-source trajectories): RIRs/s with p50/p99 latency."""
    import torch

    from paper_1810_11359_amd import ism, workloads
    from paper_1810_11359_amd.serving import GpuExecutor, Job, Scheduler, replay

    reqs = workloads.serving_stream(rate=rate, n_jobs=n_jobs, seed=0, feasible=_feasible(ism))
    jobs = [Job(i, ism.room_for(r.workload), r.workload.src, r.workload.rcv, r.arrival) for i, r in enumerate(reqs)]
    # exact tap counts cost host time proportional to the images of every job
    taps = sum(ism.count_taps(j.room, j.src, j.rcv) for j in jobs) if count_taps else None
    # warm-up: load every kernel variant once
    warm = [Job(-1, j.room, j.src[:1], j.rcv[:1], 0.0) for j in jobs[:8]]
    replay(Scheduler(GpuExecutor(2), budget_bytes=8 << 30, n_slots=2), warm)
    torch.cuda.synchronize()
    sch = Scheduler(GpuExecutor(n_slots), budget_bytes=budget, n_slots=n_slots, max_batch_jobs=256)
    st = replay(sch, jobs)
    torch.cuda.synchronize()
    res = {"workload": f"serving_poisson_{rate:g}_jobs_per_s", "offered_jobs_per_s": rate, "n_jobs": len(jobs),
           "slots": n_slots, "budget_bytes": budget, "warmup_jobs": len(warm)}
    res.update(st.as_dict())
    if taps is not None:
        res["taps"] = int(taps)
        res["taps_per_s"] = taps / st.makespan_s
    return res


def serve(args) -> int:
    """Serving mode (--rate): one JSON line with the serving leg as the headline."""
    s = serving_leg(args.rate, args.jobs, args.count_taps)
    out = {"metric": METRIC, "value": s["rirs_per_s"], "unit": "RIRs/s", "n_gpus": 1, "steps": s["n_jobs"],
           "warmup": s["warmup_jobs"], "ms_per_step": s["makespan_s"] * 1e3 / s["n_jobs"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": s["workload"], "n_jobs": s["n_jobs"], "n_rirs": s["n_rirs"], "slots": s["slots"],
                      "budget_bytes": s["budget_bytes"], "parallelism": "single GPU"},
           "serving": s}
    print(json.dumps(out), flush=True)
    return 0


# Moving-source workloads: (room [m], T60 = T_max [s], fs [Hz], T_w [s], trajectory end points)
MOVING_SOURCE = {
    "moving_source_10s": ([4.0, 5.0, 3.0], 0.5, 16000.0, 0.004, ([0.8, 0.8, 1.6], [3.2, 4.2, 1.6])),
    "moving_source_48k_96000": ([6.0, 9.0, 3.5], 2.0, 48000.0, 0.002, ([1.0, 1.0, 1.6], [5.0, 8.0, 1.6])),
}


def bench_moving_source(args) -> int:
    """Moving-source filtering (ism_filter_trajectory): a 10 s signal through
    the RIRs of 100 trajectory points to an 8-mic array (5 cm radius): a
    4 x 5 x 3 m room at T60 0.5 s and 16 kHz (RIRs of 8000 samples), or a
    6 x 9 x 3.5 m room at T60 2 s and 48 kHz (RIRs of 96 000 samples). The
    RIRs are computed once by ism_simulate outside the timed region (their
    time is reported beside). One step = one filter call; value in G MAC/s
    (n_x x n_rir x n_mic multiply-adds), roofline against the FP32 vector peak
    at 2 FLOP per multiply-add."""
    import torch

    from paper_1810_11359_amd import ism

    L, t60, fs, t_w, (p0, p1) = MOVING_SOURCE[args.workload]
    room = ism.Room(L, list(ism.beta_from_t60(L, t60)), ism.n_img_for_time(L, 343.0, t60), 343.0, fs, t60, t_w)
    rng = np.random.default_rng(0)
    pts = np.linspace(p0, p1, 100).astype(np.float32)
    ctr = np.array([L[0] / 2, L[1] / 2, 1.2])
    mics = (ctr + 0.05 * np.stack([np.cos(np.arange(8) * np.pi / 4), np.sin(np.arange(8) * np.pi / 4),
                                   np.zeros(8)], 1))
    sim = ism.Simulator(room, pts, mics.astype(np.float32))
    sim.run()
    torch.cuda.synchronize()
    t_sim0 = time.perf_counter()
    rirs = sim.run()
    torch.cuda.synchronize()
    sim_ms = (time.perf_counter() - t_sim0) * 1e3
    x = torch.from_numpy(rng.standard_normal(int(10 * fs)).astype(np.float32)).cuda()
    n_pos, n_mic, n_rir = rirs.shape
    macs = x.shape[0] * n_rir * n_mic
    method = args.filter_method
    resolved = "fft" if ism.filter_workspace_size(x.shape[0], n_pos, n_mic, n_rir, method) > 0 else "direct"
    ws = torch.empty(max(1, ism.filter_workspace_size(x.shape[0], n_pos, n_mic, n_rir, method)), dtype=torch.uint8,
                     device=x.device)
    for _ in range(args.warmup):
        ism.filter_trajectory(x, rirs, method=method, ws=ws)
    torch.cuda.synchronize()
    _prewarm(lambda: ism.filter_trajectory(x, rirs, method=method, ws=ws), args.prewarm_s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        ism.filter_trajectory(x, rirs, method=method, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    achieved = 2.0 * macs / (ms_step / 1e3) / 1e12
    # value: the direct sum's multiply-adds per second of filtering (the FFT path
    # does far fewer operations for the same output; its rate in these units is
    # an equivalent rate). Roofline: the direct sum against the FP32 vector
    # peak (2 FLOP per multiply-add); the FFT path against HBM with the
    # filter's algorithmic bytes (RIRs and signal read once, output written
    # once) over the whole call
    alg_bytes = 4 * (n_pos * n_mic * n_rir + int(x.shape[0]) + n_mic * (int(x.shape[0]) + n_rir - 1))
    if resolved == "fft":
        gbs = alg_bytes / (ms_step / 1e3) / 1e9
        roofline = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK, "unit": "GB/s", "frac": gbs / HBM_PEAK,
                    "traffic": measured_traffic(args.workload, "fp32", "traffic_bytes_per_call_fft"),
                    "traffic_unit": "B per call, all kernels (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    "kernel": "partitioned FFT path (whole call)", "kernel_ms_mean": ms_step,
                    "algorithmic_bytes": alg_bytes}
    else:
        roofline = {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK, "unit": "TFLOP/s",
                    "frac": achieved / FP32_VECTOR_PEAK,
                    "traffic": measured_traffic(args.workload, "fp32", "traffic_bytes_per_launch_direct"),
                    "traffic_unit": "B per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                    "kernel": "filter_kernel (whole call)", "kernel_ms_mean": ms_step, "flop_per_mac": 2,
                    "algorithmic_bytes": alg_bytes}
    out = {"metric": "moving-source filter multiply-adds/s (G/s)", "value": macs / (ms_step / 1e3) / 1e9,
           "unit": "G MAC/s (direct-sum equivalent)", "filter_method": resolved,
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "prewarm_s": args.prewarm_s, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": f"{args.workload}_{fs / 1000:g}k_100pts_8mics_{n_rir}_taps",
                      "n_x": int(x.shape[0]), "n_pos": n_pos, "n_mic": n_mic, "n_rir": n_rir, "macs_per_step": macs,
                      "parallelism": "single GPU"},
           "simulate_rirs_ms": sim_ms,
           "wall_s_timed": time.perf_counter() - wall0,
           "roofline": roofline}
    print(json.dumps(out), flush=True)
    return 0


def calibrate_hbm(mib: int = 256) -> int:
    """A plain device-to-device copy of known size (3 x ``mib`` MiB), run under
    the rocprofv3 FETCH_SIZE / WRITE_SIZE passes to scale those counters."""
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_hbm": {"mib_per_copy": mib, "copies": 3}}), flush=True)
    return 0


def _roofline(taps: int, kern_ms, workload: str, precision: str, kernel: str):
    kmean = float(np.mean(kern_ms))
    achieved = FLOP_PER_TAP * taps / (kmean / 1e3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK, "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK, "traffic": measured_traffic(workload, precision),
            "traffic_unit": "B per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": kernel, "kernel_ms_mean": kmean, "kernel_ms_p50": float(np.median(kern_ms)),
            "flop_per_tap": FLOP_PER_TAP}


def bench_batch(args) -> int:
    """The default run: the 1024-room batch in FP32 (headline), the same batch in
    packed FP16, a serving leg and the oracle baseline, in one JSON line."""
    import torch

    from paper_1810_11359_amd import ism, workloads

    ws = workloads.batch_rooms(1024, seed=0, feasible=_feasible(ism))
    rooms = [ism.room_for(w) for w in ws]
    jobs = [(r, w.src, w.rcv) for r, w in zip(rooms, ws)]
    taps = sum(ism.count_taps(r, w.src, w.rcv) for r, w in zip(rooms, ws))
    sample = _sample_jobs(ws, args.cpu_sample)
    n_rooms_sample = len(sample)

    legs = {}
    precisions = [args.precision] + (["fp16"] if args.precision == "fp32" and not args.no_fp16 else [])
    for prec in precisions:
        sim = ism.BatchSimulator(jobs, precision=prec)
        ms_step, kern_ms = _time_runs(sim, args.steps, args.warmup, args.prewarm_s)
        legs[prec] = {"ms_per_step": ms_step, "kern_ms": kern_ms, "n_rir": sim.n_rirs,
                      "outs": [o.cpu().numpy() for o in sim.outs[:n_rooms_sample]]}
        del sim
        torch.cuda.empty_cache()

    head = legs[args.precision]
    n_rir = head["n_rir"]
    config = {"workload": f"batch_1024_rooms_{n_rir}_rirs", "n_rooms": len(ws), "n_rirs": n_rir, "fs": 16000.0,
              "t_w_s": 0.004, "room_m": "U(3,10)^3", "t60_s": "U(0.2,1.0)", "taps_per_step": int(taps),
              "parallelism": "single GPU"}
    ms_step = head["ms_per_step"]
    out = {"metric": METRIC, "value": taps / (ms_step / 1e3) / 1e9, "unit": "G taps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "prewarm_s": args.prewarm_s, "ms_per_step": ms_step,
           "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic", "config": config,
           "rirs_per_s": n_rir / (ms_step / 1e3),
           "roofline": _roofline(taps, head["kern_ms"], "batch_rooms", args.precision, "accumulate_batch_kernel")}
    if "fp16" in legs and args.precision != "fp16":
        h = legs["fp16"]
        kmean = float(np.mean(h["kern_ms"]))
        out["fp16"] = {"value": taps / (h["ms_per_step"] / 1e3) / 1e9, "unit": "G taps/s",
                       "ms_per_step": h["ms_per_step"], "rirs_per_s": n_rir / (h["ms_per_step"] / 1e3),
                       "speedup_vs_fp32": ms_step / h["ms_per_step"], "kernel_ms_mean": kmean,
                       "kernel_speedup_vs_fp32": out["roofline"]["kernel_ms_mean"] / kmean,
                       "taps_per_s_over_fp32_peak_at_18_flop": FLOP_PER_TAP * taps / (kmean / 1e3) / 1e12
                       / FP32_VECTOR_PEAK}
    if not args.no_serving:
        out["serving"] = serving_leg(args.serving_rate, args.serving_jobs)
    if not args.no_cpu_baseline:
        base, errs = cpu_baseline(ws, args.cpu_sample, {k: v["outs"] for k, v in legs.items()},
                                  lut_q=16 if args.precision == "lut" else 0)
        out["cpu_baseline"] = base
        out["max_err_vs_oracle"] = errs[args.precision]
        if "fp16" in out:
            out["fp16"]["max_err_vs_oracle"] = errs["fp16"]
    print(json.dumps(out), flush=True)
    return 0


# The full-ISM cases of the paper's Table 4 (1, 16 and 128 RIRs at T60 0.7 s)
# and Table 5 (128 RIRs at T60 0.3, 0.7 and 1.1 s): (T60 [s], RIRs)
PAPER_TABLE_CASES = [(0.7, 1), (0.7, 16), (0.7, 128), (0.3, 128), (1.1, 128)]


def bench_paper_tables(args) -> int:
    """The room of the paper's Tables 4 and 5 (3 x 4 x 2.5 m, 16 kHz and 4 ms
    assumed): one ism_simulate call per case and precision (FP32 and packed
    FP16 taps), timed as the other single-room workloads. One JSON line with a
    row per case; value = RIRs/s of the 128-RIR FP32 case at T60 0.7 s."""
    from paper_1810_11359_amd import ism, workloads

    rows = []
    for t60, n_rcv in PAPER_TABLE_CASES:
        w = workloads.paper_table_room(t60, n_rcv, 0)
        room = ism.room_for(w)
        taps = ism.count_taps(room, w.src, w.rcv)
        row = {"t60_s": t60, "n_rirs": n_rcv, "n_samples": room.n_samples, "n_img": list(room.n_img),
               "taps_per_call": int(taps)}
        for prec in ("fp32", "fp16"):
            sim = ism.Simulator(room, w.src, w.rcv, precision=prec)
            ms, kern = _time_runs(sim, args.steps, args.warmup, args.prewarm_s)
            row[prec] = {"ms_per_call": ms, "rirs_per_s": n_rcv / (ms / 1e3), "taps_per_s": taps / (ms / 1e3),
                         "kernel_ms_mean": float(np.mean(kern))}
        rows.append(row)
    head = next(r for r in rows if r["t60_s"] == 0.7 and r["n_rirs"] == 128)
    out = {"metric": "RIRs/s of the paper's full-ISM table cases", "value": head["fp32"]["rirs_per_s"],
           "unit": "RIRs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "prewarm_s": args.prewarm_s,
           "ms_per_step": head["fp32"]["ms_per_call"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": "paper_tables_room_3x4x2.5", "fs": 16000.0, "t_w_s": 0.004,
                      "parallelism": "single GPU"},
           "cases": rows}
    print(json.dumps(out), flush=True)
    return 0


def bench_single(args) -> int:
    """A single-room workload: one ism_simulate (or ism_simulate_diffuse) per step."""
    from paper_1810_11359_amd import ism, workloads

    w = workloads.WORKLOADS[args.workload](0)
    room = ism.room_for(w)
    if w.t_diff > 0.0:
        # ISM part up to t_diff, diffuse tail after it: taps are those of the ISM part
        sim = ism.DiffuseSimulator(room, w.src, w.rcv, w.t_diff, w.t60, seed=0, precision=args.precision)
        ism_room = ism.Room(room.room, room.beta, room.n_img, room.c, room.fs, w.t_diff, room.t_w)
        taps = ism.count_taps(ism_room, w.src, w.rcv)
    else:
        sim = ism.Simulator(room, w.src, w.rcv, precision=args.precision)
        taps = ism.count_taps(room, w.src, w.rcv)
    n_rir = sim.n_src * sim.n_rcv
    config = {"workload": w.name, "room_m": list(map(float, w.room)), "t60_s": w.t60, "fs": w.fs,
              "t_w_s": w.t_w, "n_src": int(sim.n_src), "n_rcv": int(sim.n_rcv), "n_samples": room.n_samples,
              "n_img": list(room.n_img), "taps_per_step": int(taps), "parallelism": "single GPU"}
    if w.t_diff > 0.0:
        config["t_diff_s"] = w.t_diff
    ms_step, kern_ms = _time_runs(sim, args.steps, args.warmup, args.prewarm_s)
    out = {"metric": METRIC, "value": taps / (ms_step / 1e3) / 1e9, "unit": "G taps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "prewarm_s": args.prewarm_s, "ms_per_step": ms_step,
           "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic", "config": config,
           "rirs_per_s": n_rir / (ms_step / 1e3),
           "roofline": _roofline(taps, kern_ms, args.workload, args.precision, "accumulate_kernel")}
    if not args.no_cpu_baseline and w.t_diff == 0.0:
        base, errs = cpu_baseline([w], args.cpu_sample, {args.precision: [sim.out.cpu().numpy()]},
                                  lut_q=16 if args.precision == "lut" else 0)
        out["cpu_baseline"] = base
        out["max_err_vs_oracle"] = errs[args.precision]
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prewarm-s", type=float, default=PREWARM_S,
                    help="untimed seconds of steps after the warm-up steps, so the clocks settle (0: none)")
    ap.add_argument("--workload", default="batch_rooms",
                    choices=["batch_rooms", "room_32_receivers", "single_rir", "large_room_uca",
                             "paper_room_128rir", "paper_room_diffuse_1024rir", "moving_source_10s",
                             "moving_source_48k_96000", "paper_tables"])
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="RIRs the CPU oracle baseline computes (default 64 for the batch, 16 otherwise)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp16", "lut"],
                    help="tap arithmetic (accumulation is FP32 in all): FP32, packed FP16, or FP32 "
                         "interpolation in a table of the windowed sinc")
    ap.add_argument("--no-fp16", action="store_true", help="batch: skip the packed-FP16 leg")
    ap.add_argument("--no-serving", action="store_true", help="batch: skip the serving leg")
    ap.add_argument("--serving-rate", type=float, default=1000.0, help="batch: serving leg offered jobs/s")
    ap.add_argument("--serving-jobs", type=int, default=500, help="batch: serving leg jobs")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serving mode: replay a Poisson stream of mixed RIR jobs at this many jobs/s")
    ap.add_argument("--jobs", type=int, default=2000, help="serving mode: jobs in the stream")
    ap.add_argument("--count-taps", action="store_true", help="serving mode: also count the exact taps (slow)")
    ap.add_argument("--filter-method", default="auto", choices=["auto", "direct", "fft"],
                    help="moving-source workloads: direct sum, partitioned FFT convolution, or auto")
    ap.add_argument("--calibrate-hbm", type=int, default=0, metavar="MIB",
                    help="copy MIB MiB three times and exit (HBM counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the ISM path here does not "
              "shard across GPUs.", file=sys.stderr)
        return 2
    if args.precision == "lut" and args.rate > 0:
        print("the serving loop takes fp32 or fp16 taps, not table taps (--precision lut)", file=sys.stderr)
        return 2
    if args.cpu_sample is None:
        args.cpu_sample = 64 if args.workload == "batch_rooms" else 16
    if args.calibrate_hbm > 0:
        return calibrate_hbm(args.calibrate_hbm)
    if args.rate > 0:
        return serve(args)
    if args.workload in MOVING_SOURCE:
        return bench_moving_source(args)
    if args.workload == "batch_rooms":
        return bench_batch(args)
    if args.workload == "paper_tables":
        return bench_paper_tables(args)
    return bench_single(args)


if __name__ == "__main__":
    sys.exit(main())
