#!/usr/bin/env python3
"""Throughput benchmark of the ISM hot path on one MI355X.

One step = one ``ism_simulate`` call over the whole workload (host planning,
axis tables, shell enumeration + windowed-sinc accumulation, ordered partial
reduction), with positions, output and workspace already resident in HBM.
Prints one JSON line: image-source sinc taps/s (G/s) with RIRs/s, the roofline
of the tap-accumulation kernel (timed live with HIP events around each of its
launches) and the FP64 CPU oracle's rate on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "image-source sinc taps/s (G/s) + RIRs/s, FP32 vs FP16; p50/p99 serving latency"
FLOP_PER_TAP = 18          # frozen accounting of one windowed-sinc tap
FP32_VECTOR_PEAK = 157.3   # TFLOP/s, MI355X FP32 vector peak (256 CUs x 2.4 GHz x 256 FLOP/clk)
# rocprofv3 summaries holding the calibrated HBM traffic of the timed kernel,
# valid while the library bench.py loads hashes to the value recorded beside
# it (the build is deterministic: edits that leave the code unchanged keep it)
TRAFFIC_PROFILES = {"room_32_receivers": "profiles/accumulate_kernel_room_4x5x3_32rcv.md"}


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


def measured_traffic(workload: str, precision: str):
    """HBM bytes per launch of the accumulate kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when there is
    none for this workload or the library changed since it was taken."""
    rel = TRAFFIC_PROFILES.get(workload) if precision == "fp32" else None
    if rel is None or not os.path.exists(os.path.join(ROOT, rel)):
        return None
    vals = {}
    with open(os.path.join(ROOT, rel)) as fh:
        for line in fh:
            if ":" in line and line.split(":", 1)[0] in ("traffic_bytes_per_launch", "library_sha256"):
                k, v = line.split(":", 1)
                vals[k] = v.strip()
    if "traffic_bytes_per_launch" not in vals or not os.path.exists(ism_lib_path()):
        return None
    if vals.get("library_sha256") != library_sha256():
        return None
    return int(vals["traffic_bytes_per_launch"])


def _oracle_args(orc, w):
    beta = orc.beta_from_t60(w.room, w.t60)
    if w.beta_jitter is not None:
        beta = np.minimum(beta * np.asarray(w.beta_jitter), 0.999)
    n = orc.n_img_for_time(w.room, w.c, w.t_max)
    return (w.room, beta, n, w.c, w.fs, w.t_max, w.t_w)


def cpu_baseline(ws, n_rcv_sample: int, gpu_outs=None, lut_q: int = 0):
    """FP64 oracle on a bounded sample: the first ``n_rcv_sample`` receivers of a
    single-room workload, or the first rooms of a batch up to that many RIRs.
    With ``gpu_outs`` (host arrays [n_src, n_rcv, nS] per workload) it also
    reports the largest max|h_gpu - h_oracle| / max|h_oracle| over the sample.
    lut_q > 0: the oracle's table taps (Eq. (9)) at lut_q points per sample."""
    from oracle import oracle as orc

    orc.build()
    jobs, left = [], n_rcv_sample
    for w in ws:
        if left <= 0:
            break
        k = min(left, w.rcv.shape[0])
        jobs.append((w, w.rcv[:k]))
        left -= k
    threads = max(1, min(os.cpu_count() or 1, 16, sum(r.shape[0] for _, r in jobs)))
    taps = sum(orc.count_taps(*_oracle_args(orc, w), w.src, r) for w, r in jobs)
    t0 = time.perf_counter()
    refs = [orc.rir(*_oracle_args(orc, w), w.src, r, n_threads=min(threads, r.shape[0]), lut_q=lut_q)
            for w, r in jobs]
    dt = time.perf_counter() - t0
    n = sum(r.shape[0] for _, r in jobs)
    out = {"value": taps / dt / 1e9, "unit": "G taps/s", "cores": threads, "kind": "oracle",
           "sample": f"{n} full RIRs of the workload ({len(jobs)} room(s); {taps} taps, {dt:.2f} s wall, "
                     f"up to {threads} threads)",
           "rirs_per_s": n / dt}
    if gpu_outs is not None:
        err = 0.0
        for (w, r), ref, got in zip(jobs, refs, gpu_outs):
            g = np.asarray(got, dtype=np.float64)[:, :r.shape[0], :]
            peak = np.max(np.abs(ref), axis=-1)
            err = max(err, float(np.max(np.max(np.abs(g - ref), axis=-1) / peak)))
        out["max_err_vs_oracle"] = err
    return out


def serve(args) -> int:
    """Continuous-batching serving of a Poisson stream; prints RIRs/s with p50/p99 latency."""
    import torch

    from paper_1810_11359_amd import ism, workloads
    from paper_1810_11359_amd.serving import GpuExecutor, Job, Scheduler, replay

    def feasible(room, t60):
        try:
            ism.beta_from_t60(room, t60)
            return True
        except ism.IsmError:
            return False

    reqs = workloads.serving_stream(rate=args.rate, n_jobs=args.jobs, seed=0, feasible=feasible)
    jobs = [Job(i, ism.room_for(r.workload), r.workload.src, r.workload.rcv, r.arrival) for i, r in enumerate(reqs)]
    # exact tap counts cost host time proportional to the images of every job
    taps = sum(ism.count_taps(j.room, j.src, j.rcv) for j in jobs) if args.count_taps else None
    # warm-up: compile/load every kernel variant once
    warm = [Job(-1, j.room, j.src[:1], j.rcv[:1], 0.0) for j in jobs[:8]]
    replay(Scheduler(GpuExecutor(2), budget_bytes=8 << 30, n_slots=2), warm)
    torch.cuda.synchronize()
    n_slots = 4
    sch = Scheduler(GpuExecutor(n_slots), budget_bytes=64 << 30, n_slots=n_slots, max_batch_jobs=256)
    st = replay(sch, jobs)
    torch.cuda.synchronize()
    out = {"metric": METRIC, "value": st.rirs_per_s, "unit": "RIRs/s", "n_gpus": 1, "steps": len(jobs),
           "warmup": len(warm), "ms_per_step": st.makespan_s * 1e3 / len(jobs), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": f"serving_poisson_{args.rate:g}_jobs_per_s", "n_jobs": len(jobs),
                      "n_rirs": st.n_rirs, "taps": None if taps is None else int(taps), "slots": n_slots,
                      "budget_bytes": 64 << 30, "parallelism": "single GPU"},
           "serving": st.as_dict(), "taps_per_s": None if taps is None else taps / st.makespan_s}
    print(json.dumps(out), flush=True)
    return 0


def bench_moving_source(args) -> int:
    """Moving-source filtering (ism_filter_trajectory): a 10 s signal at 16 kHz
    through the RIRs of 100 trajectory points to an 8-mic array in a 4 x 5 x 3 m
    room at T60 0.5 s (RIRs of 8000 samples, computed once by ism_simulate,
    outside the timed region). One step = one filter call; value in G MAC/s
    (n_x x n_rir x n_mic multiply-adds), roofline against the FP32 vector peak
    at 2 FLOP per multiply-add."""
    import torch

    from paper_1810_11359_amd import ism

    L, t60, fs = [4.0, 5.0, 3.0], 0.5, 16000.0
    room = ism.Room(L, list(ism.beta_from_t60(L, t60)), ism.n_img_for_time(L, 343.0, t60), 343.0, fs, t60, 0.004)
    rng = np.random.default_rng(0)
    pts = np.linspace([0.8, 0.8, 1.6], [3.2, 4.2, 1.6], 100).astype(np.float32)
    mics = (np.array([2.0, 2.5, 1.2]) + 0.05 * np.stack([np.cos(np.arange(8) * np.pi / 4),
                                                          np.sin(np.arange(8) * np.pi / 4), np.zeros(8)], 1))
    rirs = ism.simulate(room, pts, mics.astype(np.float32))
    x = torch.from_numpy(rng.standard_normal(int(10 * fs)).astype(np.float32)).cuda()
    n_pos, n_mic, n_rir = rirs.shape
    macs = x.shape[0] * n_rir * n_mic
    for _ in range(args.warmup):
        ism.filter_trajectory(x, rirs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        ism.filter_trajectory(x, rirs)
    e1.record()
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / args.steps
    achieved = 2.0 * macs / (ms_step / 1e3) / 1e12
    out = {"metric": "moving-source filter multiply-adds/s (G/s)", "value": macs / (ms_step / 1e3) / 1e9,
           "unit": "G MAC/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
           "config": {"workload": "moving_source_10s_16k_100pts_8mics", "n_x": int(x.shape[0]), "n_pos": n_pos,
                      "n_mic": n_mic, "n_rir": n_rir, "macs_per_step": macs, "parallelism": "single GPU"},
           "wall_s_timed": time.perf_counter() - wall0,
           "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK, "unit": "TFLOP/s",
                        "frac": achieved / FP32_VECTOR_PEAK, "traffic": None, "kernel": "filter_kernel (whole call)",
                        "kernel_ms_mean": ms_step, "flop_per_mac": 2}}
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="room_32_receivers",
                    choices=["room_32_receivers", "single_rir", "large_room_uca", "batch_rooms",
                             "paper_room_128rir", "paper_room_diffuse_1024rir", "moving_source_10s"])
    ap.add_argument("--cpu-sample", type=int, default=16, help="receivers the CPU oracle baseline computes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp16", "lut"],
                    help="tap arithmetic (accumulation is FP32 in all): FP32, packed FP16, or FP32 "
                         "interpolation in a table of the windowed sinc (single-room workloads)")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serving mode: replay a Poisson stream of mixed RIR jobs at this many jobs/s")
    ap.add_argument("--jobs", type=int, default=2000, help="serving mode: jobs in the stream")
    ap.add_argument("--count-taps", action="store_true", help="serving mode: also count the exact taps (slow)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the ISM path here does not "
              "shard across GPUs.", file=sys.stderr)
        return 2

    if args.precision == "lut" and args.rate > 0:
        print("the serving loop takes fp32 or fp16 taps, not table taps (--precision lut)", file=sys.stderr)
        return 2

    import torch

    from paper_1810_11359_amd import ism, workloads

    if args.rate > 0:
        return serve(args)
    if args.workload == "moving_source_10s":
        return bench_moving_source(args)
    if args.workload == "batch_rooms":
        def feasible(room, t60):
            try:
                ism.beta_from_t60(room, t60)
                return True
            except ism.IsmError:
                return False

        ws = workloads.batch_rooms(1024, seed=0, feasible=feasible)
        rooms = [ism.room_for(w) for w in ws]
        sim = ism.BatchSimulator([(r, w.src, w.rcv) for r, w in zip(rooms, ws)], precision=args.precision)
        n_rir = sim.n_rirs
        taps = sum(ism.count_taps(r, w.src, w.rcv) for r, w in zip(rooms, ws))
        config = {"workload": f"batch_1024_rooms_{n_rir}_rirs", "n_rooms": len(ws), "n_rirs": n_rir, "fs": 16000.0,
                  "t_w_s": 0.004, "room_m": "U(3,10)^3", "t60_s": "U(0.2,1.0)", "taps_per_step": int(taps),
                  "parallelism": "single GPU"}
    else:
        w = workloads.WORKLOADS[args.workload](0)
        ws = [w]
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
    hip = _HipEvents()
    ev_a = [hip.create() for _ in range(args.steps)]
    ev_b = [hip.create() for _ in range(args.steps)]

    for _ in range(args.warmup):
        sim.run()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    e0.record()
    for i in range(args.steps):
        sim.run(ev_start=ev_a[i], ev_stop=ev_b[i])
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = e0.elapsed_time(e1)
    kern_ms = [hip.elapsed_ms(a, b) for a, b in zip(ev_a, ev_b)]
    for ev in ev_a + ev_b:
        hip.destroy(ev)

    ms_step = ms_total / args.steps
    value = taps / (ms_step / 1e3) / 1e9
    kmean = float(np.mean(kern_ms))
    achieved = FLOP_PER_TAP * taps / (kmean / 1e3) / 1e12
    traffic = measured_traffic(args.workload, args.precision)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "G taps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": config,
        "rirs_per_s": n_rir / (ms_step / 1e3),
        "wall_s_timed": wall,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK, "traffic": traffic,
                     "traffic_unit": "B per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "accumulate_kernel" if args.workload != "batch_rooms" else "accumulate_batch_kernel",
                     "kernel_ms_mean": kmean,
                     "kernel_ms_p50": float(np.median(kern_ms)), "flop_per_tap": FLOP_PER_TAP},
    }
    if not args.no_cpu_baseline and all(getattr(x, "t_diff", 0.0) == 0.0 for x in ws):
        res = sim.outs if args.workload == "batch_rooms" else [sim.out]
        gpu_outs = [o.cpu().numpy() for o in res[:args.cpu_sample]]
        out["cpu_baseline"] = cpu_baseline(ws, args.cpu_sample, gpu_outs, lut_q=16 if args.precision == "lut" else 0)
        out["max_err_vs_oracle"] = out["cpu_baseline"].pop("max_err_vs_oracle")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
