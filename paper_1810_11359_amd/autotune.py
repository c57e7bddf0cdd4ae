"""Work-schedule tuner. Run it on the target GPU:

    python -m paper_1810_11359_amd.autotune --out paper_1810_11359_amd/csrc/ism_tuning.h

For every window length W (32, 64, 96, 128 samples), tap precision and RIR
length bucket (up to 8192, 32768 and more samples) it times the
tap-accumulation kernel (HIP events the library records around it) on
representative single-room and batch workloads of that bucket over a grid of
(min_item_taps, balance_items) pairs and keeps the pair with the best
geometric-mean time relative to each workload's fastest pair. Every
candidate of a grid is prepared first and the candidates are timed in
interleaved rounds once the clocks have settled, since neighbouring
candidates differ by less than a box drifts over a minute. For the
persistent batch launches of W = 64 it also picks, on the 1024-room batch, the
workgroups per SIMD of the grid and the largest item of a batch job. It writes
the table header the host planner compiles in; rebuild
the library afterwards. Candidate values reach the library as the call's
explicit schedule (``ism_schedule``).

The kernel's compile-time shape (256-sample tiles, two images per step,
seven waves per SIMD) is not a knob here: 512-sample tiles (five waves per
SIMD) and four images per step were built and timed on the 1024-room batch,
the 32-receiver room, the 64-microphone 48 kHz room and a single RIR, and
were no faster anywhere (the timings are in the design notes).
"""
from __future__ import annotations

import argparse
import ctypes
import math
import os
import sys
from dataclasses import replace

import numpy as np

from . import ism, workloads

MIN_TAPS = (6.0e4, 1.2e5, 2.4e5, 4.8e5)
BALANCE = (24576.0, 49152.0, 98304.0, 196608.0)
NS_BUCKETS = (8192, 32768, 2147483647)   # RIR length buckets (samples), upper bounds
BATCH_WAVES = (4, 5, 6, 7, 8)
BATCH_ITEM_TAPS = (1.2e5, 2.5e5, 5.0e5)


class _Events:
    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def pair(self):
        a, b = ctypes.c_void_p(), ctypes.c_void_p()
        if self.hip.hipEventCreate(ctypes.byref(a)) or self.hip.hipEventCreate(ctypes.byref(b)):
            raise RuntimeError("hipEventCreate failed")
        return a.value, b.value

    def ms(self, a, b) -> float:
        v = ctypes.c_float()
        if self.hip.hipEventElapsedTime(ctypes.byref(v), ctypes.c_void_p(a), ctypes.c_void_p(b)):
            raise RuntimeError("hipEventElapsedTime failed")
        return v.value

    def free(self, *evs):
        for e in evs:
            self.hip.hipEventDestroy(ctypes.c_void_p(e))


def _feasible(room, t60):
    try:
        ism.beta_from_t60(room, t60)
        return True
    except ism.IsmError:
        return False


def _room(L, t_max, fs, t_w, n_rcv, seed=0):
    """A room simulated for t_max seconds; its T60 is t_max, or 0.2 s where
    Sabine's formula cannot reach a shorter one in this room."""
    rng = np.random.default_rng(seed)
    L = np.asarray(L, dtype=float)
    src = rng.uniform(0.5, L - 0.5, (1, 3)).astype(np.float32)
    rcv = rng.uniform(0.5, L - 0.5, (n_rcv, 3)).astype(np.float32)
    t60 = t_max if _feasible(L, t_max) else 0.2
    return workloads.Workload(f"room_{L[0]:g}x{L[1]:g}x{L[2]:g}_t_{t_max:.3g}_{n_rcv}rcv_{fs / 1000:g}k", L, t60, src,
                              rcv, fs=fs, t_max=t_max, t_w=t_w)


def bucket_workloads(wt: int, ns_max: int):
    """Representative workloads of one window length and RIR length bucket:
    (name, [workloads]); several workloads form one batch."""
    fs, t_w = {32: (8000.0, 0.004), 64: (16000.0, 0.004), 96: (48000.0, 0.002), 128: (32000.0, 0.004)}[wt]
    ns_lo = {8192: 0, 32768: 8192}.get(ns_max, 32768)
    if ns_lo > 2.5 * fs:
        return []  # RIRs longer than 2.5 s at this rate: the previous bucket's entry is reused
    # T60 (= T_max) in the middle of the bucket (RIRs up to 2.5 s) and the room it is run in
    t_mid = (ns_lo + min(ns_max, 2.5 * fs)) / 2.0 / fs
    out = [(f"room_t60_{t_mid:.2f}_{fs / 1000:g}k", [_room([4.0, 5.0, 3.0], t_mid, fs, t_w, 16 if t_mid < 1.0 else 4)])]
    if wt == 64:
        rooms = workloads.batch_rooms(256, seed=0, feasible=_feasible)
        sel = [w for w in rooms if ns_lo < w.t_max * fs <= ns_max]
        if sel:
            out.append((f"batch_{len(sel)}_rooms_16k", sel))
    return out


def _interleaved(sims, ev: _Events, reps: int, rounds: int):
    """Mean kernel ms of every simulator, timed in interleaved rounds
    (alternating order) after the clocks have settled."""
    import time

    import torch

    keys = list(sims)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 1.5:
        sims[keys[0]].run()
        torch.cuda.synchronize()
    acc = {k: [] for k in keys}
    for rnd in range(rounds):
        for k in (keys if rnd % 2 == 0 else keys[::-1]):
            evs = [ev.pair() for _ in range(reps)]
            for a, b in evs:
                sims[k].run(ev_start=a, ev_stop=b)
            torch.cuda.synchronize()
            acc[k] += [ev.ms(a, b) for a, b in evs]
            for a, b in evs:
                ev.free(a, b)
    return {k: float(np.mean(v)) for k, v in acc.items()}


def _simulator(ws, precision: str, schedule):
    if len(ws) == 1:
        w = ws[0]
        return ism.Simulator(ism.room_for(w), w.src, w.rcv, precision=precision, schedule=schedule)
    return ism.BatchSimulator([(ism.room_for(w), w.src, w.rcv) for w in ws], precision=precision, schedule=schedule)


def time_item_grid(loads, precision: str, ev: _Events, reps: int, rounds: int = 3):
    """{(min_item_taps, balance_items): [mean kernel ms per workload]} over the
    grid, every pair and workload prepared first and timed in interleaved
    rounds (neighbouring pairs differ by about a percent, the drift of a box
    over a minute)."""
    pairs = [(mt, bal) for mt in MIN_TAPS for bal in BALANCE]
    sims = {(pr, i): _simulator(ws, precision, ism.Schedule(min_item_taps=pr[0], balance_items=pr[1]))
            for pr in pairs for i, (_, ws) in enumerate(loads)}
    t = _interleaved(sims, ev, reps, rounds)
    return {pr: [t[(pr, i)] for i in range(len(loads))] for pr in pairs}


def time_batch_grid(batch, precision: str, ev: _Events, reps: int, rounds: int = 4):
    """Mean accumulate-kernel time (ms) of the batch for every (waves per SIMD,
    item cap) pair, as {pair: [ms]}. The pairs differ by a few tenths of a
    percent, less than the drift of one box over a minute, so every pair is
    prepared first and the pairs are timed in interleaved rounds."""
    jobs = [(ism.room_for(w), w.src, w.rcv) for w in batch]
    pairs = [(k, it) for k in BATCH_WAVES for it in BATCH_ITEM_TAPS]
    sims = {pr: ism.BatchSimulator(jobs, precision=precision, schedule=ism.Schedule(batch_waves=pr[0], item_taps=pr[1]))
            for pr in pairs}
    return {pr: [t] for pr, t in _interleaved(sims, ev, reps, rounds).items()}


def _score(times, n_loads):
    best_each = [min(t[i] for t in times.values()) for i in range(n_loads)]
    return {k: math.exp(np.mean([math.log(t / b) for t, b in zip(v, best_each)])) for k, v in times.items()}


def tune(reps: int = 3, classes=(32, 64, 96, 128), precisions=("fp32", "fp16"), log=print):
    """Returns ({(wt, prec, ns_max): (best pair, scores, times, names)},
    {(wt, prec): ((best waves, best batch item taps), scores)})."""
    ev = _Events()
    results, waves = {}, {}
    for wt in classes:
        for prec in precisions:
            prev = None
            for ns_max in NS_BUCKETS:
                loads = bucket_workloads(wt, ns_max)
                if not loads:
                    results[(wt, prec, ns_max)] = prev
                    continue
                times = time_item_grid(loads, prec, ev, reps)
                for (mt, bal), tl in times.items():
                    log(f"W={wt} {prec} nS<={ns_max} min_item_taps={mt:g} balance_items={bal:g}: "
                        + ", ".join(f"{name} {t:.3f} ms" for (name, _), t in zip(loads, tl)))
                score = _score(times, len(loads))
                best = min(score, key=score.get)
                results[(wt, prec, ns_max)] = prev = (best, score, times, [n for n, _ in loads])
                log(f"W={wt} {prec} nS<={ns_max}: best min_item_taps={best[0]:g} balance_items={best[1]:g} "
                    f"(score {score[best]:.4f}; default pair {score[(1.2e5, 49152.0)]:.4f})")
            if wt == 64:
                batch = workloads.batch_rooms(1024, seed=0, feasible=_feasible)
                t = time_batch_grid(batch, prec, ev, reps)
                sc = _score(t, 1)
                waves[(wt, prec)] = (min(sc, key=sc.get), sc)
                log(f"W={wt} {prec} batch (waves per SIMD, item taps): "
                    + ", ".join(f"({k}, {it:g}) {t[(k, it)][0]:.3f} ms" for k, it in t))
    return results, waves


def write_header(results, waves, path: str, device: str) -> None:
    lines = [
        "// Work-item schedule per window length, tap precision and RIR length, read by",
        "// the host planner, and the grid of the persistent batch launch. Written by",
        f"// paper_1810_11359_amd/autotune.py from timings on the target GPU ({device}).",
        "//   min_item_taps  estimated taps of the smallest work item",
        "//   balance_items  items a large call is split into (about eight per",
        "//                  resident wave), which sets the item size of large calls",
        "//   ns_max         the entry applies to RIRs of at most this many samples",
        "//                  (first match in table order)",
        "//   waves          workgroups per SIMD of a persistent batch launch",
        "//   item_taps      largest work item of a batch job (estimated taps)",
        "//",
        "// Score: geometric mean over the bucket's workloads of kernel time relative",
        "// to the fastest pair on that workload (1.0 = fastest everywhere).",
    ]
    for (wt, prec, ns_max), (best, score, times, names) in sorted(results.items()):
        lines.append(f"// W={wt} {prec} nS<={ns_max} ({', '.join(names)}): best {best[0]:g} / {best[1]:g}, "
                     f"score {score[best]:.4f}, default 1.2e5 / 49152 score {score[(1.2e5, 49152.0)]:.4f}")
    for (wt, prec), (best, sc) in sorted(waves.items()):
        lines.append(f"// W={wt} {prec} batch: best {best[0]} waves per SIMD, items <= {best[1]:g} taps; "
                     + ", ".join(f"({k}, {it:g}): {v:.4f}" for (k, it), v in sorted(sc.items())))
    lines += ["#pragma once", "", "namespace ism {", "", "struct ItemTuning {",
              "  int wt;        // window cap in samples", "  int half;      // 1: FP16 taps, 0: FP32 taps",
              "  int ns_max;    // RIR length bucket (samples)", "  double min_item_taps;", "  double balance_items;",
              "};", "", "struct BatchTuning {", "  int wt;", "  int half;", "  int waves;", "  double item_taps;", "};",
              "",
              "constexpr ItemTuning kItemTuning[] = {"]
    for (wt, prec, ns_max), (best, _, _, _) in sorted(results.items()):
        lines.append(f"    {{{wt}, {1 if prec == 'fp16' else 0}, {ns_max}, {best[0]:.6g}, {best[1]:.1f}}},")
    lines += ["};", "", "constexpr BatchTuning kBatchTuning[] = {"]
    for (wt, prec), (best, _) in sorted(waves.items()):
        lines.append(f"    {{{wt}, {1 if prec == 'fp16' else 0}, {best[0]}, {best[1]:.6g}}},")
    if not waves:
        lines.append("    {0, 0, 0, 0.0},")
    lines += ["};", "", "}  // namespace ism", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True, help="header to write (the library's csrc/ism_tuning.h)")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    import torch

    if not torch.cuda.is_available():
        print("autotune needs a GPU", file=sys.stderr)
        return 2
    results, waves = tune(args.reps, log=lambda s: print(s, flush=True))
    write_header(results, waves, args.out, torch.cuda.get_device_name(0))
    print(f"wrote {args.out}; rebuild the library to use it", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
