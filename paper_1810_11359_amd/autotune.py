"""Work-item schedule tuner. Run it on the target GPU:

    python -m paper_1810_11359_amd.autotune --out paper_1810_11359_amd/csrc/ism_tuning.h

For every window length W (32, 64, 96, 128 samples) and tap precision it times
the tap-accumulation kernel (HIP events the library records around it) on
representative workloads over a grid of (min_item_taps, balance_items) pairs,
keeps the pair with the best geometric-mean time relative to each workload's
fastest pair, and writes the table header the host planner compiles in.
Rebuild the library afterwards. The candidate values reach the planner as
the call's explicit schedule (``ism_schedule``: min_item_taps,
balance_items).
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


def class_workloads(wt: int):
    """Representative single-room and batch workloads for one window length."""
    base = workloads.room_32_receivers(0)
    if wt == 32:
        return [("room_4x5x3_32rcv_8k", [replace(base, fs=8000.0)])]
    if wt == 64:
        return [("room_4x5x3_32rcv_16k", [base]),
                ("batch_256_rooms_16k", workloads.batch_rooms(256, seed=0, feasible=_feasible))]
    if wt == 96:
        return [("room_6x9x3.5_uca64_48k", [workloads.large_room_uca(0)])]
    if wt == 128:
        w = replace(base, fs=32000.0, t60=0.5, t_max=0.5, rcv=base.rcv[:16])
        return [("room_4x5x3_16rcv_32k", [w])]
    raise ValueError(wt)


def time_kernel(ws, precision: str, ev: _Events, reps: int, schedule=None) -> float:
    """Mean accumulate-kernel time (ms) of one call over the workload(s)."""
    import torch

    if len(ws) == 1:
        w = ws[0]
        sim = ism.Simulator(ism.room_for(w), w.src, w.rcv, precision=precision, schedule=schedule)
    else:
        sim = ism.BatchSimulator([(ism.room_for(w), w.src, w.rcv) for w in ws], precision=precision,
                                 schedule=schedule)
    sim.run()
    torch.cuda.synchronize()
    pairs = [ev.pair() for _ in range(reps)]
    for a, b in pairs:
        sim.run(ev_start=a, ev_stop=b)
    torch.cuda.synchronize()
    t = [ev.ms(a, b) for a, b in pairs]
    for a, b in pairs:
        ev.free(a, b)
    return float(np.mean(t))


def tune(reps: int = 3, classes=(32, 64, 96, 128), precisions=("fp32", "fp16"), log=print):
    ev = _Events()
    results = {}
    for wt in classes:
        loads = class_workloads(wt)
        for prec in precisions:
            times = {}
            for mt in MIN_TAPS:
                for bal in BALANCE:
                    sc = ism.Schedule(min_item_taps=mt, balance_items=bal)
                    times[(mt, bal)] = [time_kernel(ws, prec, ev, reps, sc) for _, ws in loads]
                    log(f"W={wt} {prec} min_item_taps={mt:g} balance_items={bal:g}: "
                        + ", ".join(f"{name} {t:.3f} ms" for (name, _), t in zip(loads, times[(mt, bal)])))
            best_each = [min(t[i] for t in times.values()) for i in range(len(loads))]
            score = {k: math.exp(np.mean([math.log(t / b) for t, b in zip(v, best_each)])) for k, v in times.items()}
            best = min(score, key=score.get)
            results[(wt, prec)] = (best, score, times, [n for n, _ in loads])
            log(f"W={wt} {prec}: best min_item_taps={best[0]:g} balance_items={best[1]:g} "
                f"(score {score[best]:.4f}; default pair {score[(1.2e5, 49152.0)]:.4f})")
    return results


def write_header(results, path: str, device: str) -> None:
    lines = [
        "// Work-item schedule per window length and tap precision, read by the host",
        "// planner. Written by paper_1810_11359_amd/autotune.py from timings on the",
        f"// target GPU ({device}).",
        "//   min_item_taps  estimated taps of the smallest work item",
        "//   balance_items  items a large call is split into (about eight per",
        "//                  resident wave), which sets the item size of large calls",
        "//",
        "// Score: geometric mean over the class's workloads of kernel time relative",
        "// to the fastest pair on that workload (1.0 = fastest everywhere).",
    ]
    for (wt, prec), (best, score, times, names) in sorted(results.items()):
        lines.append(f"// W={wt} {prec} ({', '.join(names)}): best {best[0]:g} / {best[1]:g}, "
                     f"score {score[best]:.4f}, default 1.2e5 / 49152 score {score[(1.2e5, 49152.0)]:.4f}")
    lines += ["#pragma once", "", "namespace ism {", "", "struct ItemTuning {",
              "  int wt;        // window length in samples", "  int half;      // 1: FP16 taps, 0: FP32 taps",
              "  double min_item_taps;", "  double balance_items;", "};", "", "constexpr ItemTuning kItemTuning[] = {"]
    for (wt, prec), (best, _, _, _) in sorted(results.items()):
        lines.append(f"    {{{wt}, {1 if prec == 'fp16' else 0}, {best[0]:.6g}, {best[1]:.1f}}},")
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
    results = tune(args.reps, log=lambda s: print(s, flush=True))
    write_header(results, args.out, torch.cuda.get_device_name(0))
    print(f"wrote {args.out}; rebuild the library to use it", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
