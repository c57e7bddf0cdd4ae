"""Host-side behaviour of bench.py (no GPU): the one-GPU guard and the
traffic figure taken from the committed counter summary."""
import os
import subprocess
import sys

import numpy as np

import bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=bench.ROOT, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_table_taps_refused_for_serving():
    r = subprocess.run([sys.executable, "bench.py", "--rate", "100", "--precision", "lut"],
                       cwd=bench.ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "serving loop" in r.stderr


def test_traffic_only_for_the_profiled_library(monkeypatch):
    # at least the output bytes of each workload, when the loaded library is
    # the profiled one (a rebuild from other sources gives None)
    t = bench.measured_traffic("room_32_receivers", "fp32")
    assert t is None or (isinstance(t, int) and t > 1_433_600)
    t = bench.measured_traffic("batch_rooms", "fp32")
    assert t is None or (isinstance(t, int) and t > 180_828_612)
    assert bench.measured_traffic("room_32_receivers", "fp16") is None
    assert bench.measured_traffic("single_rir", "fp32") is None
    # moving-source filter: the RIRs (307.2 MB) at least, direct and FFT
    for key in ("traffic_bytes_per_launch_direct", "traffic_bytes_per_call_fft"):
        t = bench.measured_traffic("moving_source_48k_96000", "fp32", key)
        assert t is None or (isinstance(t, int) and t > 307_200_000)
    monkeypatch.setattr(bench, "library_sha256", lambda: "0" * 64)
    assert bench.measured_traffic("room_32_receivers", "fp32") is None
    assert bench.measured_traffic("batch_rooms", "fp32") is None


def test_tuner_header_round_trip(tmp_path):
    """The tuner's header lists one entry per (window, precision, RIR length
    bucket) with the chosen pair, and the chosen batch grid per class."""
    from paper_1810_11359_amd import autotune

    res, waves = {}, {}
    for wt in (32, 64):
        for prec in ("fp32", "fp16"):
            for ns in autotune.NS_BUCKETS:
                score = {(mt, bal): 1.0 + 0.01 * i for i, (mt, bal) in
                         enumerate((a, b) for a in autotune.MIN_TAPS for b in autotune.BALANCE)}
                res[(wt, prec, ns)] = ((autotune.MIN_TAPS[0], autotune.BALANCE[0]), score, {}, ["w"])
    waves[(64, "fp32")] = ((6, 2.5e5), {(k, it): 1.0 for k in autotune.BATCH_WAVES
                                         for it in autotune.BATCH_ITEM_TAPS})
    p = tmp_path / "ism_tuning.h"
    autotune.write_header(res, waves, str(p), "test device")
    text = p.read_text()
    first = f"{autotune.MIN_TAPS[0]:.6g}, {autotune.BALANCE[0]:.1f}}}"
    for ns in autotune.NS_BUCKETS:
        assert text.count(f"{{32, 0, {ns}, " + first) == 1 and text.count(f"{{64, 1, {ns}, " + first) == 1
    assert "constexpr ItemTuning kItemTuning[]" in text and "{64, 0, 6, 250000}," in text


def test_committed_tuning_table_covers_every_exact_window():
    """Every exact window and precision has a catch-all entry (the last
    bucket), so every RIR length finds its schedule."""
    import re

    text = open(os.path.join(bench.ROOT, "paper_1810_11359_amd", "csrc", "ism_tuning.h")).read()
    entries = re.findall(r"\{(\d+), ([01]), (\d+), ([0-9.e+]+), ([0-9.e+]+)\}", text)
    for wt in (32, 64, 96, 128):
        for half in ("0", "1"):
            assert any(int(e[0]) == wt and e[1] == half and int(e[2]) == 2147483647 for e in entries), (wt, half)


def test_paper_table_cases_are_nested():
    from paper_1810_11359_amd import workloads

    full = workloads.paper_room_128rir(0)
    for t60, n_rcv in bench.PAPER_TABLE_CASES:
        w = workloads.paper_table_room(t60, n_rcv, 0)
        assert w.t60 == t60 and w.t_max == t60
        np.testing.assert_array_equal(w.src, full.src)
        np.testing.assert_array_equal(w.rcv, full.rcv[:n_rcv])
