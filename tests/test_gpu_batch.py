"""Batches of rooms through ism_batch_prepare / ism_batch_run (GPU).

A batch must give, job by job, bitwise the same RIRs as ism_simulate of that
job alone with the same work split (single calls without the tail taper),
match the FP64 oracle within 1e-5 of the peak, and replay identically from
a captured HIP graph.
"""
import sys

import numpy as np
import pytest

from paper_1810_11359_amd import ism, workloads

from .helpers import assert_no_value_above_peak, oracle_peak, oracle_room_args, rel_err

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ism.lib()
    return torch


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _mixed_jobs():
    rng = np.random.default_rng(7)
    jobs = []
    specs = [((3.0, 4.0, 2.5), 0.25, 16000.0, 0.004, 1, 3), ((4.4, 3.1, 2.7), 0.15, 48000.0, 0.002, 2, 2),
             ((6.0, 5.0, 3.0), 0.3, 8000.0, 0.004, 1, 1), ((2.5, 2.5, 2.5), 0.12, 16000.0, 0.004, 1, 5),
             ((8.0, 7.0, 3.5), 0.4, 16000.0, 0.004, 1, 2)]
    for L, t60, fs, tw, ns, nr in specs:
        beta = ism.beta_from_t60(L, t60) * rng.uniform(0.92, 1.0, 6)
        room = ism.Room(list(L), list(beta), ism.n_img_for_time(L, 343.0, t60), 343.0, fs, t60, tw)
        src = rng.uniform(0.5, np.array(L) - 0.5, (ns, 3)).astype(np.float32)
        rcv = rng.uniform(0.5, np.array(L) - 0.5, (nr, 3)).astype(np.float32)
        jobs.append((room, src, rcv))
    return jobs


# with an explicit item size every job of a batch is planned exactly as its
# single call with the same schedule (bitwise equal results); by default a
# batch sizes its items from its total work, so a job agrees with its single
# call within the rounding of another split
SHARED = ism.Schedule(item_taps=60000.0)
UNTAPERED = ism.Schedule(tail_rounds=0.0)


def _close(a, b, peak_of):
    import torch

    peak = torch.amax(torch.abs(peak_of), dim=-1)
    return bool(torch.all(torch.amax(torch.abs(a - b), dim=-1) <= 1e-6 * peak))


def test_batch_equals_single_room_calls(oracle_mod):
    import torch

    jobs = _mixed_jobs()
    _say("mixed batch")
    outs = [o.clone() for o in ism.BatchSimulator(jobs).run()]
    shared = [o.clone() for o in ism.BatchSimulator(jobs, schedule=SHARED).run()]
    torch.cuda.synchronize()
    for (room, src, rcv), o, sh in zip(jobs, outs, shared):
        single = ism.simulate(room, src, rcv, schedule=SHARED)
        alone = ism.BatchSimulator([(room, src, rcv)]).run()[0]
        untapered = ism.simulate(room, src, rcv, schedule=UNTAPERED)
        tapered = ism.simulate(room, src, rcv)
        torch.cuda.synchronize()
        assert torch.equal(sh, single), f"batch differs from the single call with its schedule for {room.room}"
        assert torch.equal(alone, untapered), f"a one-job batch differs from the untapered call for {room.room}"
        # other splits (batch-sized items, the single call's tapered tail): same sums within rounding
        assert _close(o, single, single) and _close(tapered, o, single) and _close(alone, o, single)
    # oracle on two of the jobs
    for k in (0, 1):
        room, src, rcv = jobs[k]
        ref = oracle_mod.rir(room.room, room.beta, room.n_img, room.c, room.fs, room.t_max, room.t_w, src, rcv)
        err = rel_err(outs[k].cpu().numpy(), ref)
        print("job", k, "rel err", err)
        assert np.all(err <= TOL_FP32)


def test_batch_table_taps_equal_single_calls():
    """Table taps (Eq. (9)) through the batch path: each job bitwise equal to
    its own single-room call with the same precision (and schedule)."""
    import torch

    jobs = _mixed_jobs()
    _say("mixed batch, table taps")
    b = ism.BatchSimulator(jobs, precision="lut", schedule=SHARED)
    outs = [o.clone() for o in b.run()]
    torch.cuda.synchronize()
    for (room, src, rcv), o in zip(jobs, outs):
        single = ism.simulate(room, src, rcv, precision="lut", schedule=SHARED)
        torch.cuda.synchronize()
        assert torch.equal(o, single), f"batch differs from single-room call for {room.room}"


def test_batch_directional_jobs_equal_single_calls():
    """A batch mixing directional and omnidirectional jobs (one shared item
    size): every job bitwise equal to itself alone in a batch, omnidirectional
    jobs bitwise equal to their single call (their pattern factor is exactly
    1), directional jobs within rounding of ism_simulate_polar (whose default
    schedule tapers the tail)."""
    import torch

    jobs = _mixed_jobs()
    rng = np.random.default_rng(11)
    patterns = ["cardioid", None, "bidirectional", None, "hypercardioid"]
    batch_jobs = []
    for (room, src, rcv), pat in zip(jobs, patterns):
        if pat is None:
            batch_jobs.append((room, src, rcv))
        else:
            batch_jobs.append((room, src, rcv, rng.standard_normal((len(rcv), 3)).astype(np.float32), pat))
    _say("mixed batch, directional jobs")
    b = ism.BatchSimulator(batch_jobs, schedule=SHARED)
    outs = [o.clone() for o in b.run()]
    torch.cuda.synchronize()
    for job, o in zip(batch_jobs, outs):
        alone = ism.BatchSimulator([job], schedule=SHARED).run()[0]
        torch.cuda.synchronize()
        assert torch.equal(o, alone), f"batch job differs from the job alone for {job[0].room}"
        if len(job) == 5:
            single = ism.simulate_polar(job[0], job[1], job[2], job[3], job[4])
            torch.cuda.synchronize()
            assert _close(single, o, single)
        else:
            single = ism.simulate(job[0], job[1], job[2], schedule=SHARED)
            torch.cuda.synchronize()
            assert torch.equal(o, single), f"batch differs from single-room call for {job[0].room}"


def _feasible(oracle_mod):
    def ok(room, t60):
        try:
            oracle_mod.beta_from_t60(room, t60)
            return True
        except ValueError:
            return False

    return ok


def test_batch_1024_rooms_sampled(oracle_mod):
    import torch

    ws = workloads.batch_rooms(1024, seed=0, feasible=_feasible(oracle_mod))
    jobs = [(ism.room_for(w), w.src, w.rcv) for w in ws]
    _say(f"1024-room batch, {sum(w.src.shape[0] * w.rcv.shape[0] for w in ws)} RIRs")
    b = ism.BatchSimulator(jobs)
    outs = b.run()
    torch.cuda.synchronize()
    # rooms with the fewest and the most image taps per RIR (volume vs T60^3) + random ones
    dens = np.array([w.t60 ** 3 / np.prod(w.room) for w in ws])
    pick = [int(np.argmin(dens)), int(np.argmax(dens))] + list(np.random.default_rng(1).choice(len(ws), 3, replace=False))
    for k in pick:
        w = ws[k]
        args = oracle_room_args(oracle_mod, w)
        got = outs[k].cpu().numpy()
        assert np.all(np.isfinite(got))
        nS = got.shape[-1]
        if nS * w.t60 ** 3 / np.prod(w.room) < 40.0:
            ref = oracle_mod.rir(*args, w.src, w.rcv)
            err = rel_err(got, ref)
        else:  # long, dense RIR: early window (holds the peak) and the last window
            peak, _ = oracle_peak(oracle_mod, args, w.src, w.rcv, nS)
            assert_no_value_above_peak(got, peak, TOL_FP32)
            err = np.zeros(peak.shape)
            for k0, k1 in [(0, 1200), (nS - 1200, nS)]:
                ref = oracle_mod.rir(*args, w.src, w.rcv, k_begin=k0, k_end=k1)
                err = np.maximum(err, np.max(np.abs(got[..., k0:k1] - ref), axis=-1) / peak)
        print("room", k, w.room.round(2), "t60", round(w.t60, 3), "rel err", err.ravel())
        assert np.all(err <= TOL_FP32)


def test_batch_fp16_sampled(oracle_mod):
    """FP16 taps through the batch path at the 1024-room size, on sampled
    rooms (the sparsest, the densest and random ones), within 2e-3 of the peak."""
    import torch

    ws = workloads.batch_rooms(1024, seed=0, feasible=_feasible(oracle_mod))
    jobs = [(ism.room_for(w), w.src, w.rcv) for w in ws]
    _say("1024-room batch, fp16")
    b = ism.BatchSimulator(jobs, precision="fp16")
    outs = b.run()
    torch.cuda.synchronize()
    dens = np.array([w.t60 ** 3 / np.prod(w.room) for w in ws])
    pick = [int(np.argmin(dens)), int(np.argmax(dens))] + list(np.random.default_rng(2).choice(len(ws), 2, replace=False))
    for k in pick:
        w = ws[k]
        args = oracle_room_args(oracle_mod, w)
        got = outs[k].cpu().numpy()
        assert np.all(np.isfinite(got))
        nS = got.shape[-1]
        peak, _ = oracle_peak(oracle_mod, args, w.src, w.rcv, nS)
        assert_no_value_above_peak(got, peak, 2e-3)
        err = np.zeros(peak.shape)
        for k0, k1 in [(0, min(nS, 1200)), (max(0, nS - 600), nS)]:
            ref = oracle_mod.rir(*args, w.src, w.rcv, k_begin=k0, k_end=k1)
            err = np.maximum(err, np.max(np.abs(got[..., k0:k1] - ref), axis=-1) / peak)
        print("room", k, "fp16 rel err", err.ravel())
        assert np.all(err <= 2e-3)


def test_batch_graph_replay():
    import torch

    jobs = _mixed_jobs()
    _say("graph replay")
    b = ism.BatchSimulator(jobs)
    eager = [o.clone() for o in b.run()]
    torch.cuda.synchronize()
    for o in b.outs:
        o.zero_()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        b.run(stream=s)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for o in b.outs:
            o.fill_(float(rep + 1))  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for e, o in zip(eager, b.outs):
            assert torch.equal(e, o), f"replay {rep} differs from the eager run"


def test_long_runs_reduce(oracle_mod):
    """Tiles split into 64 items or more (a fine fixed split) take the reduce
    that sums long runs in slices on several threads: the single call agrees
    with the oracle, and a one-job batch with the same split (which sums the
    same runs in the same order) is bitwise equal to it. The last tiles of
    this 4800-sample RIR hold about 1e6 estimated taps each, so 2000-tap items
    split them into the cap of 255."""
    import torch

    w = workloads.single_rir(0)
    room = ism.room_for(w)
    fine = ism.Schedule(item_taps=2000.0)
    _say("long reduce runs (items of 2000 taps)")
    single = ism.simulate(room, w.src, w.rcv, schedule=fine)
    alone = ism.BatchSimulator([(room, w.src, w.rcv)], schedule=fine).run()[0]
    torch.cuda.synchronize()
    assert torch.equal(single, alone), "one-job batch differs from the single call with the same split"
    ref = oracle_mod.rir(room.room, room.beta, room.n_img, room.c, room.fs, room.t_max, room.t_w, w.src, w.rcv)
    err = rel_err(single.cpu().numpy(), ref)
    print("rel err", err.ravel(), flush=True)
    assert np.all(err <= TOL_FP32)
