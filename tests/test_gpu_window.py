"""Windows of any length (Eq. (6): W = T_w fs samples, any real W up to 256):
parity of the general-mode kernels with the FP64 oracle, which takes any W.

Each case is a small room the oracle finishes in seconds, at sampling rates
and window lengths whose W is not one of the exact-mode windows {32, 64, 96,
128}: 44.1 kHz x 4 ms (W = 176.4), 22.05 kHz x 4 ms (88.2), 48 kHz x 4 ms
(192), 16 kHz x 2.5 ms (40), an odd W = 33, a short W = 16.5 and very short
W = 6.4 and 4.4 (few taps per image, each with a large window-phase term).
Tolerance: max|err| / oracle peak <= 1e-5 (FP32 taps), <= 2e-3 (FP16 taps).
"""
import sys

import numpy as np
import pytest

from paper_1810_11359_amd import ism

from .helpers import assert_no_value_above_peak, rel_err

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5
TOL_FP16 = 2e-3

# (name, fs, t_w, t_max)
WINDOWS = [
    ("44k1_4ms_W176.4", 44100.0, 0.004, 0.09),
    ("22k05_4ms_W88.2", 22050.0, 0.004, 0.12),
    ("48k_4ms_W192", 48000.0, 0.004, 0.08),
    ("16k_2.5ms_W40", 16000.0, 0.0025, 0.15),
    ("11k_3ms_W33", 11000.0, 0.003, 0.15),
    ("5.5k_3ms_W16.5", 5500.0, 0.003, 0.2),
    ("8k_0.8ms_W6.4", 8000.0, 0.0008, 0.2),
    ("11k_0.4ms_W4.4", 11000.0, 0.0004, 0.15),
]


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _case(fs, t_w, t_max, n_rcv=3, seed=3):
    rng = np.random.default_rng(seed)
    L = [3.7, 4.3, 2.8]
    beta = list(ism.beta_from_t60(L, 0.3) * rng.uniform(0.9, 1.0, 6))
    room = ism.Room(L, beta, ism.n_img_for_time(L, 343.0, t_max), 343.0, fs, t_max, t_w)
    src = rng.uniform(0.5, np.array(L) - 0.5, (1, 3)).astype(np.float32)
    rcv = rng.uniform(0.5, np.array(L) - 0.5, (n_rcv, 3)).astype(np.float32)
    return room, src, rcv


def _oracle(oracle_mod, room, src, rcv):
    return oracle_mod.rir(room.room, room.beta, room.n_img, room.c, room.fs, room.t_max, room.t_w, src, rcv)


@pytest.mark.parametrize("name,fs,t_w,t_max", WINDOWS, ids=[w[0] for w in WINDOWS])
def test_general_window_fp32(oracle_mod, name, fs, t_w, t_max):
    import torch

    room, src, rcv = _case(fs, t_w, t_max)
    _say(f"window {name}: W = {fs * t_w:g}, nS = {room.n_samples}, n_img = {room.n_img}")
    got = ism.simulate(room, src, rcv)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.float64)
    ref = _oracle(oracle_mod, room, src, rcv)
    peak = np.max(np.abs(ref), axis=-1)
    assert_no_value_above_peak(got, peak, TOL_FP32)
    err = rel_err(got, ref)
    print("rel err", err.ravel(), flush=True)
    assert np.all(err <= TOL_FP32)
    # a fine fixed split (many items per tile, split tiles, margins) agrees
    fine = ism.simulate(room, src, rcv, schedule=ism.Schedule(item_taps=4000.0))
    torch.cuda.synchronize()
    assert np.all(rel_err(fine.cpu().numpy(), ref) <= TOL_FP32)


@pytest.mark.parametrize("name,fs,t_w,t_max", [WINDOWS[0], WINDOWS[3], WINDOWS[4]],
                         ids=[WINDOWS[0][0], WINDOWS[3][0], WINDOWS[4][0]])
def test_general_window_fp16(oracle_mod, name, fs, t_w, t_max):
    import torch

    room, src, rcv = _case(fs, t_w, t_max, seed=4)
    _say(f"window {name} fp16")
    got = ism.simulate(room, src, rcv, precision="fp16")
    torch.cuda.synchronize()
    ref = _oracle(oracle_mod, room, src, rcv)
    err = rel_err(got.cpu().numpy(), ref)
    print("fp16 rel err", err.ravel(), flush=True)
    assert np.all(err <= TOL_FP16)


def test_general_window_polar(oracle_mod):
    import torch

    room, src, rcv = _case(44100.0, 0.004, 0.09, seed=5)
    o = np.random.default_rng(6).standard_normal(rcv.shape).astype(np.float32)
    _say("window 44k1 cardioid")
    got = ism.simulate_polar(room, src, rcv, o, "cardioid")
    torch.cuda.synchronize()
    ref = oracle_mod.rir_polar(room.room, room.beta, room.n_img, room.c, room.fs, room.t_max, room.t_w, src, rcv, o,
                               0.5)
    err = rel_err(got.cpu().numpy(), ref)
    print("polar rel err", err.ravel(), flush=True)
    assert np.all(err <= TOL_FP32)


def test_general_windows_in_one_batch(oracle_mod):
    """Jobs of four windows (two exact, two general; three caps) in one batch
    with a shared item size: each bitwise equal to its single call with that
    schedule, one checked against the oracle."""
    import torch

    jobs = []
    for k, (fs, t_w, t_max) in enumerate([(16000.0, 0.004, 0.12), (44100.0, 0.004, 0.06), (48000.0, 0.002, 0.06),
                                          (22050.0, 0.004, 0.1)]):
        jobs.append(_case(fs, t_w, t_max, n_rcv=2, seed=10 + k))
    _say("batch of windows 64, 176.4, 96, 88.2")
    sched = ism.Schedule(item_taps=50000.0)
    outs = [o.clone() for o in ism.BatchSimulator(jobs, schedule=sched).run()]
    torch.cuda.synchronize()
    for (room, src, rcv), o in zip(jobs, outs):
        single = ism.simulate(room, src, rcv, schedule=sched)
        torch.cuda.synchronize()
        assert torch.equal(o, single), f"batch differs from single call at W = {room.fs * room.t_w:g}"
    room, src, rcv = jobs[1]
    assert np.all(rel_err(outs[1].cpu().numpy(), _oracle(oracle_mod, room, src, rcv)) <= TOL_FP32)
