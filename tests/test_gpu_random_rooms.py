"""Seeded random rooms through the HIP path against the FP64 oracle.

Each case draws a shoebox (sides 1.5-9 m), six signed reflection
coefficients in [-0.97, 0.97] (a zero coefficient now and then), image counts
per axis of either parity, a sampling rate and window from a list that mixes
the exact windows (32, 64, 96, 128 samples) with general ones (W = 16.5 up to
256), positions anywhere inside the room down to 1 cm from a wall, and a tap
precision. Tolerances as for the fixed cases: max |err| / oracle peak
<= 1e-5 for FP32 and table taps (the latter against the oracle's own table
taps), <= 2e-3 for FP16 taps.
"""
import sys

import numpy as np
import pytest

from paper_1810_11359_amd import ism

from .helpers import assert_no_value_above_peak, rel_err

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "lut": 1e-5, "fp16": 2e-3}
# (fs, t_w): exact windows W = 32, 64, 96, 128 and general ones
WINDOWS = [(8000.0, 0.004), (16000.0, 0.004), (48000.0, 0.002), (32000.0, 0.004), (44100.0, 0.004),
           (22050.0, 0.003), (11000.0, 0.0015), (16000.0, 0.016), (48000.0, 0.0053)]
N_CASES = 16


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    L = rng.uniform(1.5, 9.0, 3)
    beta = rng.uniform(0.3, 0.97, 6) * rng.choice([-1.0, 1.0], 6)
    if rng.random() < 0.3:
        beta[rng.integers(0, 6)] = 0.0
    fs, t_w = WINDOWS[seed % len(WINDOWS)]
    W = fs * t_w
    exact = abs(W - round(W)) < 1e-9 and int(round(W)) in (32, 64, 96, 128)
    precision = ["fp32", "fp16", "lut"][seed % 3] if exact else ["fp32", "fp16"][seed % 2]
    t_max = float(rng.uniform(0.03, 0.25))
    n_img = tuple(int(v) for v in rng.integers(3, 24, 3))
    n_src, n_rcv = int(rng.integers(1, 3)), int(rng.integers(1, 4))
    margin = 0.01 if seed % 4 == 0 else 0.2
    src = rng.uniform(margin, L - margin, (n_src, 3)).astype(np.float32)
    rcv = rng.uniform(margin, L - margin, (n_rcv, 3)).astype(np.float32)
    # keep every receiver at least 5 cm from every source (A = 1 / (4 pi d))
    for k in range(n_rcv):
        while np.min(np.linalg.norm(src - rcv[k], axis=-1)) < 0.05:
            rcv[k] = rng.uniform(margin, L - margin).astype(np.float32)
    room = ism.Room([float(v) for v in L], [float(b) for b in beta], n_img, 343.0, fs, t_max, t_w)
    return room, src, rcv, precision


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_room(oracle_mod, seed):
    import torch

    room, src, rcv, precision = _case(seed)
    print(f"[case] seed {seed}: L={np.round(room.room, 2).tolist()} n_img={room.n_img} fs={room.fs:g} "
          f"W={room.fs * room.t_w:g} nS={room.n_samples} {precision} {src.shape[0]}x{rcv.shape[0]}", flush=True)
    sys.stdout.flush()
    got = ism.simulate(room, src, rcv, precision=precision)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.float64)
    ref = oracle_mod.rir(room.room, room.beta, room.n_img, room.c, room.fs, room.t_max, room.t_w, src, rcv,
                         lut_q=16 if precision == "lut" else 0)
    peak = np.max(np.abs(ref), axis=-1)
    assert np.all(peak > 0.0)
    assert_no_value_above_peak(got, peak, TOL[precision])
    err = rel_err(got, ref, peak)
    print("rel err", err.ravel(), flush=True)
    assert np.all(err <= TOL[precision])


def test_random_rooms_in_one_batch(oracle_mod):
    """All the random rooms as one FP32 batch: eight window classes (four exact
    windows, four general caps) in one call, each job against the oracle."""
    import torch

    cases = [_case(seed)[:3] for seed in range(N_CASES)]
    print(f"[case] batch of {len(cases)} random rooms", flush=True)
    sys.stdout.flush()
    outs = [o.clone() for o in ism.BatchSimulator(cases).run()]
    torch.cuda.synchronize()
    for seed, ((room, src, rcv), o) in enumerate(zip(cases, outs)):
        ref = oracle_mod.rir(room.room, room.beta, room.n_img, room.c, room.fs, room.t_max, room.t_w, src, rcv)
        peak = np.max(np.abs(ref), axis=-1)
        got = o.cpu().numpy().astype(np.float64)
        assert_no_value_above_peak(got, peak, TOL["fp32"])
        err = rel_err(got, ref, peak)
        assert np.all(err <= TOL["fp32"]), (seed, err)
