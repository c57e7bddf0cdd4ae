"""The diffuse tail on the GPU (ism_simulate_diffuse) against the FP64 oracle.

Both sides draw the same Philox4x32-10 words, so the tail is compared sample
by sample: the ISM part within 1e-5 of the RIR peak (as ism_simulate), the
tail within 2e-4 of its own envelope sqrt(A env(k)) (FP32 logarithms and the
level A estimated from the FP32 ISM part).
"""
import sys

import numpy as np
import pytest

from paper_1810_11359_amd import ism

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


CASES = [
    # name, room, t60, fs, t_w, t_diff, t_max, src, rcv, seed
    ("paper_t2_6rir", [3.0, 4.0, 2.5], 1.0, 16000.0, 0.004, 0.25, 1.0,
     [[1.0, 1.5, 1.2], [2.1, 2.6, 1.0]], [[2.0, 3.0, 1.5], [0.8, 0.9, 1.1], [1.5, 2.0, 2.0]], 1),
    ("w96_48k_short_ism", [4.4, 3.1, 2.7], 0.6, 48000.0, 0.002, 0.05, 0.4,
     [[1.3, 0.9, 1.1]], [[3.0, 2.2, 2.0]], 1 << 40),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_diffuse_matches_oracle(oracle_mod, case):
    import torch

    name, L, t60, fs, t_w, t_diff, t_max, src, rcv, seed = case
    beta = ism.beta_from_t60(L, t60)
    n = ism.n_img_for_time(L, 343.0, t_diff)
    room = ism.Room(L, list(beta), n, 343.0, fs, t_max, t_w)
    _say(f"{name} n_img={n} nS={room.n_samples}")
    got = ism.simulate_diffuse(room, src, rcv, t_diff, t60, seed).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    ref = oracle_mod.diffuse_rir(L, beta, n, 343.0, fs, t_max, t_w, t_diff, t60, seed, src, rcv)
    assert got.shape == ref.shape
    k_diff = oracle_mod.n_samples(t_diff, fs)
    peak = np.max(np.abs(ref[..., :k_diff]), axis=-1)
    e_ism = np.max(np.abs(got[..., :k_diff] - ref[..., :k_diff]), axis=-1) / peak
    ism_ref = ref[..., :k_diff]
    A = oracle_mod.envelope_level(ism_ref, fs, t_diff, t60)
    k = np.arange(k_diff, ref.shape[-1])
    scale = np.sqrt(A[..., None] * oracle_mod.envelope(k, fs, t_diff, t60))
    e_tail = np.max(np.abs(got[..., k_diff:] - ref[..., k_diff:]) / scale, axis=-1)
    print(name, "ism rel err", e_ism.ravel(), "tail err / envelope", e_tail.ravel())
    assert np.all(np.isfinite(got))
    assert np.all(e_ism <= 1e-5)
    assert np.all(e_tail <= 2e-4)


def test_diffuse_streams_differ_by_seed_and_pair():
    import torch

    L, t60 = [3.0, 4.0, 2.5], 0.7
    beta = ism.beta_from_t60(L, t60)
    room = ism.Room(L, list(beta), ism.n_img_for_time(L, 343.0, 0.1), 343.0, 16000.0, 0.5, 0.004)
    src, rcv = [[1.0, 1.5, 1.2]], [[2.0, 3.0, 1.5], [2.0, 3.0, 1.5]]
    _say("seeds")
    a = ism.simulate_diffuse(room, src, rcv, 0.1, t60, seed=3).cpu().numpy()
    b = ism.simulate_diffuse(room, src, rcv, 0.1, t60, seed=3).cpu().numpy()
    c = ism.simulate_diffuse(room, src, rcv, 0.1, t60, seed=4).cpu().numpy()
    torch.cuda.synchronize()
    k = ism.n_samples(0.1, 16000.0)
    assert np.array_equal(a, b)                          # deterministic
    assert np.array_equal(a[0, 0, :k], a[0, 1, :k])      # same position: same ISM part
    assert not np.allclose(a[0, 0, k:], a[0, 1, k:])     # but its own noise stream
    assert not np.allclose(a[0, 0, k:], c[0, 0, k:])     # and another seed, another tail


@pytest.mark.parametrize("precision", ["fp16", "lut"])
def test_diffuse_other_tap_modes(precision):
    """The diffuse call plans its ISM part like a single call with
    T_max = t_diff, so with FP16 or table taps that part equals ism_simulate's
    result bit for bit; the tail draws the same words as the FP32 call, so it
    is the FP32 tail times one constant per RIR, sqrt(A_mode / A_fp32)."""
    import torch

    name, L, t60, fs, t_w, t_diff, t_max, src, rcv, seed = CASES[0]
    beta = ism.beta_from_t60(L, t60)
    n = ism.n_img_for_time(L, 343.0, t_diff)
    room = ism.Room(L, list(beta), n, 343.0, fs, t_max, t_w)
    room_ism = ism.Room(L, list(beta), n, 343.0, fs, t_diff, t_w)
    _say(f"diffuse {precision} {name}")
    got = ism.simulate_diffuse(room, src, rcv, t_diff, t60, seed, precision=precision).cpu().numpy()
    ism_part = ism.simulate(room_ism, src, rcv, precision=precision).cpu().numpy()
    ref32 = ism.simulate_diffuse(room, src, rcv, t_diff, t60, seed).cpu().numpy()
    torch.cuda.synchronize()
    k_diff = ism.n_samples(t_diff, fs)
    assert np.array_equal(got[..., :k_diff], ism_part)
    tail, tail32 = got[..., k_diff:].astype(np.float64), ref32[..., k_diff:].astype(np.float64)
    for i in np.ndindex(tail.shape[:-1]):
        big = np.abs(tail32[i]) > 1e-3 * np.max(np.abs(tail32[i]))
        ratio = tail[i][big] / tail32[i][big]
        c = np.median(ratio)
        assert 0.9 < c < 1.1  # the level moves with the tap mode's small error only
        assert np.max(np.abs(ratio - c)) <= 1e-5 * abs(c)


def test_diffuse_directional_receivers():
    """ism_simulate_diffuse_polar: the ISM part equals ism_simulate_polar's
    RIR for T_max = t_diff bit for bit, and the tail draws the same words as
    the omnidirectional call, so it is that tail times one constant per RIR
    (the square root of the ratio of the two levels A)."""
    import torch

    name, L, t60, fs, t_w, t_diff, t_max, src, rcv, seed = CASES[0]
    beta = ism.beta_from_t60(L, t60)
    n = ism.n_img_for_time(L, 343.0, t_diff)
    room = ism.Room(L, list(beta), n, 343.0, fs, t_max, t_w)
    room_ism = ism.Room(L, list(beta), n, 343.0, fs, t_diff, t_w)
    o = np.array([[1.0, 0.0, 0.0], [0.0, -1.0, 0.5], [0.3, 0.3, 1.0]], dtype=np.float32)
    _say(f"diffuse cardioid {name}")
    got = ism.simulate_diffuse_polar(room, src, rcv, o, t_diff, t60, seed, "cardioid").cpu().numpy()
    ism_part = ism.simulate_polar(room_ism, src, rcv, o, "cardioid").cpu().numpy()
    omni = ism.simulate_diffuse(room, src, rcv, t_diff, t60, seed).cpu().numpy()
    torch.cuda.synchronize()
    k_diff = ism.n_samples(t_diff, fs)
    assert np.array_equal(got[..., :k_diff], ism_part)
    assert not np.allclose(got[..., :k_diff], omni[..., :k_diff])
    tail, tail_o = got[..., k_diff:].astype(np.float64), omni[..., k_diff:].astype(np.float64)
    for i in np.ndindex(tail.shape[:-1]):
        big = np.abs(tail_o[i]) > 1e-3 * np.max(np.abs(tail_o[i]))
        ratio = tail[i][big] / tail_o[i][big]
        c = np.median(ratio)
        assert 0.0 < c < 1.5
        assert np.max(np.abs(ratio - c)) <= 1e-5 * c
