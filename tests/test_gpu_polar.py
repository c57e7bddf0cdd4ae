"""Parity of directional receivers (ism_simulate_polar: first-order patterns
a + (1 - a) cos(theta)) with the float64 oracle, through the C ABI.

The pattern factor adds one FMA and one product to each image's amplitude,
with the projection of the displacement onto the orientation carried in FP32
(relative error ~1e-7 of |d|), so the FP32 tolerance of the plain path, 1e-5
of the RIR peak, applies. The omni pattern must give the plain RIR bit for
bit (the factor is exactly 1).
"""
import sys

import numpy as np
import pytest

from paper_1810_11359_amd import ism, workloads

from .helpers import oracle_room_args, rel_err
from .test_gpu_parity import CASES

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ism.lib()
    return torch


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _orients(n, seed):
    rng = np.random.default_rng(seed)
    o = rng.standard_normal((n, 3)).astype(np.float32)
    o[0] = [1.0, 0.0, 0.0]
    return o


@pytest.mark.parametrize("pattern", ["cardioid", "hypercardioid", "bidirectional"])
@pytest.mark.parametrize("case", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_small_rooms_polar(oracle_mod, case, pattern):
    import torch

    name, L, beta, n, fs, t_max, t_w, src, rcv = case
    room = ism.Room(L, beta, n, 343.0, fs, t_max, t_w)
    o = _orients(len(rcv), len(name))
    a = ism.PATTERNS[pattern]
    _say(f"polar {name} {pattern}")
    got = ism.simulate_polar(room, src, rcv, o, pattern)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.float64)
    ref = oracle_mod.rir_polar(L, beta, n, 343.0, fs, t_max, t_w, src, rcv, o, a)
    err = rel_err(got, ref)
    print(name, pattern, "polar rel err", err)
    assert np.all(err <= TOL)


def test_omni_is_the_plain_rir():
    import torch

    w = workloads.room_32_receivers(0)
    room = ism.room_for(w)
    _say("polar omni = plain")
    plain = ism.simulate(room, w.src, w.rcv[:4])
    omni = ism.simulate_polar(room, w.src, w.rcv[:4], _orients(4, 1), "omni")
    torch.cuda.synchronize()
    assert torch.equal(plain, omni)


def test_polar_workload_sampled(oracle_mod):
    import torch

    w = workloads.room_32_receivers(0)
    room = ism.room_for(w)
    o = _orients(32, 7)
    _say("polar room_32_receivers cardioid")
    got = ism.simulate_polar(room, w.src, w.rcv, o, "cardioid")
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(got))
    pick = [0, 21]
    L, beta, n, c, fs, t_max, t_w = oracle_room_args(oracle_mod, w)
    ref = oracle_mod.rir_polar(L, beta, n, c, fs, t_max, t_w, w.src, w.rcv[pick], o[pick], 0.5)
    err = rel_err(got[:, pick], ref)
    print("polar 32rcv rel err", err)
    assert np.all(err <= TOL)


@pytest.mark.parametrize("precision,tol,lut_q", [("fp16", 2e-3, 0), ("lut", 1e-5, 16)])
@pytest.mark.parametrize("case", [CASES[1], CASES[2]], ids=[CASES[1][0], CASES[2][0]])
def test_polar_other_tap_modes(oracle_mod, case, precision, tol, lut_q):
    """The pattern scales each image's amplitude before its taps, so it composes
    with the FP16 taps (their 2e-3 bound) and the table taps (compared with the
    oracle's table taps, 1e-5)."""
    import torch

    name, L, beta, n, fs, t_max, t_w, src, rcv = case
    room = ism.Room(L, beta, n, 343.0, fs, t_max, t_w)
    o = _orients(len(rcv), 3)
    _say(f"polar {precision} {name}")
    got = ism.simulate_polar(room, src, rcv, o, "hypercardioid", precision=precision)
    torch.cuda.synchronize()
    got = got.cpu().numpy().astype(np.float64)
    ref = oracle_mod.rir_polar(L, beta, n, 343.0, fs, t_max, t_w, src, rcv, o, 0.25, lut_q=lut_q)
    err = rel_err(got, ref)
    print(name, precision, "polar rel err", err)
    assert np.all(err <= tol)
