"""Degenerate shapes of the problem on the GPU, against the FP64 oracle.

- direct path only: one lattice index per axis (N = 1 gives n = 0 alone), so
  the RIR is the single windowed-sinc tap of Eq. (6) at d fs / c;
- a three-sample RIR: one tile, almost every tap of each window outside
  [0, nS);
- an RIR of zeros: T_max ends more than W/2 samples before the direct path
  arrives, so no image reaches the output; every sample must still be
  written (a NaN-filled output must come back as exact zeros);
- one source with many receivers at the same point as another receiver
  (identical pairs give identical RIRs, bit for bit);
- the limits: nS = ISM_MAX_SAMPLES exactly, and ISM_MAX_N_IMG lattice
  indices along one axis.
Tolerance as for the other FP32 cases: max|err| / oracle peak <= 1e-5.
"""
import sys

import numpy as np
import pytest

from paper_1810_11359_amd import ism

from .helpers import rel_err

pytestmark = pytest.mark.gpu

TOL_FP32 = 1e-5


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _oracle(oracle_mod, room, src, rcv):
    return oracle_mod.rir(room.room, room.beta, room.n_img, room.c, room.fs, room.t_max, room.t_w, src, rcv)


def _host(room, src, rcv, precision="fp32"):
    import torch

    out = torch.full((len(src), len(rcv), room.n_samples), float("nan"), dtype=torch.float32, device="cuda")
    ism.simulate_host(room, np.asarray(src, np.float32), np.asarray(rcv, np.float32), precision=precision, out=out)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


CASES = [
    # (name, room, beta, n_img, fs, t_max, t_w, src, rcv)
    ("direct_path_only", [3.0, 4.0, 2.5], [0.9] * 6, (1, 1, 1), 16000.0, 0.02, 0.004,
     [[1.0, 1.0, 1.0]], [[2.0, 3.0, 1.5], [2.5, 0.5, 2.0]]),
    ("three_samples", [3.0, 4.0, 2.5], [0.9] * 6, (4, 4, 4), 16000.0, 3.0 / 16000.0, 0.004,
     [[1.0, 1.0, 1.0]], [[1.01, 1.0, 1.0], [1.0, 1.02, 1.01]]),
    ("one_tile_general_window", [3.0, 4.0, 2.5], [0.8] * 6, (6, 6, 6), 11025.0, 0.02, 0.003,
     [[1.2, 2.0, 1.1]], [[1.3, 2.2, 1.0]]),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_degenerate_shapes(oracle_mod, case, precision):
    name, L, beta, n, fs, t_max, t_w, src, rcv = case
    room = ism.Room(L, beta, n, 343.0, fs, t_max, t_w)
    _say(f"{name} {precision} nS={room.n_samples}")
    got = _host(room, src, rcv, precision)
    ref = _oracle(oracle_mod, room, src, rcv)
    assert np.all(np.isfinite(got)), "some output sample was not written"
    err = rel_err(got, ref)
    print(name, precision, "rel err", err.ravel(), flush=True)
    assert np.all(err <= (TOL_FP32 if precision == "fp32" else 2e-3))


def test_all_zero_rir(oracle_mod):
    # direct path 2.5 m away: 116.6 samples at 16 kHz; nS = 16 and W/2 = 32,
    # so the first tap of any image sits past the end of the RIR
    room = ism.Room([4.0, 5.0, 3.0], [0.9] * 6, (8, 8, 8), 343.0, 16000.0, 0.001, 0.004)
    src, rcv = [[1.0, 1.0, 1.0]], [[3.5, 1.0, 1.0]]
    _say(f"all-zero RIR nS={room.n_samples}")
    ref = _oracle(oracle_mod, room, src, rcv)
    assert np.all(ref == 0.0)
    got = _host(room, src, rcv)
    assert np.all(got == 0.0)


def test_identical_pairs_identical_rirs():
    import torch

    room = ism.Room([5.0, 4.0, 3.0], [0.85] * 6, ism.n_img_for_time([5.0, 4.0, 3.0], 343.0, 0.1), 343.0, 16000.0,
                    0.1, 0.004)
    rcv = np.array([[3.0, 2.5, 1.2], [1.5, 1.0, 2.0], [3.0, 2.5, 1.2], [3.0, 2.5, 1.2]], np.float32)
    _say("identical receivers")
    got = ism.simulate(room, np.array([[1.0, 1.0, 1.0]], np.float32), rcv)
    torch.cuda.synchronize()
    assert torch.equal(got[0, 0], got[0, 2]) and torch.equal(got[0, 0], got[0, 3])
    assert not torch.equal(got[0, 0], got[0, 1])


def test_maximum_samples_sparse_lattice(oracle_mod):
    """nS = ISM_MAX_SAMPLES exactly (1025 tiles, most without an image): a
    3 x 3 x 3 lattice whose taps sit at the start of a 16.4 s RIR."""
    fs = 16000.0
    room = ism.Room([3.0, 4.0, 2.5], [0.9] * 6, (3, 3, 3), 343.0, fs, ism.ISM_MAX_SAMPLES / fs, 0.004)
    assert room.n_samples == ism.ISM_MAX_SAMPLES
    src, rcv = [[1.0, 1.5, 1.0]], [[2.2, 3.1, 1.7]]
    _say(f"maximum nS = {room.n_samples}")
    got = _host(room, src, rcv)
    ref = _oracle(oracle_mod, room, src, rcv)
    assert np.all(np.isfinite(got))
    err = rel_err(got, ref)
    print("rel err", err.ravel(), flush=True)
    assert np.all(err <= TOL_FP32)


def test_maximum_images_per_axis(oracle_mod):
    """N = ISM_MAX_N_IMG images along one axis (2048 lattice indices, delays up
    to ~95 000 samples), one along the others."""
    room = ism.Room([1.0, 4.0, 3.0], [0.999] * 6, (ism.ISM_MAX_N_IMG, 1, 1), 343.0, 16000.0, 6.25, 0.004)
    src, rcv = [[0.3, 2.0, 1.5]], [[0.8, 2.5, 1.2]]
    _say(f"N = {room.n_img}, nS = {room.n_samples}")
    got = _host(room, src, rcv)
    ref = _oracle(oracle_mod, room, src, rcv)
    assert np.all(np.isfinite(got))
    err = rel_err(got, ref)
    print("rel err", err.ravel(), flush=True)
    assert np.all(err <= TOL_FP32)
