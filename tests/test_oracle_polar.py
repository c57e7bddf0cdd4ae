"""Pins of the directional-receiver oracle (receiver polar patterns: the
paper's library takes a pattern and an orientation per receiver, Sec. 4, and
gives no formula; the reading is the first-order family a + (1 - a) cos(theta)).

Pinned against facts outside the oracle: the direct path in free field against
numpy geometry and Eq. (4)-(6) written with np.sinc; the omni pattern equals
the plain RIR (itself pinned in test_oracle_pins.py); back-to-back receivers
add up to 2a times the omni RIR (the cos terms cancel image by image);
an orientation's length does not matter."""
import numpy as np
import pytest

ROOM = dict(L=[4.0, 5.0, 3.0], c=343.0, fs=16000.0, t_max=0.03, t_w=0.004)


def _direct(src, rcv, orient, a):
    """Free-field direct path: A g(theta) times the windowed sinc of Eq. (6)."""
    src, rcv, orient = (np.asarray(v, dtype=np.float32).astype(np.float64) for v in (src, rcv, orient))
    d_vec = src - rcv
    d = np.linalg.norm(d_vec)
    cos_t = d_vec @ orient / (d * np.linalg.norm(orient))
    x = d / ROOM["c"] * ROOM["fs"]
    W = ROOM["t_w"] * ROOM["fs"]
    k = np.arange(int(np.ceil(ROOM["t_max"] * ROOM["fs"])))
    v = k - x
    taps = np.where(np.abs(v) < W / 2, 0.5 * (1 + np.cos(2 * np.pi * v / W)) * np.sinc(v), 0.0)
    return (a + (1 - a) * cos_t) / (4 * np.pi * d) * taps


@pytest.mark.parametrize("a", [0.0, 0.25, 0.5, 1.0])
def test_free_field_direct_path(oracle_mod, a):
    src = [1.0, 2.0, 1.5]
    rcvs = [[3.0, 2.0, 1.5], [2.0, 4.0, 1.0], [1.5, 1.0, 2.5]]
    orients = [[-1.0, 0.0, 0.0],   # facing the source: g = 1
               [0.3, 1.0, -0.2],   # facing away, oblique
               [0.0, 0.0, 1.0]]    # oblique
    h = oracle_mod.rir_polar(ROOM["L"], [0.0] * 6, (1, 1, 1), ROOM["c"], ROOM["fs"], ROOM["t_max"], ROOM["t_w"],
                             [src], rcvs, orients, a)[0]
    for r, (rcv, o) in enumerate(zip(rcvs, orients)):
        want = _direct(src, rcv, o, a)
        assert np.max(np.abs(h[r] - want)) <= 1e-13 * np.max(np.abs(_direct(src, rcv, o, 1.0)))
    # facing the source: full gain whatever the pattern
    assert np.isclose(np.max(np.abs(h[0])), np.max(np.abs(_direct(src, rcvs[0], [1, 0, 0], 1.0))), rtol=1e-12)


def test_omni_equals_plain_rir(oracle_mod):
    args = (ROOM["L"], [0.9, -0.8, 0.7, 0.85, 0.6, 0.95], (8, 6, 10), ROOM["c"], ROOM["fs"], ROOM["t_max"],
            ROOM["t_w"], [[1.2, 3.1, 0.7]])
    rcv = [[2.5, 1.5, 2.0], [3.3, 4.1, 1.1]]
    h = oracle_mod.rir(*args, rcv)
    hp = oracle_mod.rir_polar(*args, rcv, [[0.2, -1.0, 0.4], [1.0, 1.0, 1.0]], 1.0)
    assert np.array_equal(h, hp)


@pytest.mark.parametrize("a", [0.0, 0.3, 0.5])
def test_back_to_back_sum(oracle_mod, a):
    args = (ROOM["L"], [0.9, 0.8, 0.7, 0.85, 0.6, 0.95], (10, 8, 10), ROOM["c"], ROOM["fs"], ROOM["t_max"],
            ROOM["t_w"], [[1.2, 3.1, 0.7]])
    rcv = [[2.5, 1.5, 2.0]]
    o = np.array([[0.3, -0.5, 0.8]])
    h = oracle_mod.rir(*args, rcv)
    front = oracle_mod.rir_polar(*args, rcv, o, a)
    back = oracle_mod.rir_polar(*args, rcv, -o, a)
    assert np.max(np.abs(front + back - 2 * a * h)) <= 1e-12 * np.max(np.abs(h))
    if a < 1.0:
        assert np.max(np.abs(front - back)) > 0.1 * np.max(np.abs(h))


def test_orientation_length_is_irrelevant(oracle_mod):
    args = (ROOM["L"], [0.9] * 6, (6, 6, 6), ROOM["c"], ROOM["fs"], ROOM["t_max"], ROOM["t_w"], [[1.2, 3.1, 0.7]])
    rcv = [[2.5, 1.5, 2.0]]
    h1 = oracle_mod.rir_polar(*args, rcv, [[0.5, 0.25, -0.5]], 0.5)
    h2 = oracle_mod.rir_polar(*args, rcv, [[2.0, 1.0, -2.0]], 0.5)
    assert np.max(np.abs(h1 - h2)) <= 1e-13 * np.max(np.abs(h1))


def test_bad_arguments(oracle_mod):
    args = (ROOM["L"], [0.9] * 6, (4, 4, 4), ROOM["c"], ROOM["fs"], ROOM["t_max"], ROOM["t_w"], [[1.2, 3.1, 0.7]])
    with pytest.raises(ValueError):
        oracle_mod.rir_polar(*args, [[2.5, 1.5, 2.0]], [[0.0, 0.0, 0.0]], 0.5)
    with pytest.raises(ValueError):
        oracle_mod.rir_polar(*args, [[2.5, 1.5, 2.0]], [[1.0, 0.0, 0.0]], 1.5)
