"""Pins of the lookup-table oracle (Sec. 3.5, Eq. (9)) against facts that do
not come from the oracle itself: the table holds Eq. (6) at Q points per
sample (checked against numpy's sinc and the Hann window), the sinc's zeros at
the integers, linearity between neighbouring entries, the error bound of
linear interpolation, h^2/8 max|s''| with h = 1/Q, and, for whole RIRs, the
same bound summed over the images that reach each sample, against the exact
oracle (itself pinned in test_oracle_pins.py)."""
import numpy as np
import pytest

Q = 16


def _eq6(v, W):
    """Eq. (6) sampled at offset v (samples): Hann window of W samples times sinc."""
    v = np.asarray(v, dtype=np.float64)
    return np.where(np.abs(v) < W / 2, 0.5 * (1.0 + np.cos(2.0 * np.pi * v / W)) * np.sinc(v), 0.0)


def _bound(W):
    """h^2/8 max|s''| for s = Eq. (6), h = 1/Q; max|s''| from a fine grid
    (second differences at spacing 1e-3, 2 % margin)."""
    d = 1e-3
    v = np.arange(-W / 2 + d, W / 2 - d, d)
    s2 = (_eq6(v + d, W) - 2 * _eq6(v, W) + _eq6(v - d, W)) / d**2
    return (1.0 / Q) ** 2 / 8.0 * np.max(np.abs(s2)) * 1.02


@pytest.mark.parametrize("W", [32, 64, 96, 128])
def test_table_points_are_eq6(oracle_mod, W):
    n = np.arange(-Q * W // 2 + 1, Q * W // 2)
    v = n / Q
    got = oracle_mod.lut_taps(v, W, Q)
    assert np.max(np.abs(got - _eq6(v, W))) <= 1e-15


@pytest.mark.parametrize("W", [32, 64])
def test_integer_offsets_hit_the_sinc_zeros(oracle_mod, W):
    k = np.arange(-W // 2 + 1, W // 2)
    got = oracle_mod.lut_taps(k.astype(np.float64), W, Q)
    assert got[k == 0][0] == 1.0
    assert np.max(np.abs(got[k != 0])) <= 1e-15  # sin(pi k) in double: a few ulps of pi k
    # at and beyond the window's ends nothing is added
    assert np.all(oracle_mod.lut_taps(np.array([-W / 2, W / 2, W / 2 + 0.3]), W, Q) == 0.0)


def test_linear_between_entries(oracle_mod):
    W = 64
    rng = np.random.default_rng(3)
    n = rng.integers(-Q * W // 2, Q * W // 2 - 1, size=500)
    a = rng.random(500)
    v = (n + a) / Q
    want = (1 - a) * _eq6(n / Q, W) + a * _eq6((n + 1) / Q, W)
    got = oracle_mod.lut_taps(v, W, Q)
    assert np.max(np.abs(got - want)) <= 1e-14


@pytest.mark.parametrize("W", [32, 64, 128])
def test_interpolation_error_bound(oracle_mod, W):
    rng = np.random.default_rng(W)
    v = rng.uniform(-W / 2, W / 2, 20000)
    err = np.abs(oracle_mod.lut_taps(v, W, Q) - _eq6(v, W))
    b = _bound(W)
    assert b < 1.7e-3
    assert np.max(err) <= b
    # the table is really interpolated (a nearest-entry read would break the
    # bound; an exact evaluation would leave no error at all)
    assert np.max(err) >= 0.3 * b


def test_rir_within_the_summed_bound(oracle_mod):
    L, beta, n = [4.0, 5.0, 3.0], [0.9, 0.85, 0.8, 0.9, 0.7, 0.95], (8, 8, 10)
    fs, t_max, t_w, c = 16000.0, 0.06, 0.004, 343.0
    src, rcv = [[1.2, 2.0, 1.5]], [[3.1, 1.1, 2.2]]
    W = t_w * fs
    exact = oracle_mod.rir(L, beta, n, c, fs, t_max, t_w, src, rcv)[0, 0]
    lut = oracle_mod.rir(L, beta, n, c, fs, t_max, t_w, src, rcv, lut_q=Q)[0, 0]
    _, vals = oracle_mod.image_list(L, beta, n, c, fs, t_max, t_w, src, rcv)
    x, A = vals[:, 2], vals[:, 3]
    k = np.arange(exact.size)
    reach = np.abs(k[:, None] - x[None, :]) < W / 2
    bound = _bound(W) * (reach * np.abs(A)[None, :]).sum(axis=1) + 1e-15
    diff = np.abs(lut - exact)
    assert np.all(diff <= bound)
    assert np.max(diff) > 0.05 * np.max(bound)


def test_bad_table_size(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.lut_taps([0.0], 64.3, Q)
