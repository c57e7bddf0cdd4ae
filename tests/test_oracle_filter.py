"""Pins of the moving-source oracle (Sec. 3.4) on the CPU: the overlap-add of
segment convolutions against properties that do not reuse its code path."""
import numpy as np


def test_same_filter_everywhere_is_one_convolution(oracle_mod):
    """Segments partition the signal and convolution is linear: with the same
    RIR at every point the overlap-add is the convolution of the whole signal."""
    rng = np.random.default_rng(0)
    x = rng.standard_normal(1000)
    h = rng.standard_normal(37)
    rirs = np.broadcast_to(h, (7, 2, 37)).copy()
    y = oracle_mod.filter_trajectory(x, rirs)
    full = np.array([sum(x[i] * h[n - i] for i in range(max(0, n - 36), min(n, 999) + 1)) for n in range(1036)])
    np.testing.assert_allclose(y[0], full, rtol=0, atol=1e-12)
    np.testing.assert_allclose(y[1], full, rtol=0, atol=1e-12)


def test_impulse_in_a_segment_picks_that_points_rir(oracle_mod):
    rng = np.random.default_rng(1)
    n_x, n_pos, n_rir = 100, 4, 30  # segments of 25 samples
    rirs = rng.standard_normal((n_pos, 3, n_rir))
    for p, off in ((0, 0), (1, 25), (2, 57), (3, 99)):
        x = np.zeros(n_x)
        x[off] = 2.0
        y = oracle_mod.filter_trajectory(x, rirs)
        want = np.zeros((3, n_x + n_rir - 1))
        want[:, off:off + n_rir] = 2.0 * rirs[p]
        np.testing.assert_array_equal(y, want)


def test_one_sample_per_point_brute_force(oracle_mod):
    """n_pos = n_x: every input sample has its own filter,
    y[m][n] = sum_i x[i] h_i[m][n - i]."""
    rng = np.random.default_rng(2)
    n_x, n_mic, n_rir = 20, 2, 9
    x = rng.standard_normal(n_x)
    rirs = rng.standard_normal((n_x, n_mic, n_rir))
    y = oracle_mod.filter_trajectory(x, rirs)
    for m in range(n_mic):
        for n in range(n_x + n_rir - 1):
            ref = sum(x[i] * rirs[i, m, n - i] for i in range(n_x) if 0 <= n - i < n_rir)
            assert abs(y[m, n] - ref) < 1e-12


def test_ragged_last_segment_and_linearity(oracle_mod):
    rng = np.random.default_rng(3)
    n_x, n_pos, n_rir = 103, 5, 17  # segments of 21, the last of 19
    rirs = rng.standard_normal((n_pos, 2, n_rir))
    a, b = rng.standard_normal(n_x), rng.standard_normal(n_x)
    ya, yb = oracle_mod.filter_trajectory(a, rirs), oracle_mod.filter_trajectory(b, rirs)
    np.testing.assert_allclose(oracle_mod.filter_trajectory(a - 3.0 * b, rirs), ya - 3.0 * yb, rtol=0, atol=1e-12)
    # the last input sample (segment 4) is filtered by point 4
    x = np.zeros(n_x)
    x[-1] = 1.0
    np.testing.assert_array_equal(oracle_mod.filter_trajectory(x, rirs)[:, n_x - 1:], rirs[4])


def test_filter_samples_equal_the_whole_filter(oracle_mod):
    """The one-by-one outputs used at sizes where the whole filter is too slow
    agree with the overlap-add of the whole signal at every output sample."""
    rng = np.random.default_rng(21)
    x = rng.standard_normal(997)
    rirs = rng.standard_normal((9, 2, 140))
    y = oracle_mod.filter_trajectory(x, rirs)
    n = np.arange(y.shape[1])
    for m in range(2):
        np.testing.assert_allclose(oracle_mod.filter_samples(x, rirs, m, n), y[m], rtol=0, atol=1e-12)
