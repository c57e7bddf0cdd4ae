"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than its own formula:
closed forms, a brute-force image enumeration by successive wall reflections,
symmetries (reciprocity, mirror), scale invariances, and an independently
written direct summation on tiny lattices. A plausible slip in the oracle (a
swapped wall coefficient, an even/odd mix-up in Eq. (1), d*c/fs instead of
d*fs/c, a wrong window width, 2*pi instead of 4*pi, a wrong sinc cut-off) fails
at least one of them; tests/test_oracle_mutants.py plants such slips to check.
"""
import itertools
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# Host helpers (Sec. 4 helper functions, Eq. (7))
# ---------------------------------------------------------------------------

def test_n_samples_snaps_products_to_integers(oracle_mod):
    assert oracle_mod.n_samples(0.7, 16000) == 11200
    assert oracle_mod.n_samples(0.3, 16000) == 4800
    assert oracle_mod.n_samples(2.0, 48000) == 96000
    assert oracle_mod.n_samples(0.30001, 16000) == 4801  # 4800.16 -> ceil


def test_sabine_round_trip_and_infeasible(oracle_mod):
    rng = np.random.default_rng(5)
    for _ in range(50):
        L = rng.uniform(3, 10, 3)
        t60 = rng.uniform(0.5, 2.0)
        b = oracle_mod.beta_from_t60(L, t60)
        V = L.prod()
        S = np.array([L[1] * L[2], L[1] * L[2], L[0] * L[2], L[0] * L[2], L[0] * L[1], L[0] * L[1]])
        # Eq. (7) evaluated forwards with alpha_i = 1 - beta_i^2 gives back T60.
        assert abs(0.161 * V / np.sum(S * (1 - b ** 2)) - t60) < 1e-12 * t60
        assert np.all(b > 0) and np.all(b < 1)
    with pytest.raises(ValueError):
        oracle_mod.beta_from_t60([10, 10, 10], 0.1)  # alpha > 1


def test_sabine_golden_values(oracle_mod):
    # tests/golden/sabine.txt: uniform beta for the three single-room workloads.
    for line in open(os.path.join(GOLDEN, "sabine.txt")):
        if line.startswith("#") or not line.strip():
            continue
        Lx, Ly, Lz, t60, beta = map(float, line.split())
        assert abs(oracle_mod.beta_from_t60([Lx, Ly, Lz], t60)[0] - beta) < 5e-6


def test_time_for_attenuation_matches_exponential_decay(oracle_mod):
    for t60 in (0.3, 0.7, 1.9):
        for att in (13.0, 20.0, 60.0):
            t = oracle_mod.time_for_attenuation(t60, att)
            # energy decays by 60 dB over T60: 10 log10 E(t)/E(0) = -60 t / T60
            assert abs(-60.0 * t / t60 + att) < 1e-12


def _all_images_brute(L, src, rcv, reach):
    """Image positions by the Allen-Berkley pair formula 2 m L +- x, m in a wide range."""
    out = []
    m_rng = range(-reach, reach + 1)
    for mx, my, mz in itertools.product(m_rng, m_rng, m_rng):
        for sx, sy, sz in itertools.product((1, -1), repeat=3):
            p = np.array([2 * mx * L[0] + sx * src[0], 2 * my * L[1] + sy * src[1], 2 * mz * L[2] + sz * src[2]])
            out.append(p)
    return np.array(out)


def test_n_img_for_time_loses_no_reflection(oracle_mod):
    rng = np.random.default_rng(11)
    for _ in range(6):
        L = rng.uniform(1.0, 3.0, 3)
        src = rng.uniform(0.1, 1.0, 3) * L
        rcv = rng.uniform(0.1, 1.0, 3) * L
        t = rng.uniform(0.01, 0.03)
        c = 343.0
        n = oracle_mod.n_img_for_time(L, c, t)
        idx, vals = oracle_mod.image_list(L, np.ones(6), n, c, 16000, t, 0.004, src, rcv)
        lattice_d = np.sort(vals[:, 1][vals[:, 1] <= c * t])
        pos = _all_images_brute(L, _f32(src), _f32(rcv), reach=8)
        d = np.linalg.norm(pos - _f32(rcv), axis=1)
        brute_d = np.sort(d[d <= c * t])
        assert len(brute_d) == len(lattice_d)
        np.testing.assert_allclose(lattice_d, brute_d, rtol=0, atol=1e-9)


# ---------------------------------------------------------------------------
# Closed forms of a single path (Eq. (3), (4), (6))
# ---------------------------------------------------------------------------

def test_exact_integer_delay_gives_single_sample(oracle_mod):
    # tests/golden/single_sample.txt: c = 256 m/s, fs = 16384 Hz (1/64 m per
    # sample), d = 2 m -> delay exactly 128 samples, free field (beta = 0).
    rows = [l.split() for l in open(os.path.join(GOLDEN, "single_sample.txt")) if l.strip() and not l.startswith("#")]
    kv = {r[0]: [float(x) for x in r[1:]] for r in rows}
    h = oracle_mod.rir(kv["L"], np.zeros(6), [int(v) for v in kv["n_img"]], kv["c"][0], kv["fs"][0], kv["t_max"][0],
                       kv["t_w"][0], kv["src"], kv["rcv"])[0, 0]
    k0 = int(kv["k_peak"][0])
    assert h[k0] == pytest.approx(kv["h_peak"][0], rel=1e-15)
    assert abs(h[k0] - 1.0 / (8.0 * math.pi)) < 1e-17
    others = np.delete(h, k0)
    assert np.max(np.abs(others)) < 1e-15


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_free_field_closed_form(oracle_mod, seed):
    # beta = 0: every image but n = 0 has gain 0 (0^e, e >= 1); 0^0 = 1 keeps the
    # direct path. h[k] = w(k - x) sinc(k - x) / (4 pi d) with numpy's sinc and the
    # Hann window written as cos^2 (same function, different evaluation).
    rng = np.random.default_rng(seed)
    L = np.array([4.0, 5.0, 3.0])
    src = _f32(rng.uniform(0.5, 1.0, 3) * L / 2)
    rcv = _f32(src + rng.uniform(-0.4, 0.4, 3))  # short path: taps before k = 0 are dropped
    if seed == 2:
        rcv = _f32(rng.uniform(0.5, L - 0.5))
    c, fs, t_w, t_max = 343.0, 16000.0, 0.004, 0.1
    n = (6, 6, 6)
    h = oracle_mod.rir(L, np.zeros(6), n, c, fs, t_max, t_w, src, rcv)[0, 0]
    d = np.linalg.norm(rcv - src)
    x = d * fs / c
    W = t_w * fs
    k = np.arange(len(h))
    v = k - x
    ref = np.where(np.abs(v) < W / 2, np.cos(np.pi * v / W) ** 2 * np.sinc(v), 0.0) / (4 * np.pi * d)
    np.testing.assert_allclose(h, ref, rtol=0, atol=1e-14 * np.max(np.abs(ref)))
    assert np.count_nonzero(h) == np.count_nonzero(np.abs(v) < W / 2)


# ---------------------------------------------------------------------------
# Lattice: positions, wall exponents and wall naming by successive reflections
# ---------------------------------------------------------------------------

def _bfs_images(L, beta, src, max_order):
    """Images by reflecting the source across the faces of mirrored room copies.

    Cell (i, j, k) is the copy of the room occupying [i Lx, (i+1) Lx] x ...; the
    copy is flipped along an axis when its index is odd. Its face at the low end
    of an axis is the room's wall at 0 when not flipped and the wall at L when
    flipped, and the other way round for the high face. Crossing a face
    multiplies the path gain by that wall's coefficient.
    """
    start = (0, 0, 0)
    seen = {start: (np.array(src, dtype=np.float64), 1.0)}
    frontier = [start]
    for _ in range(max_order):
        nxt = []
        for cell in frontier:
            pos, g = seen[cell]
            for a in range(3):
                for step in (-1, 1):
                    nc = list(cell)
                    nc[a] += step
                    nc = tuple(nc)
                    if nc in seen:
                        continue
                    i = cell[a]
                    flipped = (i % 2) != 0
                    if step == 1:
                        plane = (i + 1) * L[a]
                        wall = 0 if flipped else 1
                    else:
                        plane = i * L[a]
                        wall = 1 if flipped else 0
                    p = pos.copy()
                    p[a] = 2 * plane - p[a]
                    seen[nc] = (p, g * beta[2 * a + wall])
                    nxt.append(nc)
        frontier = nxt
    return seen


@pytest.mark.parametrize("beta", [[0.9, 0.7, 0.8, 0.6, 0.5, 0.95], [-0.9, 0.7, 0.8, -0.6, 0.5, -0.95]])
def test_lattice_matches_reflection_bfs(oracle_mod, beta):
    L = np.array([3.0, 4.0, 2.5])
    src = _f32([0.7, 1.9, 2.1])
    rcv = _f32([2.2, 0.6, 1.3])
    order = 4
    bfs = _bfs_images(L, beta, src, order)
    counts = np.bincount([sum(abs(c) for c in cell) for cell in bfs])
    assert list(counts) == [1, 6, 18, 38, 66]
    idx, vals = oracle_mod.image_list(L, beta, (10, 10, 10), 343.0, 16000.0, 0.1, 0.004, src, rcv)
    got = {tuple(int(v) for v in i): val for i, val in zip(idx, vals) if np.sum(np.abs(i)) <= order}
    assert set(got) == set(bfs)
    for cell, (pos, g) in bfs.items():
        gain, d, x, A = got[cell]
        assert gain == pytest.approx(g, rel=1e-14, abs=0)
        assert d == pytest.approx(np.linalg.norm(rcv - pos), rel=1e-13)
        assert x == pytest.approx(d * 16000.0 / 343.0, rel=1e-14)
        assert A == pytest.approx(g / (4 * np.pi * d), rel=1e-14)


# ---------------------------------------------------------------------------
# Symmetries and scale invariances of the whole RIR
# ---------------------------------------------------------------------------

def _case(rng, n_img):
    L = _f32(rng.uniform(3, 6, 3))
    beta = rng.uniform(-0.95, 0.95, 6)
    src = _f32(rng.uniform(0.5, L - 0.5))
    rcv = _f32(rng.uniform(0.5, L - 0.5))
    return L, beta, n_img, src, rcv


@pytest.mark.parametrize("n_img", [(6, 10, 14), (10, 6, 6)])
def test_reciprocity(oracle_mod, n_img):
    rng = np.random.default_rng(sum(n_img))
    L, beta, n, src, rcv = _case(rng, n_img)
    a = oracle_mod.rir(L, beta, n, 343.0, 16000.0, 0.06, 0.004, src, rcv)[0, 0]
    b = oracle_mod.rir(L, beta, n, 343.0, 16000.0, 0.06, 0.004, rcv, src)[0, 0]
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * np.max(np.abs(a)))


def test_reciprocity_fails_for_n_multiple_of_four(oracle_mod):
    # With N = 0 (mod 4) the even images are not symmetric under n -> -n.
    rng = np.random.default_rng(3)
    L, beta, n, src, rcv = _case(rng, (8, 8, 8))
    a = oracle_mod.rir(L, beta, n, 343.0, 16000.0, 0.06, 0.004, src, rcv)[0, 0]
    b = oracle_mod.rir(L, beta, n, 343.0, 16000.0, 0.06, 0.004, rcv, src)[0, 0]
    assert np.max(np.abs(a - b)) > 1e-6 * np.max(np.abs(a))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mirror_symmetry_with_swapped_walls(oracle_mod, axis):
    rng = np.random.default_rng(40 + axis)
    L, beta, n, src, rcv = _case(rng, (7, 9, 11))
    a = oracle_mod.rir(L, beta, n, 343.0, 16000.0, 0.06, 0.004, src, rcv)[0, 0]
    src2, rcv2, beta2 = src.copy(), rcv.copy(), np.array(beta, dtype=np.float64)
    src2[axis] = L[axis] - src[axis]
    rcv2[axis] = L[axis] - rcv[axis]
    beta2[2 * axis], beta2[2 * axis + 1] = beta[2 * axis + 1], beta[2 * axis]
    b = oracle_mod.rir(L, beta2, n, 343.0, 16000.0, 0.06, 0.004, src2, rcv2)[0, 0]
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-11 * np.max(np.abs(a)))


def test_scale_invariances(oracle_mod):
    rng = np.random.default_rng(9)
    L, beta, n, src, rcv = _case(rng, (6, 6, 10))
    c, fs, t_max, t_w = 343.0, 16000.0, 0.05, 0.004
    h = oracle_mod.rir(L, beta, n, c, fs, t_max, t_w, src, rcv)[0, 0]
    # (i) lengths and c scaled by a: same delays in samples, amplitudes / a.
    h1 = oracle_mod.rir(2 * L, beta, n, 2 * c, fs, t_max, t_w, 2 * src, 2 * rcv)[0, 0]
    np.testing.assert_allclose(h1, h / 2, rtol=0, atol=1e-13 * np.max(np.abs(h)))
    # (ii) c and fs scaled by b, T_w and T_max divided by b: same samples.
    h2 = oracle_mod.rir(L, beta, n, 2 * c, 2 * fs, t_max / 2, t_w / 2, src, rcv)[0, 0]
    np.testing.assert_allclose(h2, h, rtol=0, atol=1e-13 * np.max(np.abs(h)))


# ---------------------------------------------------------------------------
# Whole RIR by an independently written direct summation (tiny lattice)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_tiny_lattice_direct_summation(oracle_mod, seed):
    rng = np.random.default_rng(100 + seed)
    L = _f32(rng.uniform(2, 4, 3))
    beta = rng.uniform(-0.9, 0.9, 6)
    src = _f32(rng.uniform(0.3, L - 0.3))
    rcv = _f32(rng.uniform(0.3, L - 0.3))
    c, fs, t_w = 343.0, 16000.0, 0.004
    t_max = 0.04
    n = (3, 3, 3)  # n in {-1, 0, 1}^3: reflection order <= 3, all reached by the BFS
    bfs = _bfs_images(L, beta, src, 3)
    nS = oracle_mod.n_samples(t_max, fs)
    W = t_w * fs
    ref = np.zeros(nS)
    k = np.arange(nS)
    for cell, (pos, g) in bfs.items():
        if max(abs(v) for v in cell) > 1:
            continue
        d = np.linalg.norm(rcv - pos)
        v = k - d * fs / c
        ref += np.where(np.abs(v) < W / 2, np.cos(np.pi * v / W) ** 2 * np.sinc(v), 0.0) * g / (4 * np.pi * d)
    h = oracle_mod.rir(L, beta, n, c, fs, t_max, t_w, src, rcv)[0, 0]
    # different summation order: agreement to a few units of double rounding
    np.testing.assert_allclose(h, ref, rtol=0, atol=1e-12 * np.max(np.abs(ref)))


def test_tap_count_matches_image_list(oracle_mod):
    rng = np.random.default_rng(21)
    L, beta, n, src, rcv = _case(rng, (10, 10, 14))
    c, fs, t_max, t_w = 343.0, 16000.0, 0.05, 0.004
    idx, vals = oracle_mod.image_list(L, beta, n, c, fs, t_max, t_w, src, rcv)
    nS = oracle_mod.n_samples(t_max, fs)
    W = t_w * fs
    k = np.arange(nS)
    brute = sum(int(np.count_nonzero(np.abs(k - x) < W / 2)) for x in vals[:, 2])
    assert oracle_mod.count_taps(L, beta, n, c, fs, t_max, t_w, src, rcv) == brute


def test_window_restriction_equals_full_rir(oracle_mod):
    rng = np.random.default_rng(8)
    L, beta, n, src, rcv = _case(rng, (6, 6, 6))
    full = oracle_mod.rir(L, beta, n, 343.0, 16000.0, 0.05, 0.004, src, rcv)[0, 0]
    part = oracle_mod.rir(L, beta, n, 343.0, 16000.0, 0.05, 0.004, src, rcv, k_begin=123, k_end=517)[0, 0]
    assert np.array_equal(full[123:517], part)
