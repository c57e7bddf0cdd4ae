"""Pins of the diffuse-tail oracle (Sec. 2.2, Eq. (8); Sec. 3.3) on the CPU.

The noise generator is pinned bit for bit by the published Philox4x32-10
known-answer vectors (tests/golden/philox4x32_10_kat.txt) and statistically
(uniform, balanced, independent words; a single flipped counter bit changes
about half of the output bits), the logistic transform by its moments and
distribution function, the envelope by its closed form (-60 dB of power at
t_diff + T60) and the level estimate by an input whose energy follows the
envelope exactly.
"""
import math
import os

import numpy as np
import pytest


N_WORDS = 1 << 18


@pytest.fixture(scope="module")
def orc(oracle_mod):
    return oracle_mod


def _words(orc, seed=11, rir=0, n=N_WORDS):
    return orc.noise_bits(seed, rir, np.arange(n)).astype(np.uint64)


def _kat_vectors():
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if line:
                rows.append([int(v, 16) for v in line])
    assert len(rows) == 3 and all(len(r) == 10 for r in rows)
    return rows


def test_philox_known_answer_vectors(orc):
    """The generator reproduces the published known-answer vectors of
    Philox4x32-10 (Salmon et al., SC'11), word for word."""
    for row in _kat_vectors():
        ctr, key, expect = row[0:4], row[4:6], row[6:10]
        got = orc.philox4x32_10([np.array([c], dtype=np.uint64) for c in ctr], key)
        assert [int(g[0]) for g in got] == expect, (ctr, key, [hex(int(g[0])) for g in got])


def test_philox_known_answer_vectors_catch_plausible_slips(orc):
    """Plausible mistakes in a Philox implementation (high and low product
    halves swapped, the key bumped before the first round, nine rounds) give
    outputs that differ from the known answers."""
    M, Wk, mask = (0xD2511F53, 0xCD9E8D57), (0x9E3779B9, 0xBB67AE85), 0xFFFFFFFF

    def variant(ctr, key, swap=False, bump_first=False, rounds=10):
        c = list(ctr)
        k0, k1 = key
        for r in range(rounds):
            if r > 0 or bump_first:
                k0, k1 = (k0 + Wk[0]) & mask, (k1 + Wk[1]) & mask
            p0, p1 = M[0] * c[0], M[1] * c[2]
            h0, l0, h1, l1 = p0 >> 32, p0 & mask, p1 >> 32, p1 & mask
            if swap:
                h0, l0, h1, l1 = l0, h0, l1, h1
            c = [h1 ^ c[1] ^ k0, l1, h0 ^ c[3] ^ k1, l0]
        return c

    for row in _kat_vectors():
        ctr, key, expect = row[0:4], row[4:6], row[6:10]
        assert variant(ctr, key) == expect  # the plain definition, written out again
        assert variant(ctr, key, swap=True) != expect
        assert variant(ctr, key, bump_first=True) != expect
        assert variant(ctr, key, rounds=9) != expect


def test_philox_words_uniform_and_balanced(orc):
    x = _words(orc)
    # 256 equiprobable bins of the top byte: chi-square with 255 degrees of freedom
    counts = np.bincount((x >> np.uint64(24)).astype(np.int64), minlength=256)
    expect = len(x) / 256.0
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    assert 180.0 < chi2 < 340.0, chi2  # ~ +-4.7 sigma around 255
    # every bit set in half of the words
    bits = np.array([np.mean((x >> np.uint64(b)) & np.uint64(1)) for b in range(32)])
    assert np.all(np.abs(bits - 0.5) < 5.0 * 0.5 / math.sqrt(len(x))), bits


def test_philox_streams_independent(orc):
    a = _words(orc, seed=11, rir=0).astype(np.float64)
    b = _words(orc, seed=11, rir=1).astype(np.float64)
    c = _words(orc, seed=12, rir=0).astype(np.float64)
    tol = 5.0 / math.sqrt(N_WORDS)
    assert abs(np.corrcoef(a, b)[0, 1]) < tol
    assert abs(np.corrcoef(a, c)[0, 1]) < tol
    assert abs(np.corrcoef(a[:-1], a[1:])[0, 1]) < tol  # neighbouring samples
    assert abs(np.corrcoef(a[:-4], a[4:])[0, 1]) < tol  # same word, next counter


def test_philox_avalanche(orc):
    """Flipping one counter bit changes about 16 of the 32 bits of every word."""
    rng = np.random.default_rng(3)
    ctr = [rng.integers(0, 1 << 32, 4096, dtype=np.uint64) for _ in range(4)]
    base = orc.philox4x32_10(ctr, (0x1234, 0x5678))
    for lane in range(4):
        for bit in (0, 13, 31):
            flipped = list(ctr)
            flipped[lane] = ctr[lane] ^ np.uint64(1 << bit)
            out = orc.philox4x32_10(flipped, (0x1234, 0x5678))
            for w in range(4):
                d = np.bitwise_xor(base[w], out[w])
                changed = np.unpackbits(d.view(np.uint8)).reshape(-1, 32).sum(axis=1)
                assert abs(changed.mean() - 16.0) < 0.5, (lane, bit, w, changed.mean())


def test_logistic_transform_moments_and_cdf(orc):
    z = orc.logistic_from_bits(_words(orc, seed=5))
    n = len(z)
    assert abs(z.mean()) < 5.0 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 0.02
    m4 = np.mean((z - z.mean()) ** 4) / z.var() ** 2
    assert abs((m4 - 3.0) - 1.2) < 0.15  # logistic excess kurtosis 6/5
    # Kolmogorov-Smirnov distance to the logistic law of scale sqrt(3)/pi
    s = math.sqrt(3.0) / math.pi
    zs = np.sort(z)
    cdf = 1.0 / (1.0 + np.exp(-zs / s))
    ks = np.max(np.abs(cdf - (np.arange(1, n + 1) / n)))
    assert ks < 1.63 / math.sqrt(n)  # 1 % critical value
    # the transform is the logistic quantile: exact at the middle word
    assert orc.logistic_from_bits(np.array([2 ** 31 - 1]))[0] == pytest.approx(0.0, abs=1e-9)


def test_envelope_closed_form(orc):
    fs, t_diff, t60 = 16000.0, 0.25, 0.8
    k = np.array([4000, 4000 + 12800])  # t_diff and t_diff + T60
    env = orc.envelope(k, fs, t_diff, t60)
    assert env[0] == pytest.approx(1.0, rel=1e-15)
    assert env[1] == pytest.approx(1e-6, rel=1e-12)  # -60 dB of power after T60


def test_envelope_level_of_an_exact_envelope(orc):
    fs, t_diff, t60, c = 16000.0, 0.3, 1.1, 2.5e-3
    k_diff = orc.n_samples(t_diff, fs)
    k = np.arange(k_diff)
    sign = np.where(np.random.default_rng(1).random(k_diff) < 0.5, -1.0, 1.0)
    h = sign * np.sqrt(c * orc.envelope(k, fs, t_diff, t60))
    assert orc.envelope_level(h[None], fs, t_diff, t60)[0] == pytest.approx(c, rel=1e-12)
    k0, k1 = orc.diffuse_window(k_diff)
    assert (k0, k1) == (k_diff - k_diff // 5, k_diff)


def test_diffuse_rir_parts(orc):
    """ISM part = the ISM RIR up to t_diff; the tail decays 60 dB per T60."""
    L, t60, fs, t_w = [4.0, 5.0, 3.0], 0.9, 16000.0, 0.004
    beta = orc.beta_from_t60(L, t60)
    t_diff, t_max = 0.12, 0.9
    n = orc.n_img_for_time(L, 343.0, t_diff)
    src, rcv = [[1.2, 2.0, 1.5]], [[2.9, 3.1, 1.2]]
    h = orc.diffuse_rir(L, beta, n, 343.0, fs, t_max, t_w, t_diff, t60, 9, src, rcv)
    k_diff = orc.n_samples(t_diff, fs)
    assert h.shape == (1, 1, orc.n_samples(t_max, fs))
    ism = orc.rir(L, beta, n, 343.0, fs, t_diff, t_w, src, rcv)
    assert np.array_equal(h[..., :k_diff], ism)
    tail = h[0, 0, k_diff:]
    # energy per 50 ms block against time: slope -6 / T60 decades per second
    blk = 800
    nb = len(tail) // blk
    e = np.log10(np.mean(tail[: nb * blk].reshape(nb, blk) ** 2, axis=1))
    t = (k_diff + blk * (np.arange(nb) + 0.5)) / fs
    slope = np.polyfit(t, e, 1)[0]
    assert slope == pytest.approx(-6.0 / t60, rel=0.05)
    # level: the tail's power just after t_diff matches the ISM window's
    A = orc.envelope_level(ism, fs, t_diff, t60)[0, 0]
    assert np.mean(tail[:blk] ** 2) / np.mean(orc.envelope(np.arange(k_diff, k_diff + blk), fs, t_diff, t60)) \
        == pytest.approx(A, rel=0.15)
