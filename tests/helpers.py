"""Shared test utilities: oracle-side room construction and error metrics."""
import numpy as np


def oracle_room_args(oracle_mod, w):
    """(L, beta, n_img, c, fs, t_max, t_w) of a workload, built with the oracle's helpers only."""
    beta = oracle_mod.beta_from_t60(w.room, w.t60)
    if w.beta_jitter is not None:
        beta = np.minimum(beta * np.asarray(w.beta_jitter), 0.999)
    n = oracle_mod.n_img_for_time(w.room, w.c, w.t_max)
    return (w.room, beta, n, w.c, w.fs, w.t_max, w.t_w)


def rel_err(got, ref, peak=None):
    """max |got - ref| / max |ref| along the last axis (per RIR)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if peak is None:
        peak = np.max(np.abs(ref), axis=-1)
    return np.max(np.abs(got - ref), axis=-1) / peak


def oracle_peak(oracle_mod, args, src, rcv, n_samples, early=3000):
    """Per-RIR peak max|h| of the FP64 oracle, taken over the early part
    [0, min(nS, early)) of the RIR, which holds the direct path and the first
    reflections (the RIR decays after them). Parity errors are divided by this
    oracle figure, never by a peak of the GPU output."""
    k1 = min(int(n_samples), int(early))
    ref = oracle_mod.rir(*args, src, rcv, k_begin=0, k_end=k1)
    return np.max(np.abs(ref), axis=-1), ref


def assert_no_value_above_peak(got, peak, tol):
    """No GPU sample anywhere in the RIR may exceed the oracle's peak by more
    than the parity tolerance (catches a spurious large value outside the
    compared windows)."""
    got = np.asarray(got, dtype=np.float64)
    top = np.max(np.abs(got), axis=-1)
    assert np.all(np.isfinite(got))
    assert np.all(top <= peak * (1.0 + tol)), (top, peak)
