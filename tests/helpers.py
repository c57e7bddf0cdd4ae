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
