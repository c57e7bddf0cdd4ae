"""Exact check of the image enumeration of the GPU path (Sec. 2.1, Eq. (1)-(4)).

``ism_debug_enumerate`` runs the shell enumeration of the accumulation kernel
(same plan, same work items) and lists every image some work item owns. The
oracle lists the whole lattice in FP64 (``oracle.image_list``: lattice index,
gain, distance, delay x = d fs / c, amplitude). For each RIR:

- integer work is compared exactly: the set of lattice indices the GPU owns
  must be the lattice images with floor(x) < k_end = nS + W/2 - 1 (the images
  with a tap inside the RIR), each owned by exactly one work item, and the
  per-RIR image count and sum of k0 = floor(x) must match;
- the only allowed exception is an image whose delay lies within 1e-6 samples
  of an integer, where either floor is correct; such images are counted and
  reported, and their k0 may differ by one;
- the delay (k0 plus the 24-bit fraction the taps use) is within 1e-6
  samples of the oracle's x, and the FP32 amplitude within 1e-6 (relative) of
  the oracle's beta_n / (4 pi d_n).
"""
import sys

import numpy as np
import pytest

from paper_1810_11359_amd import ism, workloads

from .helpers import oracle_room_args

pytestmark = pytest.mark.gpu

NEAR = 1e-6       # samples: a delay this close to an integer may floor either way
TOL_X = 1e-6      # samples
TOL_A = 1e-6      # relative


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _key(n):
    n = np.asarray(n, dtype=np.int64) + 4096
    return (n[:, 0] << 26) | (n[:, 1] << 13) | n[:, 2]


def check_enumeration(oracle_mod, room, args, src, rcv, schedule=None):
    """Compares ism_debug_enumerate with the oracle's lattice, RIR by RIR.
    Returns (images compared, images excluded as near-integer delays)."""
    W = room.t_w * room.fs
    assert abs(W - round(W)) < 1e-9 and round(W) % 2 == 0
    k_end = room.n_samples + int(round(W)) // 2 - 1
    recs = ism.debug_enumerate(room, src, rcv, schedule)
    n_rcv = np.asarray(rcv).reshape(-1, 3).shape[0]
    total, excluded = 0, 0
    for si, s in enumerate(np.asarray(src, dtype=np.float32).reshape(-1, 3)):
        for ri, r in enumerate(np.asarray(rcv, dtype=np.float32).reshape(-1, 3)):
            rir = si * n_rcv + ri
            idx, vals = oracle_mod.image_list(*args, s[None], r[None])
            x, amp = vals[:, 2], vals[:, 3]
            k0_or = np.floor(x).astype(np.int64)
            near = np.abs(x - np.rint(x)) < NEAR
            owned_or = k0_or < k_end
            g = recs[recs["rir"] == rir]
            kg = _key(g["n"])
            # every owned image exactly once
            assert np.unique(kg).size == kg.size, f"rir {rir}: an image is owned by two work items"
            ko = _key(idx)
            order = np.argsort(ko)
            pos = np.searchsorted(ko[order], kg)
            assert np.all(pos < ko.size) and np.all(ko[order][np.minimum(pos, ko.size - 1)] == kg), \
                f"rir {rir}: the GPU lists an image outside the lattice"
            j = order[pos]  # oracle row of each GPU record
            in_g = np.zeros(ko.size, dtype=bool)
            in_g[j] = True
            # set equality except near-integer delays at the k_end boundary
            diff = in_g != owned_or
            assert np.all(near[diff] & (np.rint(x[diff]) == k_end)), \
                f"rir {rir}: {int(diff.sum())} images owned on one side only " \
                f"(e.g. lattice {idx[diff][:3].tolist()}, x {x[diff][:3].tolist()})"
            # integer delays exact, except near-integer delays
            k0_g = g["k0"].astype(np.int64)
            ok = ~near[j]
            assert np.array_equal(k0_g[ok], k0_or[j][ok]), f"rir {rir}: k0 differs"
            assert np.all(np.abs(k0_g[~ok] - k0_or[j][~ok]) <= 1)
            sel = owned_or & ~near
            assert int(ok.sum()) == int(sel.sum()), f"rir {rir}: image count differs"
            assert int(k0_g[ok].sum()) == int(k0_or[sel].sum()), f"rir {rir}: sum of k0 differs"
            # fractional delay and amplitude
            xg = k0_g + g["fq"].astype(np.float64) * 2.0 ** -24
            assert np.max(np.abs(xg - x[j])) <= TOL_X, f"rir {rir}: delay off by {np.max(np.abs(xg - x[j]))}"
            a_or = amp[j]
            a_err = np.abs(g["amp"].astype(np.float64) - a_or)
            assert np.all(a_err <= TOL_A * np.abs(a_or) + 1e-30), f"rir {rir}: amplitude off by {np.max(a_err / np.abs(a_or))}"
            total += int(kg.size)
            excluded += int((near & (owned_or | in_g)).sum())
    return total, excluded


def test_enumeration_room_32_receivers(oracle_mod):
    """The 32-receiver room (4 x 5 x 3 m, T60 0.7 s, 16 kHz), 4 receivers, with
    the default schedule (tapered tail) and a fine fixed split."""
    w = workloads.room_32_receivers(0)
    room = ism.room_for(w)
    args = oracle_room_args(oracle_mod, w)
    for sched in (None, ism.Schedule(item_taps=20000.0)):
        _say(f"enumeration room_32_receivers[:4] schedule={sched}")
        n, ex = check_enumeration(oracle_mod, room, args, w.src, w.rcv[:4], sched)
        print(f"compared {n} images, {ex} excluded (delay within {NEAR} of an integer)", flush=True)
        assert n > 3_000_000


def _feasible(oracle_mod):
    def ok(room, t60):
        try:
            oracle_mod.beta_from_t60(room, t60)
            return True
        except ValueError:
            return False

    return ok


def test_enumeration_batch_sparsest_and_densest(oracle_mod):
    """The rooms of the 1024-room batch with the fewest and the most images per
    RIR (T60^3 / volume), all their receivers (at most four), jittered
    per-wall beta."""
    ws = workloads.batch_rooms(1024, seed=0, feasible=_feasible(oracle_mod))
    dens = np.array([w.t60 ** 3 / np.prod(w.room) for w in ws])
    for k in (int(np.argmin(dens)), int(np.argmax(dens))):
        w = ws[k]
        room = ism.room_for(w)
        args = oracle_room_args(oracle_mod, w)
        _say(f"enumeration batch room {k} {w.room.round(2)} t60 {w.t60:.3f} n_img {room.n_img}")
        n, ex = check_enumeration(oracle_mod, room, args, w.src, w.rcv[:4])
        print(f"room {k}: compared {n} images, {ex} excluded", flush=True)
        assert n > 0


def test_enumeration_single_rir_and_signed_beta(oracle_mod):
    """The 3 x 4 x 2.5 m single RIR, and a small room with signed,
    non-uniform beta and odd lattice sizes (gains of either sign)."""
    w = workloads.single_rir(0)
    room = ism.room_for(w)
    _say("enumeration single_rir")
    check_enumeration(oracle_mod, room, oracle_room_args(oracle_mod, w), w.src, w.rcv)
    L = [3.3, 2.7, 2.9]
    beta = [0.9, -0.7, 0.8, 0.6, -0.95, 0.5]
    n_img = (21, 19, 23)
    room = ism.Room(L, beta, n_img, 343.0, 16000.0, 0.12, 0.004)
    args = (np.array(L), np.array(beta), n_img, 343.0, 16000.0, 0.12, 0.004)
    src = np.array([[1.0, 1.1, 1.2]], dtype=np.float32)
    rcv = np.array([[2.6, 0.5, 2.1], [0.4, 2.2, 0.3]], dtype=np.float32)
    _say("enumeration signed beta")
    check_enumeration(oracle_mod, room, args, src, rcv, ism.Schedule(item_taps=5000.0))
