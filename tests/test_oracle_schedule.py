"""The oracle's scheduler (Alg. 2's z, track, DM trigger and SK count; the
Adaptive, Thrs and Trck policies of Sec. 3.3), recomputed by hand from state
snapshots.

For every step t of a trajectory the oracle is stopped before its draw
(same seed, so the same trajectory), which gives the pre-step scaling
vectors r, c and, under the learned proposal, the probabilities of the
candidates. From those and the recorded path the test forms by hand:

* z = r_rho * c_gam with rho the row and gam the column end of the chosen
  edge (FP64 product of the binary32 values); under the learned proposal
  z = q(u | v), the probability actually sampled;
* track <- track * z, reset to 1 after every inner DM call;
* run_dm = All, or Thrs with z < theta_th, or Trck with track < theta_tr
  (strict comparisons);
* the SK count: Fixed K sweeps, Adaptive clamp(ceil((1 - z) K), 0, K),
  Local one repair, the learned proposal's gated fallback one repair when
  z < theta_th or DM ran (and then z of the next step is r_rho c_gam of
  the scaled proposal it draws from);

and asserts the oracle's event record (DM on/off, SK count per step) equals
it. A floor for the ceiling, z taken after the repair, a missing reset of
track or a non-strict comparison each changes some event here. Strictness
is pinned directly by setting a threshold to a z (or track) value the
trajectory actually reaches: that step must not trigger."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import mlp as R
from oracle import oracle as O
from paper_2608_15390_amd import inputs as G


def _mats():
    return [G.planted_bernoulli(36, 0.16, 3, planted="random"),
            G.planted_bernoulli(48, 0.10, 4, planted="random"),
            G.with_weights(G.planted_bernoulli(40, 0.14, 5, planted="random"), 6),
            # entries below 1: after row scaling r_rho c_gam = 1 / B_rho,gam
            # times a share of the row, so z can exceed 1 + 1/K and the
            # Adaptive count must be clamped at 0
            G.with_weights(G.planted_bernoulli(32, 0.15, 8, planted="random"), 9, lo=0.05, hi=1.0)]


def _walk(A, sched, pre, seed, k):
    """The trajectory's path and events, and for each step before the end
    the snapshot taken before its draw."""
    full = O.probe(A, sched, pre, seed, k, [], -1)
    steps = full["steps"]
    snaps = [O.probe(A, sched, pre, seed, k, [], t) for t in range(steps)]
    for t, s in enumerate(snaps):
        assert s["stopped"] == 1 and s["steps"] == t
    return full, snaps


def _expected(A, sched, full, snaps):
    """Events recomputed from the snapshots; also the z and track values."""
    n = A.n
    path = full["path"]
    exp = np.zeros(2 * n, dtype=np.int32)
    zs, tracks = [], []
    track = 1.0
    gate = sched.sk_policy == O.SK_LEARNED and sched.local_gate
    fb = False  # this step draws from the scaled proposal (gated fallback)
    steps = full["steps"]
    for t in range(steps):
        v, u = int(path[2 * t]), int(path[2 * t + 1])
        s = snaps[t]
        if sched.sk_policy == O.SK_LEARNED and not fb:
            z = float(s["prob"][list(s["cand"]).index(u)])
        else:
            rho, gam = (v, u) if v < n else (u, v)
            z = float(s["r"][rho]) * float(s["c"][gam - n])
        track = track * z
        zs.append(z)
        tracks.append(track)
        last = t + 1 >= n
        # a dead child (or the final step) ends the trajectory before the
        # schedule runs; the next snapshot exists iff the step's schedule ran
        if last or (t + 1 == steps and not full["alive"]):
            break
        run_dm = (sched.dm_policy == O.DM_ALL or
                  (sched.dm_policy == O.DM_THRS and z < sched.theta_th) or
                  (sched.dm_policy == O.DM_TRCK and track < sched.theta_tr))
        if run_dm:
            exp[2 * t] = 1
            track = 1.0
        if sched.sk_policy == O.SK_FIXED:
            exp[2 * t + 1] = sched.K
        elif sched.sk_policy == O.SK_ADAPTIVE:
            want = math.ceil((1.0 - z) * sched.K) if math.isfinite(z) else 0
            exp[2 * t + 1] = min(max(want, 0), sched.K)
        elif sched.sk_policy == O.SK_LOCAL:
            exp[2 * t + 1] = 1
        elif gate:
            fb = z < sched.theta_th or run_dm
            exp[2 * t + 1] = int(fb)
    return exp, zs, tracks


def _schedules():
    model = R.quantize(R.init(7, scale=2.0))
    return {
        "fixed_all": O.preset("fixed_all"),
        "adaptive_threshold": O.preset("adaptive_threshold"),
        "adaptive_tracked": O.preset("adaptive_tracked"),
        "local_tracked": O.preset("local_tracked"),
        "local_threshold": O.preset("local_threshold"),
        # poorly converged outer scaling: z spreads out, so many sweep
        # counts and frequent Trck resets are exercised
        "adaptive_tracked_K0_2": O.preset("adaptive_tracked").replace(K0=2, K=7, theta_tr=0.6),
        "adaptive_threshold_K0_1": O.preset("adaptive_threshold").replace(K0=1, K=9, theta_th=0.5),
        "learned_threshold": O.preset("learned_threshold").replace(model=model, mix_alpha=0.05),
        # learned with the gated local-repair fallback (z of a fallback step
        # is r_rho c_gam, of a network step the sampled probability)
        "learned_gated": O.preset("learned").replace(model=model, mix_alpha=0.05, local_gate=1, theta_th=0.4),
        "learned_threshold_gated": O.preset("learned_threshold").replace(model=model, mix_alpha=0.05,
                                                                         local_gate=1),
    }


@pytest.mark.parametrize("name", list(_schedules()))
def test_schedule_events_recomputed_from_snapshots(name):
    sched = _schedules()[name]
    seen = {"dm": 0, "no_dm": 0, "nit": set(), "z_above_1": 0}
    for M in _mats():
        A = O.OMatrix(M)
        pre = O.prep(A, sched)
        for k in range(20):
            full, snaps = _walk(A, sched, pre, 11, k)
            exp, zs, tracks = _expected(A, sched, full, snaps)
            np.testing.assert_array_equal(full["events"], exp, err_msg=f"{name} n={A.n} k={k}")
            # the counters agree with the event record
            assert full["counters"][1] == int(exp[0::2].sum())
            if sched.sk_policy in (O.SK_FIXED, O.SK_ADAPTIVE):
                assert full["counters"][2] == int(exp[1::2].sum())
            seen["dm"] += int(exp[0::2].sum())
            seen["no_dm"] += len(zs) - int(exp[0::2].sum())
            seen["nit"].update(int(x) for x in exp[1::2][: len(zs)])
            seen["z_above_1"] += sum(z > 1.0 + 1.0 / max(sched.K, 1) for z in zs)
    # the walk saw both decisions (and, for Adaptive, several sweep counts)
    if sched.dm_policy not in (O.DM_ALL, O.DM_NONE):
        assert seen["dm"] > 0 and seen["no_dm"] > 0, seen
    if sched.local_gate:
        assert seen["nit"] == {0, 1}, seen
    if sched.sk_policy == O.SK_ADAPTIVE:
        assert len(seen["nit"]) >= 3, seen
        # the clamp at 0 was needed somewhere
        assert seen["z_above_1"] > 0 and 0 in seen["nit"], seen


def _first_step_with(A, sched, pre, seed, pred):
    for k in range(40):
        full, snaps = _walk(A, sched, pre, seed, k)
        _, zs, tracks = _expected(A, sched, full, snaps)
        for t in range(min(len(zs), full["steps"] - 1)):
            if pred(zs[t], tracks[t]):
                return k, t, zs[t], tracks[t]
    raise AssertionError("no step found")


def test_thrs_comparison_is_strict():
    """theta_th set to a z the trajectory reaches at step t: z < theta is
    false there, so no DM at t; just above it, DM runs at t."""
    M = _mats()[0]
    A = O.OMatrix(M)
    base = O.preset("adaptive_threshold")
    pre = O.prep(A, base)
    k, t, z, _ = _first_step_with(A, base, pre, 13, lambda z, tr: 0.05 < z < 0.95)
    eq = base.replace(theta_th=z)
    full = O.probe(A, eq, pre, 13, k, [], -1)
    assert full["events"][2 * t] == 0
    above = base.replace(theta_th=math.nextafter(z, math.inf))
    full = O.probe(A, above, pre, 13, k, [], -1)
    assert full["events"][2 * t] == 1


def test_trck_comparison_is_strict_and_track_resets():
    """theta_tr set to the track value reached at step t (no DM before it):
    no DM at t; just above it, DM at t, and track restarts from 1, so the
    next trigger needs the product of the following z values alone to fall
    below theta_tr."""
    M = _mats()[1]
    A = O.OMatrix(M)
    base = O.preset("adaptive_tracked").replace(theta_tr=1e-300)  # never triggers
    pre = O.prep(A, base)
    k, t, _, tr = _first_step_with(A, base, pre, 17, lambda z, tr: 0.02 < tr < 0.9)
    eq = base.replace(theta_tr=tr)
    full = O.probe(A, eq, pre, 17, k, [], -1)
    assert full["events"][2 * t] == 0
    above = base.replace(theta_tr=math.nextafter(tr, math.inf))
    full, snaps = _walk(A, above, pre, 17, k)
    assert full["events"][2 * t] == 1
    exp, _, _ = _expected(A, above, full, snaps)
    np.testing.assert_array_equal(full["events"], exp)


def test_adaptive_count_is_a_ceiling():
    """At a step whose (1 - z) K is not an integer the sweep count is the
    next integer up; z is the pre-step product."""
    M = _mats()[2]
    A = O.OMatrix(M)
    sched = O.preset("adaptive_threshold").replace(dm_policy=O.DM_NONE, K0=3)
    pre = O.prep(A, sched)
    found = 0
    for k in range(10):
        full, snaps = _walk(A, sched, pre, 19, k)
        _, zs, _ = _expected(A, sched, full, snaps)
        for t, z in enumerate(zs[: full["steps"] - 1]):
            x = (1.0 - z) * sched.K
            if 0.0 < x < sched.K and x != math.floor(x):
                assert full["events"][2 * t + 1] == math.floor(x) + 1
                found += 1
    assert found > 20
