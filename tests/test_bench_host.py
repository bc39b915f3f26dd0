"""Host-side statistics of the benchmark: the prefix RSE equals the oracle's
RSE on the same trajectories, time-to-target follows the "first checkpoint
after the last miss" rule, and the bootstrap interval brackets the mean."""
from __future__ import annotations

import math

import numpy as np
import pytest

import bench
from oracle import oracle as O


def _sample(M, seed):
    g = np.random.default_rng(seed)
    lw = g.normal(3.0, 1.5, size=M)
    al = g.random(M) < 0.7
    lw[~al] = -np.inf
    return lw, al


def test_prefix_rse_matches_oracle_statistics():
    lw, al = _sample(5000, 1)
    for m in (2, 17, 1024, 5000):
        st = O.stats(lw[:m], al[:m].astype(np.uint8))
        assert bench.prefix_rse(lw, al, m) == pytest.approx(st["rse"], rel=1e-10)
    assert bench.prefix_rse(lw, np.zeros(5000, dtype=bool), 100) == math.inf


def test_time_to_rse_rule():
    lw, al = _sample(1 << 14, 2)
    out = bench.time_to_rse(lw, al, 8.0, eps_list=(1.0, 1e-2, 1e-9))
    assert out["1e-09"] is None
    M = lw.size
    cps = [1 << k for k in range(1, 14)] + [M]
    for key, eps in (("1", 1.0), ("0.01", 1e-2)):
        rses = [bench.prefix_rse(lw, al, c) for c in cps]
        last_bad = max([i for i, r in enumerate(rses) if r > eps], default=-1)
        if last_bad == len(cps) - 1:
            assert out[key] is None
        else:
            c = cps[last_bad + 1]
            assert out[key]["trajectories"] == c
            assert out[key]["seconds"] == pytest.approx(8.0 * c / M)


def test_bootstrap_interval_brackets_the_mean():
    v = [0.9, 1.1, 1.0, 0.95, 1.05]
    lo, hi = bench.bootstrap_ci(v)
    assert lo <= np.mean(v) <= hi
    assert min(v) <= lo and hi <= max(v)
    assert bench.bootstrap_ci([2.0] * 5) == [2.0, 2.0]


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout == ""


def test_pooled_statistics_match_the_oracle():
    lw, al = _sample(3000, 3)
    st = O.stats(lw, al.astype(np.uint8))
    r = bench.pooled(lw, al, 1.0)
    for k in ("log_estimate", "ess", "rse", "var_logw", "p_match"):
        assert r[k] == pytest.approx(st[k], rel=1e-10), k


def test_pooling_launch_results_equals_the_union():
    """ESS of the whole job pooled from per-launch statistics (disjoint id
    ranges) equals the ESS of the union, not the sum of per-launch ESS."""
    lw, al = _sample(4000, 4)
    lw[7] = 40.0  # one dominant weight: per-launch ESS near 1 in its launch
    al[7] = True
    parts = []
    for a in range(0, 4000, 500):
        st = O.stats(lw[a:a + 500], al[a:a + 500].astype(np.uint8))
        st["n_traj"] = 500
        parts.append(st)
    union = bench.pooled(lw, al, 1.0)["ess"]
    assert bench.pool_results(parts) == pytest.approx(union, rel=1e-9)
    assert sum(p["ess"] for p in parts) > 3 * union


def test_byte_model_unit_costs():
    """The per-unit figures of the byte model, one unit at a time."""
    z = dict(n_steps=0, n_entries_scanned=0, n_entries_scanned_v=0, n_decrements=0, n_traj=0,
             n_local_entries=0, n_local_values=0, n_full_sk=0, n_dm=0)

    def one(**kw):
        d = dict(z)
        d.update(kw)
        return bench.algorithmic_bytes(d, 10, 30, scaled=True)

    assert one(n_entries_scanned=1) == 5
    assert one(n_entries_scanned_v=1) == 4
    assert one(n_decrements=1) == 36 + 28
    assert one(n_steps=1) == 4 * 28
    assert one(n_traj=1) == 24 * 10 + 9
    assert one(n_local_entries=1) == 9 and one(n_local_values=1) == 4
    assert one(n_full_sk=1) == 18 * 30 + 16 * 10 and one(n_dm=1) == 27 * 30
    d = dict(z, n_entries_scanned_v=1)
    assert bench.algorithmic_bytes(d, 10, 30, scaled=False) == 0


def test_time_to_target_is_the_checkpoint_after_the_last_violation():
    """Sec. 4 "Metrics": the first logged checkpoint after the last one whose
    relative error exceeds the target; the first one if none does; none if
    the final one exceeds it."""
    cps = [{"rel_error": e, "seconds": float(i)} for i, e in enumerate([0.5, 0.001, 0.02, 0.004, 0.003])]
    assert bench.est_time(cps, 1e-2)["seconds"] == 3.0
    assert bench.est_time(cps, 0.6)["seconds"] == 0.0
    assert bench.est_time(cps, 1e-3) is None
