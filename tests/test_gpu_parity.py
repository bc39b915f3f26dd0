"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Same seeded inputs, same trajectory ids: sampled matchings (paths), alive
flags, path hashes and work counters must be bit-identical; log-weights
agree to 1e-12 relative (only the final FP64 log may differ in the last
ulp); statistics to 1e-10 relative (parallel vs sequential summation).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_15390_amd import inputs as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _both(name, **over):
    import paper_2608_15390_amd as P
    g = P.preset(name, **over)
    o = O.Schedule(vertex_rule=g.vertex_rule, sk_policy=g.sk_policy, dm_policy=g.dm_policy,
                   initial_dm=g.initial_dm, K0=g.K0, K=g.K, theta_th=g.theta_th, theta_tr=g.theta_tr)
    return g, o


def _gpu(M, sched, seed, first, count, force_hbm=False, path=True):
    import paper_2608_15390_amd as P
    print(f"[gpu] n={M.n} nnz={M.nnz} sched={sched.as_dict()} seed={seed} ids={first}+{count} "
          f"hbm={force_hbm}", flush=True)
    est = P.PermEst(M, force_hbm=force_hbm)
    out = est.run(first, count, seed, sched, want_hash=True, want_path=path, want_counters=True)
    torch.cuda.synchronize()
    host = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
    est.close()
    return host


def _compare(M, gsched, osched, seed, first, count, force_hbm=False, path=True):
    g = _gpu(M, gsched, seed, first, count, force_hbm=force_hbm, path=path)
    o = O.run(O.OMatrix(M), osched, seed=seed, first=first, count=count, nthreads=8, want_path=path)
    np.testing.assert_array_equal(g["alive"], o["alive"])
    np.testing.assert_array_equal(g["counters"], o["counters"])
    np.testing.assert_array_equal(g["path_hash"].view(np.uint64), o["path_hash"])
    if path:
        np.testing.assert_array_equal(g["path"], o["path"])
    live = o["alive"] == 1
    assert np.isneginf(g["logw"][~live]).all()
    np.testing.assert_allclose(g["logw"][live], o["logw"][live], rtol=1e-12, atol=0)
    st = O.stats(o["logw"], o["alive"])
    r = g["result"]
    assert r["n_traj"] == count and r["n_alive"] == int(live.sum())
    assert r["n_steps"] == int(o["counters"][:, 0].sum())
    assert r["n_local_sk"] == int(o["counters"][:, 3].sum())
    assert r["n_full_sk"] == int(o["counters"][:, 2].sum())
    if live.any():
        assert r["log_estimate"] == pytest.approx(st["log_estimate"], rel=1e-10, abs=1e-10)
        assert r["ess"] == pytest.approx(st["ess"], rel=1e-10)
        if count > 1:
            assert r["rel_spread"] == pytest.approx(st["rel_spread"], rel=1e-9, abs=1e-12)
    else:
        assert math.isinf(r["log_estimate"]) and r["log_estimate"] < 0
    return g, o


SMALL = [("small1", lambda: G.config_small(1)), ("small2", lambda: G.config_small(2)),
         ("weighted", lambda: G.with_weights(G.planted_bernoulli(40, 0.12, 5, planted="random"), 1)),
         ("grid6x6", lambda: G.grid(6, 6)),
         ("band", lambda: G.banded(50, 3, 0.8, 4)[0])]


def test_small_workload_plain_bit_exact():
    """n = 20, identity + Bernoulli(0.2), 1e4 trajectories, MD, no scaling."""
    M = G.config_small(1)
    g, o = _both("plain")
    gr, orr = _compare(M, g, o, seed=1, first=0, count=10000)
    per = O.ryser(G.to_dense(M))
    r = gr["result"]
    assert abs(math.exp(r["log_estimate"]) / per - 1) <= 4.5 * r["rse"]


@pytest.mark.parametrize("name", ["plain", "rasmussen", "local_nodm", "outer_only", "adaptive_nodm", "fixed_nodm"])
@pytest.mark.parametrize("mat", SMALL, ids=[m[0] for m in SMALL])
def test_schedules_bit_exact_small(name, mat):
    M = mat[1]()
    over = {}
    base = name
    if name == "outer_only":
        base, over = "local_threshold", dict(sk_policy=0, dm_policy=0)
    elif name == "adaptive_nodm":
        base, over = "adaptive_threshold", dict(dm_policy=0)
    elif name == "fixed_nodm":
        base, over = "fixed_all", dict(dm_policy=0)
    g, o = _both(base, **over)
    _compare(M, g, o, seed=7, first=3, count=300)


@pytest.mark.parametrize("name", ["plain", "local_nodm", "adaptive_nodm"])
def test_lds_and_hbm_tiers_agree(name):
    base, over = (name, {}) if name != "adaptive_nodm" else ("adaptive_threshold", dict(dm_policy=0))
    M = G.planted_bernoulli(150, 0.04, 9, planted="random")
    g, o = _both(base, **over)
    a, _ = _compare(M, g, o, seed=3, first=0, count=200, force_hbm=False)
    b, _ = _compare(M, g, o, seed=3, first=0, count=200, force_hbm=True)
    for k in ("logw", "alive", "path", "path_hash", "counters"):
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("n,count", [(400, 64), (3000, 32)])
def test_batch_sized_and_large_matrices(n, count):
    M = G.planted_uniform(n, 7 * n, 11)
    for name in ("plain", "local_nodm"):
        g, o = _both(name)
        _compare(M, g, o, seed=5, first=17, count=count)


def test_full_size_large_workload_sampled_ids():
    """n = 1e5, avg degree 8: sampled trajectory ids of the benchmark's
    launch, checked one by one against the oracle."""
    M = G.config_large(1)
    g, o = _both("local_nodm")
    for first in (0, 65535, 99998):
        _compare(M, g, o, seed=1, first=first, count=2, path=True)


def test_full_size_band_workload_sampled_ids():
    """n = 1e5 band matrix of mean degree 8 (the exactly known workload):
    sampled trajectory ids against the oracle, plain and local repair."""
    M, _ = G.config_band(1)
    for name in ("plain", "local_nodm"):
        g, o = _both(name)
        for first in (0, 77777):
            _compare(M, g, o, seed=1, first=first, count=2, path=True)


@pytest.mark.parametrize("name,n", [("plain", 100), ("local_nodm", 200), ("local_threshold", 200)])
def test_gpu_mean_within_ci_of_band_permanent(name, n):
    """E[X] = per(A) (Sec. 2) at n = 100 and 200, beyond Ryser's reach: the
    exact value comes from the dynamic program over the band."""
    import paper_2608_15390_amd as P
    from oracle import band as B
    M, band = G.banded(n, 3, 0.8, 7)
    lp = B.band_log_permanent(band, 3)
    est = P.PermEst(M)
    r = est.run(0, 200000, 31, P.preset(name), want_logw=False, want_alive=False)["result"]
    est.close()
    assert abs(math.exp(r["log_estimate"] - lp) - 1) <= 4.5 * r["rse"], (name, r, lp)


@pytest.mark.parametrize("name", ["plain", "local_nodm", "adaptive_nodm"])
def test_all_ones_zero_variance_on_gpu(name):
    base, over = (name, {}) if name != "adaptive_nodm" else ("adaptive_threshold", dict(dm_policy=0))
    n = 12
    g, _ = _both(base, **over)
    out = _gpu(G.all_ones(n), g, seed=2, first=0, count=256)
    assert out["alive"].all()
    np.testing.assert_allclose(out["logw"], math.lgamma(n + 1), rtol=1e-13)


def test_edge_cases():
    g, o = _both("plain")
    # order 1
    _compare(G.identity(1), g, o, seed=1, first=0, count=5)
    # an empty column: no perfect matching, every trajectory dead
    D = np.ones((5, 5)); D[:, 2] = 0
    M = G.from_dense(D)
    out, _ = _compare(M, g, o, seed=1, first=0, count=40)
    assert out["result"]["p_match"] == 0.0
    # ... and with the initial filter (the run reports p_match = 0)
    g2, o2 = _both("local_nodm")
    out, _ = _compare(M, g2, o2, seed=1, first=0, count=40)
    assert out["result"]["n_alive"] == 0
    # single perfect matching: X = 1 always
    out, _ = _compare(G.permutation(300, seed=3), g, o, seed=1, first=0, count=64)
    np.testing.assert_array_equal(out["logw"], 0.0)
    # a count that is not a multiple of anything
    _compare(G.config_small(3), g, o, seed=9, first=1000, count=77)


def test_run_is_deterministic_and_range_consistent():
    import paper_2608_15390_amd as P
    M = G.config_small(5)
    s = P.preset("local_nodm")
    est = P.PermEst(M)
    a = est.run(0, 500, 42, s, want_hash=True, want_path=True, want_counters=True)
    b = est.run(0, 500, 42, s, want_hash=True, want_path=True, want_counters=True)
    c = est.run(200, 100, 42, s, want_hash=True, want_path=True, want_counters=True)
    for k in ("logw", "alive", "path", "path_hash", "counters"):
        assert torch.equal(a[k], b[k])
        assert torch.equal(a[k][200:300], c[k])
    est.close()


@pytest.mark.parametrize("gseed", [1, 2, 3, 4])
def test_gpu_mean_within_ci_of_ryser(gseed):
    import paper_2608_15390_amd as P
    M = G.config_small(gseed)
    per = O.ryser(G.to_dense(M))
    for name in ("plain", "local_nodm"):
        est = P.PermEst(M)
        r = est.run(0, 200000, 1000 + gseed, P.preset(name), want_logw=False, want_alive=False)["result"]
        est.close()
        assert abs(math.exp(r["log_estimate"]) / per - 1) <= 4.5 * r["rse"], (name, r)


PAPER_PRESETS = ["fixed_all", "adaptive_threshold", "local_threshold", "adaptive_tracked", "local_tracked"]
DM_MATS = [("small1", lambda: G.config_small(1)), ("small3", lambda: G.config_small(3)),
           ("weighted", lambda: G.with_weights(G.planted_bernoulli(40, 0.12, 5, planted="random"), 1)),
           ("batch60", lambda: G.planted_bernoulli(60, 5.0 / 59, 21, planted="random")),
           ("band", lambda: G.banded(50, 3, 0.8, 4)[0])]


@pytest.mark.parametrize("name", PAPER_PRESETS)
@pytest.mark.parametrize("mat", DM_MATS, ids=[m[0] for m in DM_MATS])
def test_paper_presets_with_inner_dm_bit_exact(name, mat):
    """The five variants of Sec. 4, inner DM included, on small inputs."""
    M = mat[1]()
    g, o = _both(name)
    out, orc = _compare(M, g, o, seed=13, first=0, count=200)
    if name == "fixed_all":
        assert out["alive"].all()  # DM at every child keeps p_match = 1
    assert out["result"]["n_dm"] == int(orc["counters"][:, 1].sum())


@pytest.mark.parametrize("name", ["adaptive_threshold", "local_threshold"])
def test_batch_sized_matrix_with_inner_dm(name):
    M = G.planted_bernoulli(300, 6.0 / 299, 77, planted="random")
    g, o = _both(name)
    _compare(M, g, o, seed=2, first=5, count=24)


@pytest.mark.parametrize("name", ["local_threshold", "adaptive_tracked"])
def test_tiers_agree_with_inner_dm(name):
    M = G.planted_bernoulli(120, 5.0 / 119, 3, planted="random")
    g, o = _both(name)
    a, _ = _compare(M, g, o, seed=4, first=0, count=64, force_hbm=False)
    b, _ = _compare(M, g, o, seed=4, first=0, count=64, force_hbm=True)
    for k in ("logw", "alive", "path", "path_hash", "counters"):
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("gseed", [1, 2])
def test_gpu_paper_presets_unbiased(gseed):
    import paper_2608_15390_amd as P
    M = G.config_small(gseed)
    per = O.ryser(G.to_dense(M))
    for name in PAPER_PRESETS:
        est = P.PermEst(M)
        r = est.run(0, 40000, 500 + gseed, P.preset(name), want_logw=False, want_alive=False)["result"]
        est.close()
        assert abs(math.exp(r["log_estimate"]) / per - 1) <= 4.5 * r["rse"], (name, r)
