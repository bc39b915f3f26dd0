"""Batched runs: many matrices of uneven order in one persistent launch.

Every matrix's trajectories must equal the oracle's for the same (matrix
index b, trajectory id) bit for bit, whatever the launch shape the
autotuner picks."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_15390_amd import inputs as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _osched(g):
    return O.Schedule(vertex_rule=g.vertex_rule, sk_policy=g.sk_policy, dm_policy=g.dm_policy,
                      initial_dm=g.initial_dm, K0=g.K0, K=g.K, theta_th=g.theta_th, theta_tr=g.theta_tr)


def _small_batch(count=10, seed=3, nmax=120):
    return G.config_batch(seed, count=count, nmin=30, nmax=nmax)


@pytest.mark.parametrize("name", ["local_nodm", "adaptive_threshold", "local_threshold", "plain"])
def test_batch_matches_oracle_per_matrix(name):
    import paper_2608_15390_amd as P
    mats = _small_batch()
    counts = [40 + 7 * b for b in range(len(mats))]
    sched = P.preset(name)
    print(f"[gpu] batch of {len(mats)} n={[M.n for M in mats]} sched={name}", flush=True)
    bt = P.PermEstBatch(mats)
    out = bt.run(counts, 11, sched, want_hash=True)
    torch.cuda.synchronize()
    lw = out["logw"].cpu().numpy()
    al = out["alive"].cpu().numpy()
    ph = out["path_hash"].cpu().numpy().view(np.uint64)
    off = out["offsets"]
    for b, M in enumerate(mats):
        o = O.run(O.OMatrix(M), _osched(sched), seed=11, first=0, count=counts[b], b=b, nthreads=8)
        sl = slice(off[b], off[b + 1])
        np.testing.assert_array_equal(al[sl], o["alive"], err_msg=f"matrix {b}")
        np.testing.assert_array_equal(ph[sl], o["path_hash"], err_msg=f"matrix {b}")
        live = o["alive"] == 1
        np.testing.assert_allclose(lw[sl][live], o["logw"][live], rtol=1e-12, atol=0)
        st = O.stats(o["logw"], o["alive"])
        r = out["results"][b]
        assert r["n_traj"] == counts[b] and r["n_alive"] == int(live.sum())
        if live.any():
            assert r["log_estimate"] == pytest.approx(st["log_estimate"], rel=1e-10, abs=1e-10)
    bt.close()


def test_autotuned_shape_gives_identical_results():
    import paper_2608_15390_amd as P
    mats = _small_batch(count=6, seed=5)
    sched = P.preset("adaptive_threshold")
    bt = P.PermEstBatch(mats)
    a = bt.run(300, 2, sched, want_hash=True)
    b = bt.run(300, 2, sched, want_hash=True, autotune=True)
    c = bt.run(300, 2, sched, want_hash=True, autotune=True)  # cached shape
    for k in ("logw", "alive", "path_hash"):
        assert torch.equal(a[k], b[k]) and torch.equal(a[k], c[k])
    bt.close()


def test_matrix_zero_of_a_batch_equals_a_single_run():
    import paper_2608_15390_amd as P
    mats = _small_batch(count=4, seed=8)
    sched = P.preset("local_nodm")
    bt = P.PermEstBatch(mats)
    out = bt.run(256, 4, sched, want_hash=True)
    single = P.PermEst(mats[0]).run(0, 256, 4, sched, want_hash=True)
    assert torch.equal(out["logw"][:256], single["logw"])
    assert torch.equal(out["path_hash"][:256], single["path_hash"])
    bt.close()


def test_full_batch_workload_sampled():
    """256 matrices, n ~ U{30..400}, mean degree U[3,12], 4096 trajectories
    each, adaptive SK + threshold DM, one autotuned persistent launch; sampled
    (matrix, trajectory) pairs are recomputed one by one by the oracle."""
    import paper_2608_15390_amd as P
    mats = G.config_batch(1)
    sched = P.preset("adaptive_threshold")
    bt = P.PermEstBatch(mats)
    out = bt.run(4096, 1, sched, want_hash=True, autotune=True)
    torch.cuda.synchronize()
    lw = out["logw"].cpu().numpy()
    al = out["alive"].cpu().numpy()
    ph = out["path_hash"].cpu().numpy().view(np.uint64)
    rng = np.random.default_rng(0)
    for b in sorted(rng.choice(len(mats), 6, replace=False)):
        for k in (0, int(rng.integers(1, 4096)), 4095):
            o = O.run(O.OMatrix(mats[b]), _osched(sched), seed=1, first=k, count=1, b=int(b))
            q = 4096 * b + k
            assert al[q] == o["alive"][0] and ph[q] == o["path_hash"][0], (b, k)
            if o["alive"][0]:
                assert lw[q] == pytest.approx(o["logw"][0], rel=1e-12)
    for r in out["results"]:
        assert r["n_traj"] == 4096 and 0.0 <= r["p_match"] <= 1.0
    bt.close()


def test_batch_estimates_unbiased_on_known_permanents():
    import paper_2608_15390_amd as P
    mats = [G.config_small(s) for s in range(1, 9)]
    pers = [O.ryser(G.to_dense(M)) for M in mats]
    bt = P.PermEstBatch(mats)
    out = bt.run(50000, 9, P.preset("local_threshold"), want_logw=False, want_alive=False)
    for r, per in zip(out["results"], pers):
        assert abs(math.exp(r["log_estimate"]) / per - 1) <= 4.5 * r["rse"]
    bt.close()


def test_graph_replays_equal_eager_runs():
    """The captured launch sequence replays to the eager results on every
    replay, with eager launches of other seeds and shapes in between."""
    import paper_2608_15390_amd as P
    mats = _small_batch(count=5, seed=12)
    sched = P.preset("adaptive_threshold")
    bt = P.PermEstBatch(mats)
    counts = [200 + 13 * b for b in range(len(mats))]
    for rep, seed in enumerate((3, 4, 3, 9)):
        print(f"[gpu] graph replay {rep} seed {seed}", flush=True)
        g = bt.run(counts, seed, sched, want_hash=True, graph=True)
        torch.cuda.synchronize()
        other = bt.run(17, seed + 100, P.preset("plain"), want_hash=True)  # eager work in between
        torch.cuda.synchronize()
        e = bt.run(counts, seed, sched, want_hash=True)
        torch.cuda.synchronize()
        for k in ("logw", "alive", "path_hash"):
            assert torch.equal(g[k], e[k]), (rep, k)
        for rg, re_ in zip(g["results"], e["results"]):
            for f in ("log_estimate", "ess", "p_match", "n_alive", "n_steps"):
                assert rg[f] == re_[f] or (math.isnan(rg[f]) and math.isnan(re_[f])), (rep, f)
        assert other["results"][0]["n_traj"] == 17
    bt.close()


@pytest.mark.parametrize("name", ["local_nodm", "plain"])
def test_mixed_tiers_in_one_launch(name):
    """Small matrices run with their state in LDS and a large one in HBM
    within the same launch; every matrix still equals the oracle."""
    import paper_2608_15390_amd as P
    mats = _small_batch(count=6, seed=21) + [G.planted_bernoulli(2500, 6.0 / 2500, 77, planted="random")]
    counts = [400] * 6 + [2]
    sched = P.preset(name)
    print(f"[gpu] mixed tiers n={[M.n for M in mats]} sched={name}", flush=True)
    bt = P.PermEstBatch(mats)
    out = bt.run(counts, 13, sched, want_hash=True)
    torch.cuda.synchronize()
    lw = out["logw"].cpu().numpy()
    al = out["alive"].cpu().numpy()
    ph = out["path_hash"].cpu().numpy().view(np.uint64)
    off = out["offsets"]
    for b, M in enumerate(mats):
        o = O.run(O.OMatrix(M), _osched(sched), seed=13, first=0, count=counts[b], b=b, nthreads=8)
        sl = slice(off[b], off[b + 1])
        np.testing.assert_array_equal(al[sl], o["alive"], err_msg=f"matrix {b}")
        np.testing.assert_array_equal(ph[sl], o["path_hash"], err_msg=f"matrix {b}")
        live = o["alive"] == 1
        np.testing.assert_allclose(lw[sl][live], o["logw"][live], rtol=1e-12, atol=0)
    bt.close()
