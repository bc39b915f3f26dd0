"""Parity at the large sizes, in the launch shapes the benchmark uses.

* The learned proposal on the n = 1e5, average-degree-8 workload: one
  benchmark step (5000 trajectory ids in one launch) with sampled ids
  recomputed one by one by the oracle.
* One matrix of order 6e5, where the min-tree over 2n degree leaves needs
  three levels (more than 64 x 64 groups of 256 leaves): the plain
  estimator (default launch and forced whole waves), the local repair and
  the learned proposal, on a planted uniform matrix and on a power-law one
  (degrees up to 200).  At this order four trees per wave no longer fit
  four waves in a CU's LDS, so every launch takes whole waves with the
  tree's lowest level in the state slot.
* A batch holding an order-1.5e5 matrix (level 0 in the state slot) beside
  a small LDS-tier one.
* The learned proposal in the four-per-wave kernel with a two-level tree,
  level 0 in LDS (n = 5e4) and in the state slots (n = 8e4).

Paths, alive flags, counters and path hashes compare bit for bit, ln X to
1e-12 relative (the oracle's stated FP64 agreement)."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import mlp as R
from oracle import oracle as O
from paper_2608_15390_amd import inputs as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _osched(g, model=None, mix_alpha=0.05):
    return O.Schedule(vertex_rule=g.vertex_rule, sk_policy=g.sk_policy, dm_policy=g.dm_policy,
                      initial_dm=g.initial_dm, K0=g.K0, K=g.K, theta_th=g.theta_th, theta_tr=g.theta_tr,
                      model=model, mix_alpha=mix_alpha)


def _check_sampled(M, sched, osch, seed, first, count, picks, model=None, alpha=0.01, **flags):
    """One GPU launch of ids first..first+count-1; the ids `picks` of it
    recomputed by the oracle one at a time."""
    import paper_2608_15390_amd as P
    print(f"[gpu] n={M.n} nnz={M.nnz} sched={sched.as_dict()} ids={first}+{count} picks={picks} "
          f"flags={flags}", flush=True)
    est = P.PermEst(M, **flags)
    if model is not None:
        est.set_model(torch.as_tensor(model, dtype=torch.float32, device="cuda"), alpha)
    out = est.run(first, count, seed, sched, want_hash=True, want_counters=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")}
    g["result"] = out["result"]
    est.close()
    A = O.OMatrix(M)
    pre = O.prep(A, osch)
    for k in picks:
        o = O.run(A, osch, seed=seed, first=k, count=1, pre=pre)
        i = k - first
        assert g["alive"][i] == o["alive"][0], k
        np.testing.assert_array_equal(g["counters"][i], o["counters"][0], err_msg=str(k))
        assert g["path_hash"].view(np.uint64)[i] == o["path_hash"][0], k
        if o["alive"][0]:
            assert g["logw"][i] == pytest.approx(o["logw"][0], rel=1e-12, abs=0), k
        else:
            assert np.isneginf(g["logw"][i]), k
    return g


@pytest.mark.timeout(600)
def test_learned_headline_workload_benchmark_launch():
    """n = 1e5, avg degree 8, learned proposal (quantised network, uniform
    share 0.01 as in the benchmark): one benchmark step of 5000 ids."""
    import paper_2608_15390_amd as P
    M = G.config_large(1)
    model = R.quantize(R.init(31, scale=1.5))
    sched = P.preset("learned")
    _check_sampled(M, sched, _osched(sched, model, 0.01), 1, 0, 5000, [0, 2500, 4999], model=model)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("n", [50_000, 80_000])
def test_learned_rows_two_level_tree(n):
    """Learned proposal in the four-per-wave kernel on a matrix whose
    min-tree has two internal levels: at n = 5e4 four whole trees per wave
    cost no resident blocks and level 0 stays in LDS; at n = 8e4 it moves to
    the rows' state slots.  Sampled ids of one launch against the oracle."""
    import paper_2608_15390_amd as P
    M = G.planted_uniform(n, 7 * n, 41)
    model = R.quantize(R.init(34, scale=1.5))
    sched = P.preset("learned")
    g = _check_sampled(M, sched, _osched(sched, model, 0.01), 5, 0, 600, [0, 299, 599], model=model)
    assert g["result"]["launch_trajectories_per_wave"] == 4


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,flags", [("plain", {}), ("plain", {"wave_per_trajectory": True}),
                                        ("local_nodm", {}), ("learned", {})])
def test_three_level_min_tree_planted_uniform(name, flags):
    """Order 6e5 (three min-tree levels), planted permutation + 7n entries."""
    import paper_2608_15390_amd as P
    M = G.planted_uniform(600_000, 4_200_000, 23)
    sched = P.preset(name)
    model = R.quantize(R.init(31, scale=1.5)) if name == "learned" else None
    count = 1 if name == "local_nodm" else 2
    _check_sampled(M, sched, _osched(sched, model, 0.01), 3, 5, count, list(range(5, 5 + count)),
                   model=model, **flags)


@pytest.mark.timeout(600)
def test_three_level_min_tree_power_law_learned():
    """Order 6e5, power-law row degrees (exponent 2.5 on [2, 200]) plus a
    planted permutation, learned proposal."""
    import paper_2608_15390_amd as P
    M = G.power_law(600_000, 77)
    sched = P.preset("learned")
    model = R.quantize(R.init(32, scale=1.5))
    _check_sampled(M, sched, _osched(sched, model, 0.01), 4, 11, 2, [11, 12], model=model)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["learned", "local_nodm", "plain"])
def test_tree_level0_in_state_slot_batch(name):
    """A batch (one trajectory per wave) with a matrix of order 1.5e5, whose
    min-tree keeps its lowest internal level in the trajectory's state slot
    (above 2^18 leaves), beside a small LDS-tier matrix: sampled ids of both
    against the oracle."""
    import paper_2608_15390_amd as P
    # a permuted band (no dead ends, so every sampled trajectory completes)
    mats = [G.config_band(1, n=150_000)[0], G.planted_bernoulli(200, 0.04, 79, planted="random")]
    sched = P.preset(name)
    model = R.quantize(R.init(33, scale=1.5)) if name == "learned" else None
    counts = [6, 40]
    print(f"[gpu] level-0-in-state batch n={[M.n for M in mats]} sched={name}", flush=True)
    bt = P.PermEstBatch(mats)
    if model is not None:
        bt.set_model(torch.as_tensor(model, dtype=torch.float32, device="cuda"), 0.01)
    out = bt.run(counts, 9, sched, want_hash=True)
    torch.cuda.synchronize()
    lw, al = out["logw"].cpu().numpy(), out["alive"].cpu().numpy()
    ph = out["path_hash"].cpu().numpy().view(np.uint64)
    off = out["offsets"]
    osch = _osched(sched, model, 0.01)
    bt.close()
    for b, M in enumerate(mats):
        A = O.OMatrix(M)
        picks = [0, counts[b] - 1] if b == 0 else list(range(counts[b]))
        o = O.run(A, osch, seed=9, first=0, count=counts[b], b=b, nthreads=8) if b == 1 else None
        for k in picks:
            if b == 0:
                ok = O.run(A, osch, seed=9, first=k, count=1, b=b)
                ref = {key: v[0] for key, v in ok.items()}
            else:
                ref = {key: v[k] for key, v in o.items()}
            i = off[b] + k
            assert al[i] == ref["alive"], (b, k)
            assert ph[i] == ref["path_hash"], (b, k)
            if ref["alive"]:
                assert lw[i] == pytest.approx(ref["logw"], rel=1e-12, abs=0), (b, k)
