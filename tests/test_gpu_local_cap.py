"""The bounded-work (sampled) local repair on the GPU against the oracle:
power-law matrices whose hub rows and columns have lists far longer than
the cap, both local-repair paths (first-hop lists within one wave, and
longer ones), both state tiers, weights, inner DM, the gated learned
fallback and a batch.  Paths, alive flags, hashes and counters bit-exact;
ln X to 1e-12."""
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
                      model=model, mix_alpha=mix_alpha, local_gate=g.local_gate, local_cap=g.local_cap)


def _check(g, o, count):
    np.testing.assert_array_equal(g["alive"], o["alive"])
    np.testing.assert_array_equal(g["counters"], o["counters"])
    np.testing.assert_array_equal(g["path_hash"].view(np.uint64), o["path_hash"])
    if "path" in g:
        np.testing.assert_array_equal(g["path"], o["path"])
    live = o["alive"] == 1
    np.testing.assert_allclose(g["logw"][live], o["logw"][live], rtol=1e-12, atol=0)
    assert g["result"]["n_traj"] == count


MATS = [("powerlaw2k", lambda: G.power_law(2000, 41, dmax=200)),
        ("powerlaw_w", lambda: G.with_weights(G.power_law(1500, 42, dmax=120), 3)),
        ("dense_lists", lambda: G.planted_bernoulli(120, 0.8, 43, planted="random"))]


@pytest.mark.parametrize("cap", [3, 16])
@pytest.mark.parametrize("name", ["local_nodm", "local_threshold", "local_tracked"])
@pytest.mark.parametrize("mat", MATS, ids=[m[0] for m in MATS])
def test_sampled_repair_bit_exact(mat, name, cap):
    import paper_2608_15390_amd as P
    M = mat[1]()
    sched = P.preset(name, local_cap=cap)
    count = 48 if M.n > 1000 else 120
    for hbm in (False, True):
        print(f"[gpu] local_cap={cap} {name} {mat[0]} n={M.n} hbm={hbm} ids=5+{count}", flush=True)
        est = P.PermEst(M, force_hbm=hbm)
        out = est.run(5, count, 8, sched, want_hash=True, want_path=True, want_counters=True)
        torch.cuda.synchronize()
        g = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
        est.close()
        o = O.run(O.OMatrix(M), _osched(sched), seed=8, first=5, count=count, nthreads=8, want_path=True)
        _check(g, o, count)
        assert g["result"]["n_local_sk"] > 0


def test_sampled_repair_examines_fewer_entries_on_hubs():
    import paper_2608_15390_amd as P
    M = G.power_law(3000, 44, dmax=200)
    est = P.PermEst(M)
    full = est.run(0, 256, 2, P.preset("local_nodm"), want_logw=False, want_alive=False)["result"]
    capd = est.run(0, 256, 2, P.preset("local_nodm", local_cap=16), want_logw=False, want_alive=False)["result"]
    torch.cuda.synchronize()
    est.close()
    per_step = lambda r: r["n_local_entries"] / max(r["n_local_sk"], 1)  # noqa: E731
    assert per_step(capd) < 0.8 * per_step(full)


def test_sampled_gated_learned_fallback_and_batch():
    import paper_2608_15390_amd as P
    mats = [G.power_law(800, 45, dmax=150), G.planted_bernoulli(90, 0.85, 46, planted="random"),
            G.config_batch(5, count=1, nmin=60, nmax=200)[0]]
    model = R.quantize(R.init(17, scale=2.0))
    for name in ("learned_gated", "learned_threshold_gated", "local_threshold"):
        sched = P.preset(name, local_cap=8)
        counts = [40, 50, 60]
        print(f"[gpu] local_cap batch {name} n={[M.n for M in mats]}", flush=True)
        bt = P.PermEstBatch(mats)
        bt.set_model(torch.as_tensor(model, dtype=torch.float32, device="cuda"), 0.05)
        out = bt.run(counts, 13, sched, want_hash=True)
        torch.cuda.synchronize()
        lw, al = out["logw"].cpu().numpy(), out["alive"].cpu().numpy()
        ph = out["path_hash"].cpu().numpy().view(np.uint64)
        off = out["offsets"]
        osch = _osched(sched, model if name.startswith("learned") else None)
        for b, M in enumerate(mats):
            o = O.run(O.OMatrix(M), osch, seed=13, first=0, count=counts[b], b=b, nthreads=8)
            sl = slice(off[b], off[b + 1])
            np.testing.assert_array_equal(al[sl], o["alive"], err_msg=f"{name} matrix {b}")
            np.testing.assert_array_equal(ph[sl], o["path_hash"], err_msg=f"{name} matrix {b}")
            live = o["alive"] == 1
            np.testing.assert_allclose(lw[sl][live], o["logw"][live], rtol=1e-12, atol=0)
        assert sum(r["n_local_sk"] for r in out["results"]) > 0
        bt.close()
