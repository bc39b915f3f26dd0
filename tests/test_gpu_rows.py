"""Four trajectories per wave (16-lane rows) for a single matrix in HBM
scratch under the plain estimator (with or without the outer scaling) and
under the learned proposal: every trajectory equals the whole-wave
kernel's and the oracle's, bit for bit, including lists longer than a row,
weighted entries and dead ends."""
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


CASES = [
    ("sparse", lambda: G.planted_bernoulli(300, 6.0 / 300, 31, planted="random")),
    ("weighted", lambda: G.with_weights(G.planted_bernoulli(260, 5.0 / 260, 32, planted="random"), 4)),
    ("long_lists", lambda: G.planted_bernoulli(90, 0.5, 33, planted="random")),
    ("power_law", lambda: G.power_law(3000, 34)),
    ("band", lambda: G.banded(400, 4, 0.875, 35)[0]),
    ("no_matching", lambda: G.from_coo(40, np.r_[np.arange(39), 0], np.r_[np.arange(39), 1])),
]


LEARNED = {"learned": 0.05, "learned_alpha0": 0.0, "learned_alpha1": 1.0}


@pytest.mark.parametrize("case", [c[0] for c in CASES])
@pytest.mark.parametrize("name", ["plain", "plain_outer", "learned", "learned_alpha0", "learned_alpha1"])
def test_rows_match_whole_waves_and_oracle(case, name):
    import paper_2608_15390_amd as P
    M = dict(CASES)[case]()
    model, alpha = None, 0.05
    if name == "plain_outer":
        sched = P.preset("plain", initial_dm=1, K0=100)
    elif name in LEARNED:
        sched = P.preset("learned")
        model, alpha = R.quantize(R.init(61, scale=2.0)), LEARNED[name]
    else:
        sched = P.preset(name)
    count = 333
    print(f"[gpu] rows case={case} n={M.n} sched={name}", flush=True)
    outs = []
    for wave_per_traj in (False, True):
        h = P.PermEst(M, force_hbm=True, wave_per_trajectory=wave_per_traj)
        if model is not None:
            h.set_model(torch.as_tensor(model, dtype=torch.float32, device="cuda"), alpha)
        outs.append(h.run(5, count, 17, sched, want_hash=True, want_counters=True))
        torch.cuda.synchronize()
        h.close()
    rows, whole = outs
    for key in ("logw", "alive", "path_hash"):
        assert torch.equal(rows[key], whole[key]), key
    assert torch.equal(rows["counters"][:, 0], whole["counters"][:, 0])
    for f in ("log_estimate", "p_match", "ess", "n_alive", "n_steps", "n_entries_scanned", "n_decrements"):
        a, b = rows["result"][f], whole["result"][f]
        assert a == b or (a != a and b != b), f
    o = O.run(O.OMatrix(M), _osched(sched, model, alpha), seed=17, first=5, count=count, nthreads=8)
    al = rows["alive"].cpu().numpy()
    np.testing.assert_array_equal(al, o["alive"])
    np.testing.assert_array_equal(rows["path_hash"].cpu().numpy().view(np.uint64), o["path_hash"])
    live = o["alive"] == 1
    np.testing.assert_allclose(rows["logw"].cpu().numpy()[live], o["logw"][live], rtol=1e-12, atol=0)


def test_rows_large_sampled():
    """n = 1e5 (the large workload), outer-scaled plain estimator: sampled ids
    against the oracle, and the whole-wave kernel on the same ids."""
    import paper_2608_15390_amd as P
    M = G.config_large(1)
    sched = P.preset("plain", initial_dm=1, K0=100)
    h = P.PermEst(M)
    out = h.run(0, 4096, 3, sched, want_hash=True)
    torch.cuda.synchronize()
    h.close()
    w = P.PermEst(M, wave_per_trajectory=True)
    ref = w.run(0, 4096, 3, sched, want_hash=True)
    torch.cuda.synchronize()
    w.close()
    for key in ("logw", "alive", "path_hash"):
        assert torch.equal(out[key], ref[key]), key
    A = O.OMatrix(M)
    osch = _osched(sched)
    pre = O.prep(A, osch)
    lw = out["logw"].cpu().numpy()
    al = out["alive"].cpu().numpy()
    ph = out["path_hash"].cpu().numpy().view(np.uint64)
    for kk in (0, 777, 4095):
        o = O.run(A, osch, seed=3, first=kk, count=1, pre=pre)
        assert al[kk] == o["alive"][0] and ph[kk] == o["path_hash"][0], kk
        if o["alive"][0]:
            assert lw[kk] == pytest.approx(o["logw"][0], rel=1e-12)
