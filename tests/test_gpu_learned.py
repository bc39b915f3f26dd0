"""Learned proposal on the GPU: the network's matrix-core forward and
backward against the FP64 network reference, training-pair recording
against the oracle's own steps, and trajectories with the learned proposal
bit for bit against the oracle.

Tolerances of the float network (forward, loss, gradient) come from its
arithmetic: parameters and features are rounded to bfloat16 on both sides,
the GPU also rounds the first hidden layer (and, backward, the two
pre-activation gradients) to bfloat16, a relative error of 2^-9 per
value; summed over 8..64 terms that leaves a relative L2 error of about
2e-3 in the logits (measured in numpy emulation), so the bounds below keep a
margin of 5x.  The quantised network that drives sampling is exact, so
trajectories compare bit for bit."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import mlp as R
from oracle import oracle as O
from paper_2608_15390_amd import inputs as G
from oracle_tools import stats_by_hand

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _groups(seed, groups=300, kmax=9):
    g = np.random.default_rng(seed)
    sizes = g.integers(2, kmax, size=groups)
    off = np.concatenate([[0], np.cumsum(sizes)])
    X = np.zeros((off[-1], 8))
    X[:, 0:2] = g.integers(1, 30, size=(off[-1], 2)) / 64.0
    X[:, 2:5] = g.normal(0, 1, (off[-1], 3))
    X[:, 5] = g.integers(0, 2, size=off[-1])
    y = np.empty(off[-1])
    for a, b in zip(off[:-1], off[1:]):
        p = g.random(b - a) + 0.05
        y[a:b] = p / p.sum()
    return X, y, off


def _recording(X, y, off):
    G_ = len(off) - 1
    ginfo = np.zeros((G_, 4), dtype=np.int32)
    ginfo[:, 0] = np.diff(off)
    return {"x": _dev(X, torch.float32), "y": _dev(y, torch.float32),
            "gstart": _dev(off[:-1], torch.int64), "ginfo": _dev(ginfo, torch.int32), "n_groups": G_}


def test_mlp_forward_matches_reference():
    import paper_2608_15390_amd as P
    th = R.init(3)
    X, _, _ = _groups(1)
    net = P.ProposalNet(th.astype(np.float32))
    L = net.forward(_dev(X, torch.float32)).cpu().numpy().astype(np.float64)
    ref, _ = R.forward(R.bf16(th), R.bf16(X))
    rel = np.linalg.norm(L - ref) / np.linalg.norm(ref)
    print(f"[gpu] forward rel L2 {rel:.2e}", flush=True)
    assert rel <= 1e-2
    assert np.abs(L - ref).max() <= 0.05
    net.close()


@pytest.mark.parametrize("window", [(0, 300), (17, 211)])
def test_mlp_loss_and_gradient_match_reference(window):
    import paper_2608_15390_amd as P
    th = R.init(5)
    X, y, off = _groups(2)
    rec = _recording(X, y, off)
    net = P.ProposalNet(th.astype(np.float32))
    g0, g1 = window
    loss, grad = net.loss_grad(rec, g0, g1)
    grad = grad.cpu().numpy().astype(np.float64)
    sub = off[g0:g1 + 1]
    Xs, ys = R.bf16(X[sub[0]:sub[-1]]), y[sub[0]:sub[-1]]
    lref, gref = R.loss_and_grad(R.bf16(th), Xs, ys, sub - sub[0])
    rel = np.linalg.norm(grad - gref) / np.linalg.norm(gref)
    cos = grad @ gref / (np.linalg.norm(grad) * np.linalg.norm(gref))
    print(f"[gpu] window {window}: loss {loss:.6f} vs {lref:.6f}, grad rel L2 {rel:.2e} cos {cos:.6f}", flush=True)
    assert loss == pytest.approx(lref, rel=5e-3)
    assert rel <= 2e-2 and cos >= 0.9995
    # reproducible: per-wave partial gradients are summed in a fixed order
    loss2, grad2 = net.loss_grad(rec, g0, g1)
    assert loss2 == pytest.approx(loss, rel=1e-12)
    assert np.array_equal(grad2.cpu().numpy(), grad.astype(np.float32))
    net.close()


def test_training_lowers_the_loss():
    import paper_2608_15390_amd as P
    X, _, off = _groups(3, groups=2000)
    # targets from a fixed "teacher" network: reachable by training
    teacher = R.init(8)
    Lt, _ = R.forward(teacher, X)
    y = R.softmax_groups(Lt, off)
    rec = _recording(X, y, off)
    net = P.ProposalNet(R.init(4).astype(np.float32))
    l0, _ = net.loss_grad(rec)
    losses = net.train(rec, epochs=6, batch_groups=128, lr=3e-3, seed=1)
    l1, _ = net.loss_grad(rec)
    # the loss is bounded below by the targets' mean entropy; the excess is
    # the mean KL divergence to the teacher, which training must cut
    H = -np.mean([np.sum(y[a:b] * np.log(y[a:b])) for a, b in zip(off[:-1], off[1:])])
    print(f"[gpu] loss {l0:.5f} -> {losses} -> {l1:.5f} (entropy {H:.5f})", flush=True)
    assert l1 - H < 0.5 * (l0 - H)
    assert all(b <= a + 1e-3 for a, b in zip(losses, losses[1:]))
    # the trained parameters give the same loss under the FP64 reference
    th = net.params().cpu().numpy().astype(np.float64)
    lref, _ = R.loss_and_grad(R.bf16(th), R.bf16(X), y, off)
    assert l1 == pytest.approx(lref, rel=5e-3)
    net.close()


def test_training_is_independent_of_the_recording_order():
    """Groups are put in (matrix, trajectory, step) order before training, so
    a recording whose groups sit in another order trains to the same
    parameters bit for bit; two recordings of the same runs (whose slot
    claims race) do too."""
    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import learned as LR
    X, y, off = _groups(5, groups=700)
    G_ = len(off) - 1
    g = np.random.default_rng(6)
    keys = np.stack([g.integers(0, 3, G_), g.permutation(G_), g.integers(0, 50, G_)], axis=1).astype(np.int32)
    perm = g.permutation(G_)
    sizes = np.diff(off)
    Xp = np.concatenate([X[off[i]:off[i + 1]] for i in perm])
    yp = np.concatenate([y[off[i]:off[i + 1]] for i in perm])
    offp = np.concatenate([[0], np.cumsum(sizes[perm])])

    def rec(Xa, ya, offa, ka):
        gi = np.zeros((len(offa) - 1, 4), dtype=np.int32)
        gi[:, 0] = np.diff(offa)
        gi[:, 1:] = ka
        return {"x": _dev(Xa, torch.float32), "y": _dev(ya, torch.float32),
                "gstart": _dev(offa[:-1], torch.int64), "ginfo": _dev(gi, torch.int32), "n_groups": len(offa) - 1}

    outs = []
    for r in (rec(X, y, off, keys), rec(Xp, yp, offp, keys[perm])):
        net = P.ProposalNet(R.init(9).astype(np.float32))
        net.train(r, epochs=3, batch_groups=64, lr=2e-3, seed=4)
        outs.append(net.params().cpu().numpy())
        net.close()
    np.testing.assert_array_equal(outs[0], outs[1])
    # two recordings of the same teacher runs
    mats = G.config_train(2, count=24, n=200)
    params = []
    for _ in range(2):
        r = LR.record_pairs(mats, n_traj=2, seed=3)
        p, _ = LR.train(r, epochs=2, seed=2)
        params.append(p.cpu().numpy())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(params[0], params[1])


def _osched(g, model=None, mix_alpha=0.05):
    return O.Schedule(vertex_rule=g.vertex_rule, sk_policy=g.sk_policy, dm_policy=g.dm_policy,
                      initial_dm=g.initial_dm, K0=g.K0, K=g.K, theta_th=g.theta_th, theta_tr=g.theta_tr,
                      model=model, mix_alpha=mix_alpha, local_gate=g.local_gate)


def _learned_mats():
    mats = G.config_batch(4, count=6, nmin=30, nmax=120)
    # one matrix with vertex lists longer than a wave (the multi-chunk path)
    mats.append(G.planted_bernoulli(90, 0.85, 17, planted="random"))
    # a permuted band matrix (regular local structure, many equal degrees)
    mats.append(G.banded(150, 4, 0.875, 18)[0])
    return mats


@pytest.mark.parametrize("name,alpha", [("learned", 0.05), ("learned_threshold", 0.05), ("learned", 0.0),
                                        ("learned", 1.0), ("learned_gated", 0.05),
                                        ("learned_threshold_gated", 0.05)])
def test_learned_trajectories_match_oracle(name, alpha):
    import paper_2608_15390_amd as P
    mats = _learned_mats()
    model = R.quantize(R.init(11, scale=2.0))
    sched = P.preset(name)
    counts = [60 + 5 * b for b in range(len(mats))]
    print(f"[gpu] learned batch n={[M.n for M in mats]} sched={name} alpha={alpha}", flush=True)
    bt = P.PermEstBatch(mats)
    bt.set_model(_dev(model, torch.float32), alpha)
    out = bt.run(counts, 21, sched, want_hash=True)
    torch.cuda.synchronize()
    if sched.local_gate:  # the fallback fired and both tiers were exercised
        assert sum(r["n_local_sk"] for r in out["results"][:1]) > 0
    lw = out["logw"].cpu().numpy()
    al = out["alive"].cpu().numpy()
    ph = out["path_hash"].cpu().numpy().view(np.uint64)
    off = out["offsets"]
    osch = _osched(sched, model, alpha)
    for b, M in enumerate(mats):
        o = O.run(O.OMatrix(M), osch, seed=21, first=0, count=counts[b], b=b, nthreads=8)
        sl = slice(off[b], off[b + 1])
        np.testing.assert_array_equal(al[sl], o["alive"], err_msg=f"matrix {b}")
        np.testing.assert_array_equal(ph[sl], o["path_hash"], err_msg=f"matrix {b}")
        live = o["alive"] == 1
        np.testing.assert_allclose(lw[sl][live], o["logw"][live], rtol=1e-12, atol=0)
    bt.close()


def test_unquantised_parameters_are_snapped_to_the_grid():
    """set_model snaps to the 1/64 grid: a model off the grid must sample
    exactly like its snapped copy."""
    import paper_2608_15390_amd as P
    M = G.config_small(3)
    raw = R.init(12, scale=1.5)
    sched = P.preset("learned")
    h = P.PermEst(M)
    h.set_model(_dev(raw, torch.float32))
    a = h.run(0, 500, 5, sched, want_hash=True)
    h.set_model(_dev(R.quantize(raw), torch.float32))
    b = h.run(0, 500, 5, sched, want_hash=True)
    assert torch.equal(a["path_hash"], b["path_hash"]) and torch.equal(a["logw"], b["logw"])
    h.close()


def test_learned_needs_a_model_and_rejects_bad_ones():
    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import _native as N
    h = P.PermEst(G.config_small(1))
    with pytest.raises(N.PermEstError) as ei:
        h.run(0, 10, 1, P.preset("learned"))
    assert ei.value.code == N.PE_EINVAL
    bad = R.init(1)
    bad[7] = np.nan
    with pytest.raises(N.PermEstError):
        h.set_model(_dev(bad, torch.float32))
    with pytest.raises(N.PermEstError):
        h.set_model(_dev(R.init(1), torch.float32), mix_alpha=1.5)
    h.close()


def test_learned_estimates_are_unbiased():
    import paper_2608_15390_amd as P
    from oracle import band as B
    mats = [G.config_small(s) for s in range(1, 7)]
    lpers = [math.log(O.ryser(G.to_dense(M))) for M in mats]
    # and a band matrix beyond Ryser's reach (n = 60), exact by the band recursion
    Mb, band = G.banded(60, 3, 0.8, 8)
    mats.append(Mb)
    lpers.append(B.band_log_permanent(band, 3))
    bt = P.PermEstBatch(mats)
    bt.set_model(_dev(R.quantize(R.init(13)), torch.float32))
    out = bt.run(50000, 9, P.preset("learned"), want_logw=False, want_alive=False)
    for r, lp in zip(out["results"], lpers):
        assert abs(math.exp(r["log_estimate"] - lp) - 1) <= 4.5 * r["rse"], (r, lp)
    bt.close()


def _selected_vertex(o):
    """Two-sided minimum degree over the active vertices, ties to the
    smallest id (the rule both sides implement), from the oracle's state."""
    act = o["act"].astype(bool)
    deg = np.where(act, o["deg"], np.iinfo(np.int32).max)
    return int(np.argmin(deg))


def test_recorded_pairs_match_the_oracle():
    import paper_2608_15390_amd as P
    mats = G.config_batch(6, count=4, nmin=30, nmax=80)
    sched = P.preset("fixed_all", dm_policy=0)
    bt = P.PermEstBatch(mats)
    counts = [40] * len(mats)
    rec = bt.record(counts, 3, sched, rec_cap=200000, group_cap=50000, stride=3)
    plain = bt.run(counts, 3, sched, want_hash=True)
    assert rec["n_groups"] > 0
    # recording does not change the trajectories
    for r1, r2 in zip(rec["results"], plain["results"]):
        assert r1["log_estimate"] == r2["log_estimate"] and r1["n_alive"] == r2["n_alive"]
    x = rec["x"].cpu().numpy()
    y = rec["y"].cpu().numpy()
    gs = rec["gstart"].cpu().numpy()
    gi = rec["ginfo"].cpu().numpy()
    # groups tile the records in claim order
    assert gs[0] == 0
    assert np.array_equal(gs[1:], (gs + gi[:, 0])[:-1])
    assert int(gs[-1] + gi[-1, 0]) == rec["n_records"]
    # every (b, k, t) at most once; steps on the stride; targets sum to one
    keys = {(int(a), int(c) & 0xFFFFFFFF, int(d)) for _, a, c, d in gi}
    assert len(keys) == rec["n_groups"]
    assert (gi[:, 3] % 3 == 0).all() and (gi[:, 0] >= 2).all()
    sums = np.add.reduceat(y[:rec["n_records"]].astype(np.float64), gs)
    np.testing.assert_allclose(sums, 1.0, rtol=1e-5)
    osch = _osched(sched)
    rng = np.random.default_rng(0)
    for g in rng.choice(rec["n_groups"], 30, replace=False):
        kc, b, k, t = (int(v) for v in gi[g])
        M = mats[b]
        n = M.n
        A = O.OMatrix(M)
        pre = O.prep(A, osch)
        o = O.probe(A, osch, pre, seed=3, k=k & 0xFFFFFFFF, forced=[], stop_at=t, b=b)
        assert o["stopped"] == 1 and len(o["cand"]) == kc, (b, k, t)
        v = _selected_vertex(o)
        v_row = v < n
        cand = o["cand"].astype(np.int64)
        assert ((cand >= n) == v_row).all()
        sl = slice(gs[g], gs[g] + kc)
        # target: the schedule's proposal in the library's precision (float32
        # entry times float32 scaling), normalised over the group
        vals = np.ones(kc) if M.val is None else None
        if vals is None:
            lo, hi = (M.row_ptr[v], M.row_ptr[v + 1]) if v_row else (M.col_ptr[v - n], M.col_ptr[v - n + 1])
            nb = M.col_idx[lo:hi] + n if v_row else M.row_idx[lo:hi]
            if v_row:
                ent = M.val[lo:hi]
            else:
                ent = np.array([M.val[M.row_ptr[i] + np.searchsorted(M.col_idx[M.row_ptr[i]:M.row_ptr[i + 1]], v - n)]
                                for i in nb], dtype=np.float32)
            emap = dict(zip(nb.tolist(), ent.tolist()))
            vals = np.array([emap[int(u)] for u in cand], dtype=np.float32)
        sc = np.array([o["c"][u - n] if v_row else o["r"][u] for u in cand], dtype=np.float32)
        s = (vals.astype(np.float32) * sc).astype(np.float64)
        np.testing.assert_allclose(y[sl], s / s.sum(), rtol=2e-6, err_msg=str((b, k, t)))
        # features of every candidate edge, from the oracle's definition
        for i, u in enumerate(cand):
            rho, gam = (v, int(u)) if v_row else (int(u), v)
            S, c2 = stats_by_hand(M, o, int(u), v)
            fr = O.learned_features(int(o["deg"][rho]), int(o["deg"][gam]), float(pre.r[rho]),
                                    float(pre.c[gam - n]), t, n, int(v_row), S, c2)
            np.testing.assert_array_equal(x[sl][i], np.asarray(fr, dtype=np.float32), err_msg=str((b, k, t, i)))
    bt.close()


def test_stress_power_law_batch_learned_sampled():
    """Power-law degrees (exponent 2.5 on [2, 200], planted permutation), n
    from 1e4 to 4e4, learned proposal, one autotuned graph-replayed batch
    launch: sampled (matrix, trajectory) pairs are recomputed one by one by
    the oracle."""
    import paper_2608_15390_amd as P
    mats = [G.power_law(n, 100 + i) for i, n in enumerate((10000, 20000, 40000))]
    model = R.quantize(R.init(31, scale=1.5))
    sched = P.preset("learned")
    print(f"[gpu] stress batch n={[M.n for M in mats]} max deg {[int(np.diff(M.row_ptr).max()) for M in mats]}",
          flush=True)
    bt = P.PermEstBatch(mats)
    bt.set_model(_dev(model, torch.float32), 0.01)
    out = bt.run(128, 5, sched, want_hash=True, autotune=True, graph=True)
    torch.cuda.synchronize()
    lw = out["logw"].cpu().numpy()
    al = out["alive"].cpu().numpy()
    ph = out["path_hash"].cpu().numpy().view(np.uint64)
    osch = _osched(sched, model, 0.01)
    rng = np.random.default_rng(1)
    for b, M in enumerate(mats):
        A = O.OMatrix(M)
        pre = O.prep(A, osch)
        for k in sorted(rng.choice(128, 2, replace=False)):
            o = O.run(A, osch, seed=5, first=int(k), count=1, b=b, pre=pre)
            q = 128 * b + int(k)
            assert al[q] == o["alive"][0] and ph[q] == o["path_hash"][0], (b, k)
            if o["alive"][0]:
                assert lw[q] == pytest.approx(o["logw"][0], rel=1e-12)
        assert 0.0 <= out["results"][b]["p_match"] <= 1.0
    bt.close()


def test_trained_network_gains_over_the_method_without_it():
    """What training buys: on an n = 1000, average-degree-8 matrix the
    trained proposal's log-weight variance (the quantity that sets the
    relative error at a given number of trajectories) is far below that of
    the same sampler without the network (outer scaling only) and of an
    untrained network."""
    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import learned as LR
    params, info = LR.train_proposal(G.config_train(1, count=96), epochs=3, seed=2)
    print(f"[gpu] trained: {info['n_groups']} groups, loss {info['loss_initial']:.4f} -> "
          f"{info['loss_per_epoch'][-1]:.4f}", flush=True)
    assert info["loss_per_epoch"][-1] < info["loss_initial"]
    M = G.planted_uniform(1000, 7000, 5)
    h = P.PermEst(M)
    res = {}
    h.set_model(params, LR.MIX_ALPHA)
    res["trained"] = h.run(0, 20000, 3, P.preset("learned"), want_logw=False, want_alive=False)["result"]
    h.set_model(torch.as_tensor(LR.init_params(5), device="cuda"), LR.MIX_ALPHA)
    res["untrained"] = h.run(0, 20000, 3, P.preset("learned"), want_logw=False, want_alive=False)["result"]
    res["outer_only"] = h.run(0, 20000, 3, P.preset("plain", initial_dm=1, K0=100), want_logw=False,
                              want_alive=False)["result"]
    h.close()
    for k, r in res.items():
        print(f"[gpu] {k:10s} Var ln X {r['var_logw']:8.3f} p_match {r['p_match']:.4f} ESS {r['ess']:.2f}",
              flush=True)
    assert res["trained"]["var_logw"] < 0.5 * res["outer_only"]["var_logw"]
    assert res["trained"]["var_logw"] < 0.8 * res["untrained"]["var_logw"]
    assert res["trained"]["p_match"] >= res["outer_only"]["p_match"]
