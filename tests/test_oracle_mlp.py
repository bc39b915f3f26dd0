"""Pins of the FP64 network reference and of the learned proposal."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import mlp as R
from oracle import oracle as O
from paper_2608_15390_amd import inputs as G
from oracle_tools import dense_values, enumerate_tree, stats_by_hand


def _data(seed, groups=12):
    g = np.random.default_rng(seed)
    sizes = g.integers(2, 7, size=groups)
    off = np.concatenate([[0], np.cumsum(sizes)])
    X = g.normal(0, 1, (off[-1], R.IN))
    X[:, 6:] = 0
    y = np.empty(off[-1])
    for a, b in zip(off[:-1], off[1:]):
        p = g.random(b - a) + 0.05
        y[a:b] = p / p.sum()
    return X, y, off


def test_backward_matches_finite_differences():
    X, y, off = _data(1)
    th = R.init(3)
    _, grad = R.loss_and_grad(th, X, y, off)
    g = np.random.default_rng(5)
    for idx in g.choice(R.NPARAM, 60, replace=False):
        e = np.zeros(R.NPARAM)
        e[idx] = 1e-6
        lp, _ = R.loss_and_grad(th + e, X, y, off)
        lm, _ = R.loss_and_grad(th - e, X, y, off)
        fd = (lp - lm) / 2e-6
        assert grad[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_gradient_vanishes_when_the_network_already_matches_the_targets():
    X, _, off = _data(2)
    th = R.init(4)
    L, _ = R.forward(th, X)
    y = R.softmax_groups(L, off)
    loss, grad = R.loss_and_grad(th, X, y, off)
    assert np.abs(grad).max() < 1e-12
    # and the loss equals the mean entropy of the targets
    ent = -sum(np.sum(y[a:b] * np.log(y[a:b])) for a, b in zip(off[:-1], off[1:])) / (len(off) - 1)
    assert loss == pytest.approx(ent, rel=1e-12)


def test_plog2_is_piecewise_linear_log2():
    for k in range(-20, 21):
        assert O.plog2(2.0 ** k) == k
    assert O.plog2(3.0) == 1.5
    assert O.plog2(0.75) == -0.5
    xs = np.geomspace(1e-6, 1e6, 200)
    v = [O.plog2(x) for x in xs]
    assert all(b >= a for a, b in zip(v, v[1:]))
    assert max(abs(p - math.log2(x)) for p, x in zip(v, xs)) < 0.09


def _float32_logit(model, x, order8, order64):
    """The grid network in float32 with permuted summation orders."""
    W1, b1, W2, b2, w3, b3 = [np.asarray(a, dtype=np.float32) for a in R.unpack(model)]
    x = np.asarray(x, dtype=np.float32)
    q = lambda a: np.float32(min(max(np.rint(max(float(a), 0.0) * 64), 0), 255) / 64)  # noqa: E731
    h1 = np.array([q(_sum32(b1[j], [x[k] * W1[k, j] for k in order8])) for j in range(64)], np.float32)
    h2 = np.array([q(_sum32(b2[j], [h1[k] * W2[k, j] for k in order64])) for j in range(64)], np.float32)
    acc = _sum32(b3[0], [h2[k] * w3[k] for k in order64])
    return int(min(max(np.rint(float(acc) * 16), -1024), 1023))


def _sum32(start, terms):
    acc = np.float32(start)
    for t in terms:
        acc = np.float32(acc + np.float32(t))
    return acc


def test_grid_network_is_exact_in_float32_in_any_order():
    """Every partial sum of the quantised network is a float32 number, so a
    float32 evaluation in any summation order reproduces the oracle."""
    g = np.random.default_rng(7)
    model = R.quantize(R.init(9, scale=1.5))
    for trial in range(8):
        x = O.learned_features(int(g.integers(0, 40)), int(g.integers(0, 40)), float(g.uniform(0.01, 3)),
                               float(g.uniform(0.01, 3)), int(g.integers(0, 100)), 100, trial % 2,
                               int(g.integers(1 << 15, 1 << 26)), int(g.integers(0, 300)))
        ref = O.learned_logit(model, x)
        for _ in range(3):
            order8 = [int(i) for i in g.permutation(8)]
            order64 = [int(i) for i in g.permutation(64)]
            assert _float32_logit(model, x, order8, order64) == ref


def test_candidate_features_by_hand():
    # S_u = 1.5 * 2^20: plog2(1.5) = 0.5, x6 = Q(0.125) = 8/64
    x = O.learned_features(3, 2, 1.0, 1.0, 5, 10, 1, 3 << 19, 2)
    assert x[6] == 0.125 and x[7] == 2 / 64
    # degrees and counts clamp at 255, t/n on the 1/64 grid, r0 = 2 -> plog2 = 1
    x = O.learned_features(300, 7, 2.0, 0.5, 1, 3, 0, 1 << 20, 1000)
    assert x[0] == 255 / 64 and x[1] == 7 / 64 and x[7] == 255 / 64
    assert x[2] == 0.25 and x[3] == -0.25 and x[4] == 21 / 64 and x[5] == 0.0 and x[6] == 0.0


@pytest.mark.parametrize("name", ["learned", "learned_threshold"])
def test_learned_proposal_at_a_step_from_its_definition(name):
    """At a stopped step the oracle's learned proposal equals the one
    rebuilt here from the state snapshot: features (with S_u and the
    degree-<=2 count computed by hand), grid logits, integer weights."""
    model = R.quantize(R.init(21, scale=2.0))
    sched = O.preset(name).replace(model=model, mix_alpha=0.1)
    g = np.random.default_rng(3)
    checked = 0
    for trial in range(12):
        M = G.planted_bernoulli(40, 0.12, int(g.integers(1 << 30)), planted="random")
        A = O.OMatrix(M)
        pre = O.prep(A, sched)
        n = M.n
        t = int(g.integers(0, 30))
        o = O.probe(A, sched, pre, seed=5, k=trial, forced=[], stop_at=t)
        if o["stopped"] != 1 or len(o["cand"]) < 2:
            continue
        act = o["act"].astype(bool)
        v = int(np.argmin(np.where(act, o["deg"], 1 << 30)))
        v_row = v < n
        L = []
        for u in o["cand"]:
            u = int(u)
            rho, gam = (v, u) if v_row else (u, v)
            S, c2 = stats_by_hand(M, o, u, v)
            x = O.learned_features(int(o["deg"][rho]), int(o["deg"][gam]), float(pre.r[rho]),
                                   float(pre.c[gam - n]), t, n, int(v_row), S, c2)
            L.append(O.learned_logit(model, x))
        w = O.learned_weights(L, 0.1).astype(np.float64)
        np.testing.assert_array_equal(o["prob"], w / w.sum())
        checked += 1
    assert checked >= 6


def test_learned_weights_properties():
    for k in (2, 3, 7, 30):
        g = np.random.default_rng(k)
        L = g.integers(-300, 300, size=k)
        w = O.learned_weights(L, 0.05).astype(np.int64)
        assert (w >= 1).all()
        assert abs(int(w.sum()) - 2 ** 24) <= k
        assert (w >= int(0.05 * 2 ** 24 / k) - 1).all()      # the uniform share
        order = np.argsort(-L, kind="stable")
        assert (np.diff(w[order]) <= 0).all()                  # monotone in the logit
    # equal logits give equal weights
    w = O.learned_weights([5, 5, 5, 5], 0.3)
    assert len(set(w.tolist())) == 1


def _learned(model, **kw):
    base = O.preset("local_nodm")
    return base.replace(sk_policy=O.SK_LEARNED, model=model, **kw)


@pytest.mark.parametrize("initial_dm", [0, 1])
def test_learned_proposal_enumeration_is_exact(initial_dm):
    """Unbiasedness with the learned proposal: the weight uses the
    probability actually sampled, so E[X] = per(A) exactly."""
    model = R.quantize(R.init(11, scale=2.0))
    sched = _learned(model, initial_dm=initial_dm, K0=20 if initial_dm else 0)
    g = np.random.default_rng(12)
    for t in range(10):
        n = int(g.integers(2, 8))
        M = G.planted_bernoulli(n, float(g.uniform(0.2, 0.7)), int(g.integers(1 << 30)), planted="random")
        if t % 3 == 0:
            M = G.with_weights(M, t)
        A = O.OMatrix(M)
        pre = O.prep(A, sched)
        E, _, _ = enumerate_tree(A, sched, pre)
        assert E == pytest.approx(O.ryser_f64(dense_values(M)), rel=1e-12)


def test_learned_proposal_mean_within_ci():
    model = R.quantize(R.init(13))
    M = G.config_small(2)
    per = O.ryser(G.to_dense(M))
    out = O.run(O.OMatrix(M), _learned(model), seed=3, count=20000, nthreads=8)
    st = O.stats(out["logw"], out["alive"])
    assert abs(math.exp(st["log_estimate"]) / per - 1) <= 4.5 * st["rse"]


def _etab_exact(d):
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    v = Decimal(16777216) * (Decimal(-d) / Decimal(16)).exp()
    return int(v.to_integral_value(rounding="ROUND_HALF_EVEN")), v


def test_softmax_table_is_rounding_stable_and_matches_the_oracle():
    """E[d] = rint(2^24 exp(-d/16)): every entry sits at least 2e-9 (relative)
    away from a rounding boundary, so any exp correct to 1e-12 -- the
    oracle's and the device's -- yields the same integer table; the oracle's
    integer weights for two candidates with logit gap d follow from it."""
    for d in range(2048):
        e, v = _etab_exact(d)
        if v >= 0.5:
            frac = v - int(v)
            assert abs(float(frac) - 0.5) / float(v) > 1e-12
    for d in (0, 1, 7, 16, 100, 333, 1000, 2047, 2048, 5000):
        e = _etab_exact(d)[0] if d < 2048 else 0
        w = O.learned_weights([0, -d], 0.0).astype(np.int64)
        S = (1 << 24) + e
        assert w[0] == max(1, round((1 << 24) * ((1 << 24) / S)))
        assert w[1] == max(1, round((1 << 24) * (e / S)))


def test_feature_definitions_have_exact_integer_forms():
    """The FP64 definitions of the logarithmic and phase features equal
    integer forms read off the inputs' bits (the forms the matrix-core
    kernel uses): for a positive normal binary32 s, 64 plog2(s)/4 is
    (bits >> 19) - 2032 plus the low 19 bits over 2^19, rounded half to even;
    for an integer S >= 1 with 2^p <= S < 2^(p+1), 16 plog2(S / 2^20) is
    16 p + 16 S / 2^p - 16 - 320; rint(64 t / n) is the exact rational's
    rounding. Checked against the oracle's features on ties, powers of two
    and random values."""
    import struct

    def clamp(k):
        return min(255, max(-256, k))

    def from_bits(s):
        b = struct.unpack("<I", struct.pack("<f", s))[0]
        q, r = b >> 19, b & 0x7FFFF
        return clamp(q + (1 if (r > 0x40000 or (r == 0x40000 and q & 1)) else 0) - 2032) / 64.0

    def from_int(S):
        if S == 0:
            return clamp(-32) / 64.0
        p = S.bit_length() - 1
        t16 = S << 4
        q = t16 >> p
        up = 0
        if p > 0:
            r, half = t16 & ((1 << p) - 1), 1 << (p - 1)
            up = 1 if (r > half or (r == half and q & 1)) else 0
        return clamp(16 * p + q + up - 16 - 320) / 64.0

    g = np.random.default_rng(3)
    floats = [np.float32(v) for v in g.lognormal(0.0, 3.0, 4000)]
    floats += [np.float32(2.0 ** k * (1 + j / 16 + 1 / 32)) for k in range(-30, 30, 3) for j in range(16)]
    floats += [np.float32(2.0 ** k) for k in range(-126, 128, 7)]
    for s in floats:
        x = O.learned_features(3, 4, float(s), float(s), 0, 10, 1, 0, 0)
        assert x[2] == from_bits(s) and x[3] == from_bits(s), s
    ints = list(range(0, 600)) + [int(v) for v in g.integers(0, 2 ** 40, 3000)]
    ints += [(2 ** p) * (32 + 2 * j + 1) // 32 for p in range(5, 40) for j in range(16)]
    for S in ints:
        x = O.learned_features(3, 4, 1.0, 1.0, 0, 10, 1, S, 0)
        assert x[6] == from_int(S), S
    for n in (1, 2, 3, 7, 64, 100, 1000, 12800, 100000):
        for t in sorted({0, 1, n // 2, n - 1} | set(int(v) for v in g.integers(0, n, 50))):
            x = O.learned_features(3, 4, 1.0, 1.0, t, n, 1, 0, 0)
            q, r = divmod(64 * t, n)
            k = q + (1 if (2 * r > n or (2 * r == n and q & 1)) else 0)
            assert x[4] == clamp(k) / 64.0, (t, n)


# ------------------------------------------- learned proposal, gated fallback
def _gated(model, **kw):
    return _learned(model, local_gate=1, mix_alpha=0.05, **kw)


@pytest.mark.parametrize("dm", [O.DM_NONE, O.DM_THRS])
@pytest.mark.parametrize("initial_dm", [0, 1])
def test_gated_fallback_enumeration_is_exact(initial_dm, dm):
    """The fallback only changes which positive proposal a step samples
    from, and the weight still divides by the probability sampled, so
    E[X] = per(A) exactly (Sec. 2) with the gate on."""
    model = R.quantize(R.init(11, scale=2.0))
    sched = _gated(model, initial_dm=initial_dm, K0=20 if initial_dm else 0, dm_policy=dm, theta_th=0.45)
    g = np.random.default_rng(13 + dm)
    fired = 0
    for t in range(10):
        n = int(g.integers(2, 8))
        M = G.planted_bernoulli(n, float(g.uniform(0.2, 0.7)), int(g.integers(1 << 30)), planted="random")
        if t % 3 == 0:
            M = G.with_weights(M, t)
        A = O.OMatrix(M)
        pre = O.prep(A, sched)
        E, _, _ = enumerate_tree(A, sched, pre)
        assert E == pytest.approx(O.ryser_f64(dense_values(M)), rel=1e-12)
        fired += int(O.run(A, sched, seed=1, count=50, pre=pre)["counters"][:, 3].sum())
    assert fired > 0


def _scaled_weights_by_hand(M, o, v, cand):
    """Integer weights of Eq. (q) from the snapshot's r, c: s = B c (row v)
    or B r (column v) in binary32, w = max(1, rint(2^24 s / s_max))."""
    n = M.n
    D = dense_values(M)
    s = []
    for u in cand:
        u = int(u)
        if v < n:
            s.append(np.float32(D[v, u - n]) * np.float32(o["c"][u - n]))
        else:
            s.append(np.float32(D[u, v - n]) * np.float32(o["r"][u]))
    s = np.array(s, dtype=np.float32)
    smax = s.max()
    ratio = (s / smax).astype(np.float32) * np.float32(16777216.0)
    return np.maximum(1.0, np.rint(ratio)).astype(np.float64)


def test_gated_fallback_steps_from_their_definition():
    """Along gated trajectories: a step right after a repair draws from the
    scaled proposal of Eq. (q) built here from the snapshot's r, c; r and c
    change only across a step whose sampled probability fell below
    theta_th (the repair), and otherwise stay as they were."""
    model = R.quantize(R.init(21, scale=2.0))
    sched = _gated(model, initial_dm=1, K0=30, theta_th=0.4)
    g = np.random.default_rng(5)
    fb_checked = plain_checked = 0
    for trial in range(8):
        M = G.planted_bernoulli(30, 0.15, int(g.integers(1 << 30)), planted="random")
        if trial % 2:
            M = G.with_weights(M, trial)
        A = O.OMatrix(M)
        pre = O.prep(A, sched)
        n = M.n
        full = O.probe(A, sched, pre, seed=9, k=trial, forced=[], stop_at=-1)
        ev = full["events"]
        prev = None
        for t in range(full["steps"]):
            o = O.probe(A, sched, pre, seed=9, k=trial, forced=[], stop_at=t)
            assert o["stopped"] == 1
            act = o["act"].astype(bool)
            v = int(np.argmin(np.where(act, o["deg"], 1 << 30)))
            repaired = t > 0 and ev[2 * (t - 1) + 1] == 1
            if prev is not None:
                same = np.array_equal(o["r"], prev["r"]) and np.array_equal(o["c"], prev["c"])
                if not repaired:
                    assert same, (trial, t)
            if repaired and len(o["cand"]) >= 2:
                w = _scaled_weights_by_hand(M, o, v, o["cand"])
                np.testing.assert_array_equal(o["prob"], w / w.sum())
                fb_checked += 1
            elif len(o["cand"]) >= 2:
                plain_checked += 1
            prev = o
    assert fb_checked >= 5 and plain_checked >= 5
