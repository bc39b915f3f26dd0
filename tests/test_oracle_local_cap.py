"""Pins of the oracle's bounded-work local repair (the sampled variant of
Eq. (local) that Sec. 3.3 proposes for hub vertices): a list longer than the
cap B is examined at B systematic sample positions (offset from the
trajectory's Philox stream) and its normalisation sum is the sampled sum
scaled by the residual degree over the sampled active count.

* With a cap no list exceeds, the repair is Eq. (local) itself: paths and
  weights equal the exact repair's bit for bit.
* Exact trajectory-tree enumeration gives per(A) to 1e-12 at small caps
  (Sec. 2: only the proposal changes, the estimator stays unbiased).
* The sets and values of one repair are rebuilt from probe snapshots with
  dense numpy arrays and binary32 arithmetic written out here."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from oracle_tools import dense_values, enumerate_tree, residual_adjacency
from paper_2608_15390_amd import inputs as G

LOCAL = ["local_threshold", "local_tracked", "local_nodm"]


def _family(seed, count, nmax=8):
    g = np.random.default_rng(seed)
    for t in range(count):
        n = int(g.integers(3, nmax))
        M = G.planted_bernoulli(n, float(g.uniform(0.35, 0.8)), int(g.integers(1 << 30)), planted="random")
        if t % 3 == 0:
            M = G.with_weights(M, t)
        yield M


@pytest.mark.parametrize("name", LOCAL)
def test_cap_above_every_list_is_the_exact_repair(name):
    for i, M in enumerate([G.planted_uniform(150, 900, 3), G.power_law(300, 5, dmax=40),
                           G.with_weights(G.planted_uniform(120, 600, 4), 1)]):
        A = O.OMatrix(M)
        longest = int(max(np.diff(M.row_ptr).max(), np.diff(M.col_ptr).max()))
        ex = O.run(A, O.preset(name), seed=9, count=40, want_path=True)
        cp = O.run(A, O.preset(name).replace(local_cap=longest), seed=9, count=40, want_path=True)
        for k in ("alive", "path", "counters", "path_hash"):
            assert np.array_equal(ex[k], cp[k]), (i, k)
        assert np.array_equal(ex["logw"], cp["logw"])
        # and a small cap changes the proposal on these lists
        sm = O.run(A, O.preset(name).replace(local_cap=2), seed=9, count=40, want_path=True)
        assert not np.array_equal(ex["path"], sm["path"])


@pytest.mark.parametrize("name", LOCAL)
@pytest.mark.parametrize("cap", [1, 2, 3])
def test_enumeration_gives_exact_permanent_with_sampled_repair(name, cap):
    sched = O.preset(name).replace(local_cap=cap)
    for M in _family(31 + cap, 10):
        A = O.OMatrix(M)
        pre = O.prep(A, sched)
        E, _, n_paths = enumerate_tree(A, sched, pre)
        per = O.ryser_f64(dense_values(M))
        assert E == pytest.approx(per, rel=1e-12)
        if M.val is None:
            assert n_paths == round(per)


def _positions(seed, k, t, x, L, cap):
    x, L = int(x), int(L)
    if L <= cap:
        return list(range(L))
    R = O.rng64(seed, k, 0, t, 0x80000000 | x) & 0xFFFFFFFF
    o = (R * L) >> 32
    return [(o + (i * L) // cap) % L for i in range(cap)]


@pytest.mark.parametrize("dm", [O.DM_NONE, O.DM_THRS])
@pytest.mark.parametrize("cap", [2, 3])
def test_sampled_repair_follows_its_definition(dm, cap):
    sched = O.Schedule(sk_policy=O.SK_LOCAL, dm_policy=dm, initial_dm=1, K0=5, theta_th=0.5, local_cap=cap)
    g = np.random.default_rng(77 + cap)
    checked = sampled = filtered = 0
    f32 = np.float32
    for trial in range(8):
        if trial >= 6:
            # block upper-triangular: the off-diagonal block lies in no perfect
            # matching, so the initial filter removes it from every list
            h = np.random.default_rng(trial)
            blk = (h.random((14, 14)) < 0.45) | np.eye(14, dtype=bool)
            blk[7:, :7] = False
            r, c = np.nonzero(blk)
            perm_r, perm_c = h.permutation(14), h.permutation(14)
            M = G.from_coo(14, perm_r[r], perm_c[c])
        else:
            M = G.planted_bernoulli(14, 0.35, int(g.integers(1 << 30)), planted="random")
        if trial % 2:
            M = G.with_weights(M, trial)
        A = O.OMatrix(M)
        pre = O.prep(A, sched)
        n = M.n
        D = dense_values(M).astype(np.float32)
        full = O.probe(A, sched, pre, seed=5, k=trial, forced=[], stop_at=-1)
        path = full["path"].reshape(-1, 2)
        # the lists trajectories start from: entries the initial filter kept,
        # in list order (rows by column, columns by row)
        kept = pre.removed[: M.nnz] == 0
        filtered += int((~kept).sum())
        row_lists = [[int(M.col_idx[e]) for e in range(M.row_ptr[i], M.row_ptr[i + 1]) if kept[e]]
                     for i in range(n)]
        col_lists = [[i for i in range(n) for e in range(M.row_ptr[i], M.row_ptr[i + 1])
                      if kept[e] and M.col_idx[e] == j] for j in range(n)]
        for t in range(min(full["steps"], n - 1)):
            bef = O.probe(A, sched, pre, seed=5, k=trial, forced=path[:t, 1].tolist(), stop_at=t)
            aft = O.probe(A, sched, pre, seed=5, k=trial, forced=path[:t + 1, 1].tolist(), stop_at=t + 1)
            if aft["stopped"] != 1:
                continue
            v, u = path[t]
            rho, gam = (v, u - n) if v < n else (u, v - n)
            Bt = residual_adjacency(M, bef["act"], bef["removed"])
            Bn = residual_adjacency(M, aft["act"], aft["removed"])

            def row_sample(i):   # sampled child neighbours (columns) of row i, in sample order
                cols = row_lists[i]
                pos = _positions(5, trial, t, i, len(cols), cap)
                return [cols[p] for p in pos if Bn[i, cols[p]]]

            def col_sample(j):   # sampled child neighbours (rows) of column j
                rows = col_lists[j]
                pos = _positions(5, trial, t, n + j, len(rows), cap)
                return [rows[p] for p in pos if Bn[rows[p], j]]

            Nr = set(np.nonzero(Bt[rho])[0]) - {gam}
            Ng = set(np.nonzero(Bt[:, gam])[0]) - {rho}
            C_loc = set(Nr) | {j for i in Ng for j in row_sample(i)}
            R_loc = set(Ng) | {i for j in Nr for i in col_sample(j)}
            r0, c0 = bef["r"].astype(np.float32), bef["c"].astype(np.float32)
            for i in range(n):
                if i not in R_loc:
                    assert aft["r"][i] == bef["r"][i]
                    continue
                L = len(row_lists[i])
                if L <= cap:
                    s = (D[i] * Bn[i] * c0).astype(np.float64).sum()
                    if s > 0:
                        assert aft["r"][i] * s == pytest.approx(1.0, rel=3e-7 * max(1, Bn[i].sum()))
                    continue
                js = row_sample(i)
                acc = f32(0)
                for j in js:
                    acc = f32(acc + f32(D[i, j] * c0[j]))
                want = bef["r"][i]
                if js and acc != 0:
                    want = float(f32(1) / f32(acc * f32(f32(Bn[i].sum()) / f32(len(js)))))
                assert aft["r"][i] == want
                sampled += 1
            for j in range(n):
                if j not in C_loc:
                    assert aft["c"][j] == bef["c"][j]
                    continue
                L = len(col_lists[j])
                if L <= cap:
                    s = (D[:, j] * Bn[:, j] * r0).astype(np.float64).sum()
                    if s > 0:
                        assert aft["c"][j] * s == pytest.approx(1.0, rel=3e-7 * max(1, Bn[:, j].sum()))
                    continue
                is_ = col_sample(j)
                acc = f32(0)
                for i in is_:
                    acc = f32(acc + f32(D[i, j] * r0[i]))
                want = bef["c"][j]
                if is_ and acc != 0:
                    want = float(f32(1) / f32(acc * f32(f32(Bn[:, j].sum()) / f32(len(is_)))))
                assert aft["c"][j] == want
                sampled += 1
            checked += 1
    assert checked > 20 and sampled > 50 and filtered > 10
