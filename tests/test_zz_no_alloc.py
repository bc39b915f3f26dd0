"""perm_est_run_range_noalloc against perm_est_run_range: the same ids give
the same trajectories (paths, alive flags, hashes, counters bit for bit,
ln X identical) and the same statistics, on two calls in a row, the second
with fewer trajectories; a second handle with a smaller matrix then reuses
the GPU's scratch array.  Run alone and after the other GPU tests."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import mlp as R
from paper_2608_15390_amd import inputs as G

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

STAT_KEYS = ("log_estimate", "p_match", "rel_spread", "rse", "ess", "var_logw", "max_logw", "n_traj", "n_alive",
             "n_dm", "n_full_sk", "n_local_sk", "n_steps", "n_entries_scanned", "n_decrements",
             "n_local_entries", "n_local_values")


def _same(a, b, what):
    for k in ("logw", "alive", "path_hash", "counters"):
        if k in a or k in b:
            assert torch.equal(a[k], b[k]), (what, k)
    for k in STAT_KEYS:
        x, y = a["result"][k], b["result"][k]
        assert x == y or (x != x and y != y), (what, k, x, y)
    # network tiles depend on which trajectories share a wave (four per
    # wave share 16-record tiles), so a smaller grid may pack them otherwise
    assert (a["result"]["n_mlp_tiles"] > 0) == (b["result"]["n_mlp_tiles"] > 0), what


def _pair(est, first, count, seed, sched, **want):
    print(f"[gpu] no-alloc n={est.n} ids={first}+{count} sched={sched.as_dict()} want={want}", flush=True)
    ref = est.run(first, count, seed, sched, **want)
    got = est.run(first, count, seed, sched, noalloc=True, **want)
    torch.cuda.synchronize()
    _same(ref, got, (est.n, first, count))


@pytest.mark.parametrize("name", ["plain", "local_nodm", "learned", "adaptive_threshold"])
def test_noalloc_matches_run_range_twice_then_smaller(name):
    import paper_2608_15390_amd as P
    sched = P.preset(name)
    model = torch.as_tensor(R.quantize(R.init(41, scale=1.5)), dtype=torch.float32, device="cuda")
    big = G.planted_uniform(3000, 21000, 31) if name != "adaptive_threshold" else G.planted_uniform(300, 2100, 31)
    small = G.planted_uniform(900, 6300, 32) if name != "adaptive_threshold" else G.planted_uniform(60, 420, 32)
    est = P.PermEst(big)
    est.set_model(model, 0.05)
    want = dict(want_hash=True, want_counters=True)
    _pair(est, 5, 700, 3, sched, **want)              # outputs given by the caller
    _pair(est, 11, 130, 4, sched, want_logw=False)    # fewer, logw left to the scratch
    est.close()
    est = P.PermEst(small)
    est.set_model(model, 0.05)
    _pair(est, 0, 64, 5, sched, **want)
    est.close()


def test_noalloc_large_learned_state_in_scratch_slots():
    """n = 1e5, learned proposal: the per-trajectory state lives in the
    scratch's slots (fewer concurrent trajectories, same results)."""
    import paper_2608_15390_amd as P
    sched = P.preset("learned")
    model = torch.as_tensor(R.quantize(R.init(42, scale=1.5)), dtype=torch.float32, device="cuda")
    est = P.PermEst(G.config_large(1))
    est.set_model(model, 0.01)
    _pair(est, 100, 300, 1, sched, want_hash=True, want_counters=True)
    _pair(est, 7, 40, 1, sched, want_hash=True)
    est.close()


def test_noalloc_rejections():
    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import _native as N
    est = P.PermEst(G.planted_uniform(200, 1400, 33))
    # preprocessing of this (initial_dm, K0) has not run on the handle yet
    with pytest.raises(N.PermEstError) as ei:
        est.run(0, 10, 1, P.preset("local_nodm"), noalloc=True)
    assert ei.value.code == N.PE_EINVAL
    est.run(0, 10, 1, P.preset("local_nodm"))
    # the outputs left NULL for 3e6 trajectories do not fit the scratch
    with pytest.raises(N.PermEstError) as ei:
        est.run(0, 3_000_000, 1, P.preset("local_nodm"), noalloc=True, want_logw=False, want_alive=False)
    assert ei.value.code == N.PE_ENOTSUP
    est.close()
