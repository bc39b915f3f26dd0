"""Multi-seed consensus diagnostics (Sec. 4.4): the oracle's statement of
the definitions pinned by the paper's printed critical value, a standard
t-table value, coverage and false-alarm rates of the intervals on simulated
runs whose spread is known, scale invariance and degenerate cases; then the
library's host implementation (perm_est_consensus, no GPU involved) against
the oracle on random inputs."""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import consensus as CO


def _runs(Y, sd, M=10_000, alive=None, ess=None):
    """Run records for estimates Y[v][r] whose within-run standard error is sd[v][r]."""
    Y = np.asarray(Y, dtype=np.float64)
    sd = np.broadcast_to(np.asarray(sd, dtype=np.float64), Y.shape)
    ly = np.log(Y)
    rse = sd / Y
    n = np.full(Y.shape, M)
    al = np.full(Y.shape, M if alive is None else alive)
    es = np.full(Y.shape, 5000.0 if ess is None else ess)
    return ly, rse, n, al, es


def test_bonferroni_critical_value_printed_in_the_paper():
    # five variants, ten pairs, alpha 0.05: Phi^{-1}(0.9975) ~ 2.81
    assert CO.bonferroni_critical(5) == pytest.approx(2.807, abs=5e-4)
    assert round(CO.bonferroni_critical(5), 2) == 2.81


def test_t_critical_matches_tables():
    # two-sided 95 % points of Student's t (standard tables)
    for df, v in ((1, 12.706), (2, 4.303), (4, 2.776), (10, 2.228), (30, 2.042)):
        assert CO.t_critical(df) == pytest.approx(v, abs=6e-4)


def test_identical_runs_give_zero_spread_between_variants():
    ly, rse, n, al, es = _runs([[5.0] * 5] * 5, 0.1)
    c = CO.consensus(ly, rse, n, al, es)
    assert c["d_max"] == 0.0 and c["variant_ratio"] == 1.0
    # e_seed = 0, so e_P = e_in = sqrt(5 * 0.1^2) / 5 for every variant
    assert c["rel_e"] == pytest.approx([math.sqrt(5) * 0.1 / 5 / 5.0] * 5, rel=1e-12)
    assert c["provisional"]


def test_scale_invariance_in_log_space():
    g = np.random.default_rng(3)
    Y = g.uniform(0.5, 2.0, size=(5, 5))
    ly, rse, n, al, es = _runs(Y, 0.05 * Y)
    a = CO.consensus(ly, rse, n, al, es)
    b = CO.consensus(ly + 5000.0, rse, n, al, es)   # exp(5000 + ln Y) overflows FP64
    assert b["log_p_con"] - a["log_p_con"] == pytest.approx(5000.0, abs=1e-9)
    assert b["log_e_con"] - a["log_e_con"] == pytest.approx(5000.0, abs=1e-9)
    for k in ("rel_half_width", "variant_ratio", "d_max"):
        assert b[k] == pytest.approx(a[k], rel=1e-12)


def test_consensus_interval_covers_the_truth_at_the_nominal_rate():
    """Runs Y ~ N(mu, s^2) reporting their true standard error s: P_con has
    standard deviation s / sqrt(V R), which e_con must estimate (e_P >= e_in
    makes the interval conservative, not wider by a factor)."""
    g = np.random.default_rng(7)
    mu, s, V, R, reps = 100.0, 4.0, 5, 5, 4000
    cover = 0
    widths = []
    for _ in range(reps):
        Y = g.normal(mu, s, size=(V, R))
        ly, rse, n, al, es = _runs(Y, s)
        c = CO.consensus(ly, rse, n, al, es)
        pc, ec = math.exp(c["log_p_con"]), math.exp(c["log_e_con"])
        cover += abs(pc - mu) <= 1.96 * ec
        widths.append(ec)
    rate = cover / reps
    assert 0.94 <= rate <= 0.995, rate
    # e_con is about s / sqrt(V R) (between that and ~1.5x it, from the max with e_seed)
    assert s / math.sqrt(V * R) <= np.median(widths) <= 1.5 * s / math.sqrt(V * R)


def test_bonferroni_false_alarm_and_power():
    g = np.random.default_rng(11)
    s, V, R, reps = 1.0, 5, 5, 3000
    alarms = 0
    for _ in range(reps):
        Y = g.normal(50.0, s, size=(V, R))
        c = CO.consensus(*_runs(Y, s))
        alarms += c["d_max"] > c["c_bonf"]
    assert alarms / reps <= 0.05
    hits = 0
    for _ in range(300):
        Y = g.normal(50.0, s, size=(V, R))
        Y[2] += 5.0 * s  # one variant off by 5 sd: 5 / sqrt(2 / 5) = 7.9 standard errors
        c = CO.consensus(*_runs(Y, s))
        hits += c["d_max"] > c["c_bonf"]
    assert hits / 300 >= 0.99


def test_status_rules():
    Y = np.full((5, 5), 10.0)
    base = _runs(Y, 0.01)
    assert CO.consensus(*base)["provisional"]
    ly, rse, n, al, es = base
    c = CO.consensus(ly, rse, n, al, np.where(np.arange(25).reshape(5, 5) == 7, 5.0, es))
    assert not c["checks"]["ess_at_least_1000"] and not c["provisional"] and c["min_ess"] == 5.0
    c = CO.consensus(ly, rse, n, np.where(np.arange(25).reshape(5, 5) == 3, 999, al), es)
    assert not c["checks"]["alive_at_least_1000"]
    c = CO.consensus(*_runs(Y, 0.6 * Y))   # 1.96 e_con / P_con = 1.96 * 0.6 / 5 > 0.1
    assert not c["checks"]["half_width_within_10pct"]
    Y2 = Y.copy()
    Y2[0] = 20.0
    c = CO.consensus(*_runs(Y2, 0.01))
    assert not c["checks"]["t_intervals_intersect"] and not c["checks"]["d_max_within_bonferroni"]
    assert c["variant_ratio"] == pytest.approx(2.0)
    n0 = n.copy()
    n0[4, 4] = 0
    assert not CO.consensus(ly, rse, n0, al, es)["checks"]["all_runs_present"]


def _lib_consensus(ly, rse, n, al, es, alpha=0.05):
    import paper_2608_15390_amd as P
    V, R = ly.shape
    runs = [[{"log_estimate": float(ly[p, r]), "rse": float(rse[p, r]), "n_traj": int(n[p, r]),
              "n_alive": int(al[p, r]), "ess": float(es[p, r])} for r in range(R)] for p in range(V)]
    return P.consensus(runs, alpha)


@pytest.mark.parametrize("V,R", [(2, 2), (5, 5), (3, 7), (6, 4)])
def test_library_matches_oracle(V, R):
    g = np.random.default_rng(100 * V + R)
    for trial in range(20):
        ly = g.normal(0.0, 0.05 if trial % 2 else 0.5, size=(V, R)) + g.uniform(-3000, 3000)
        rse = g.uniform(0.001, 0.2, size=(V, R))
        n = g.integers(1, 100_000, size=(V, R))
        al = np.minimum(n, g.integers(500, 100_000, size=(V, R)))
        es = g.uniform(1.0, 50_000.0, size=(V, R))
        if trial == 3:
            ly[0, 0] = -math.inf
        o = CO.consensus(ly, rse, n, al, es)
        c = _lib_consensus(ly, rse, n, al, es)
        for k in ("log_p_con", "log_e_con"):
            assert c[k] == pytest.approx(o[k], rel=1e-13, abs=1e-9), k
        for k in ("rel_half_width", "variant_ratio", "min_ess", "d_max"):
            assert c[k] == pytest.approx(o[k], rel=1e-10), k
        assert c["c_bonf"] == pytest.approx(o["c_bonf"], abs=1e-10)
        assert c["t_crit"] == pytest.approx(o["t_crit"], abs=1e-9)
        assert c["checks"] == o["checks"] and c["provisional"] == o["provisional"]
        assert np.allclose(c["log_ybar"], o["log_ybar"], rtol=1e-13, atol=1e-9)
        assert np.allclose(c["rel_e"], o["rel_e"], rtol=1e-10)


def test_library_quantiles_over_many_sizes():
    # t_{0.975, R-1} for R = 2..60 and c_Bonf for V = 2..12 against the oracle's
    for R in range(2, 61):
        ly, rse, n, al, es = _runs(np.full((2, R), 3.0), 0.1)
        assert _lib_consensus(ly, rse, n, al, es)["t_crit"] == pytest.approx(CO.t_critical(R - 1), abs=1e-9)
    for V in range(2, 13):
        ly, rse, n, al, es = _runs(np.full((V, 3), 3.0), 0.1)
        for a in (0.01, 0.05, 0.2):
            assert _lib_consensus(ly, rse, n, al, es, a)["c_bonf"] == pytest.approx(
                CO.bonferroni_critical(V, a), abs=1e-10)


def test_library_rejects_bad_arguments():
    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import _native as N
    one = {"log_estimate": 1.0, "rse": 0.1, "n_traj": 10, "n_alive": 10, "ess": 5.0}
    with pytest.raises(N.PermEstError):
        P.consensus([[one, one]])                   # one variant
    with pytest.raises(N.PermEstError):
        P.consensus([[one], [one]])                 # one seed
    with pytest.raises(N.PermEstError):
        P.consensus([[one, one], [one, one]], alpha=1.5)
