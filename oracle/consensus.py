"""Multi-seed consensus diagnostics for a permanent with no known value
(Sec. 4.4, "Real-world matrices with unknown permanents"), stated plainly in
FP64 from the definitions there.

TEST INFRASTRUCTURE ONLY: the product path never imports this module; the
library's own implementation (perm_est_consensus) is checked against it.

Inputs are the final statistics of V variants x R seeds of runs on one
matrix: ln of each estimate Y (the sample mean of X), its RSE
s / (sqrt(M) |Y|), the trajectory count M, the survivors and the ESS.
Estimates of a large matrix overflow FP64, so every Y is divided by
exp(L) with L the largest ln Y first; every quantity below is either
homogeneous of degree one in the Y (reported as a logarithm, L added
back) or of degree zero (reported as is).

Definitions (Sec. 4.4):
  e_{P,r}   = s_{P,r} / sqrt(M_{P,r})                 within-run std. error
  Ybar_P    = mean_r Y_{P,r}
  e_in_P    = sqrt(sum_r e_{P,r}^2) / R
  e_seed_P  = sd_r(Y_{P,r}) / sqrt(R)                 (R - 1 denominator)
  e_P       = max(e_in_P, e_seed_P)
  P_con     = mean_P Ybar_P,   e_con = sqrt(sum_P e_P^2) / V
  rel. half-width = 1.96 e_con / |P_con|
  variant ratio   = max_P Ybar_P / min_P Ybar_P
  D_max     = max_{P < P'} |Ybar_P - Ybar_P'| / sqrt(e_P^2 + e_P'^2)
  c_Bonf    = Phi^{-1}(1 - alpha / (2 * C(V, 2)))      (2.81 for V = 5)
A matrix is a provisional consensus when all V x R runs are present (each
has trajectories and an estimate, possibly zero), the
variant-wise 95 % t-intervals Ybar_P +- t_{0.975, R-1} e_P share a point,
D_max <= c_Bonf, every run has at least 1000 surviving trajectories and an
ESS of at least 1000, and the half-width is at most 10 % of |P_con|.
Reading: the t-interval of a variant uses its combined standard error e_P
with R - 1 degrees of freedom (the paper names the interval, not its
width)."""
from __future__ import annotations

import itertools
import math
from typing import Dict, Sequence

import numpy as np
from scipy import stats as S

MIN_ALIVE = 1000
MIN_ESS = 1000.0
MAX_REL_HW = 0.10
Z95 = 1.96


def bonferroni_critical(n_variants: int, alpha: float = 0.05) -> float:
    """Two-sided Bonferroni critical value over the C(V, 2) pairs."""
    pairs = n_variants * (n_variants - 1) // 2
    return float(S.norm.ppf(1.0 - alpha / (2.0 * pairs)))


def t_critical(df: int, level: float = 0.95) -> float:
    return float(S.t.ppf(0.5 + level / 2.0, df))


def consensus(log_y: Sequence[Sequence[float]], rse: Sequence[Sequence[float]],
              n_traj: Sequence[Sequence[int]], n_alive: Sequence[Sequence[int]],
              ess: Sequence[Sequence[float]], alpha: float = 0.05) -> Dict[str, object]:
    """The diagnostics for runs indexed [variant][seed]."""
    ly = np.asarray(log_y, dtype=np.float64)
    V, R = ly.shape
    rs = np.asarray(rse, dtype=np.float64)
    M = np.asarray(n_traj, dtype=np.float64)
    al = np.asarray(n_alive, dtype=np.float64)
    es = np.asarray(ess, dtype=np.float64)
    present = bool(np.all(M > 0) and not np.any(np.isnan(ly)))
    L = float(np.max(ly[np.isfinite(ly)])) if np.any(np.isfinite(ly)) else 0.0
    Y = np.where(np.isfinite(ly), np.exp(ly - L), 0.0)
    # e = s / sqrt(M) = RSE |Y|; a run with no survivor has s = 0
    e = np.where(Y > 0, rs * Y, 0.0)
    ybar = Y.mean(axis=1)
    e_in = np.sqrt((e ** 2).sum(axis=1)) / R
    e_seed = Y.std(axis=1, ddof=1) / math.sqrt(R) if R > 1 else np.zeros(V)
    eP = np.maximum(e_in, e_seed)
    p_con = ybar.mean()
    e_con = math.sqrt(float((eP ** 2).sum())) / V
    d_max = 0.0
    for a, b in itertools.combinations(range(V), 2):
        den = math.sqrt(eP[a] ** 2 + eP[b] ** 2)
        d = abs(ybar[a] - ybar[b]) / den if den > 0 else (0.0 if ybar[a] == ybar[b] else math.inf)
        d_max = max(d_max, d)
    c_bonf = bonferroni_critical(V, alpha) if V > 1 else math.inf
    tc = t_critical(R - 1) if R > 1 else math.inf
    lo, hi = ybar - tc * eP, ybar + tc * eP
    intersect = bool(lo.max() <= hi.min())
    rel_hw = Z95 * e_con / abs(p_con) if p_con != 0 else math.inf
    checks = {
        "all_runs_present": present,
        "t_intervals_intersect": intersect,
        "d_max_within_bonferroni": bool(d_max <= c_bonf),
        "alive_at_least_1000": bool(np.all(al >= MIN_ALIVE)),
        "ess_at_least_1000": bool(np.all(es >= MIN_ESS)),
        "half_width_within_10pct": bool(rel_hw <= MAX_REL_HW),
    }
    return {
        "log_p_con": L + math.log(p_con) if p_con > 0 else -math.inf,
        "log_e_con": L + math.log(e_con) if e_con > 0 else -math.inf,
        "rel_half_width": rel_hw,
        "variant_ratio": float(ybar.max() / ybar.min()) if ybar.min() > 0 else math.inf,
        "min_ess": float(es.min()),
        "d_max": d_max,
        "c_bonf": c_bonf,
        "t_crit": tc,
        "log_ybar": [L + math.log(x) if x > 0 else -math.inf for x in ybar],
        "rel_e": [float(eP[i] / ybar[i]) if ybar[i] > 0 else math.inf for i in range(V)],
        "checks": checks,
        "provisional": all(checks.values()),
    }
