"""Pins of the exact band permanent (dynamic program over the band window)
and, through it, of the oracle's estimator at sizes Ryser cannot reach.

The dynamic program is checked against brute force, Ryser's formula, the
Fibonacci closed form of the full tridiagonal matrix, and its float64
log-space variant against its integer variant; the estimator's mean is then
checked against it at n = 60 and 200 (Sec. 2: E[X] = per(A))."""
from __future__ import annotations

import hashlib
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import band as B
from oracle import oracle as O
from paper_2608_15390_amd import inputs as G

def _brute(D):
    n = D.shape[0]
    return sum(math.prod(D[i, p[i]] for i in range(n)) for p in itertools.permutations(range(n)))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("w", [1, 2, 3])
def test_band_dp_matches_brute_force(n, w):
    for seed in range(3):
        M, band = G.banded(n, w, 0.6, seed)
        D = G.to_dense(band)
        assert B.band_permanent_exact(band, w) == int(round(_brute(D)))
        Mw, bw = G.banded(n, w, 0.6, seed, weighted=True)
        assert math.exp(B.band_log_permanent(bw, w)) == pytest.approx(_brute(G.to_dense(bw)), rel=1e-12)


@pytest.mark.parametrize("w", [1, 2, 3, 4])
@pytest.mark.parametrize("keep", [0.4, 0.875, 1.0])
def test_band_dp_matches_ryser(w, keep):
    for seed in range(2):
        M, band = G.banded(18, w, keep, 10 + seed)
        per = O.ryser(G.to_dense(band))
        # the permuted matrix has the same permanent (pins the generator)
        assert O.ryser(G.to_dense(M)) == per
        assert B.band_permanent_exact(band) == per
        lp = B.band_log_permanent(band)
        assert lp == (pytest.approx(math.log(per), rel=1e-13) if per else -math.inf)
        Mo, bo = G.banded(18, w, keep, 30 + seed, outer_only=True)
        per = O.ryser(G.to_dense(bo))
        assert O.ryser(G.to_dense(Mo)) == per and B.band_permanent_exact(bo) == per
        Mw, bw = G.banded(16, w, keep, 20 + seed, weighted=True)
        pw = O.ryser_f64(G.to_dense(bw))
        assert B.band_log_permanent(bw) == pytest.approx(math.log(pw), rel=1e-12)


def test_full_tridiagonal_is_fibonacci():
    fib = [1, 1]
    while len(fib) < 90:
        fib.append(fib[-1] + fib[-2])
    for n in (1, 2, 3, 10, 40, 85):
        _, band = G.banded(n, 1, 1.0, 0)
        assert band.nnz == 3 * n - 2
        assert B.band_permanent_exact(band, 1) == fib[n]  # per = F(n+1)
        assert B.band_log_permanent(band, 1) == pytest.approx(math.log(fib[n]), rel=1e-13, abs=1e-13)


def test_float_dp_matches_integer_dp_at_large_n():
    _, band = G.banded(600, 4, 0.875, 3)
    exact = B.band_permanent_exact(band, 4)
    assert exact > 0
    lg = math.log(exact >> (exact.bit_length() - 60)) + (exact.bit_length() - 60) * math.log(2)
    assert B.band_log_permanent(band, 4) == pytest.approx(lg, rel=1e-13)


def test_no_matching_and_out_of_band():
    # row 2 has no entry: no perfect matching
    M = G.from_coo(4, [0, 1, 1, 3], [0, 1, 2, 3])
    assert B.band_permanent_exact(M, 1) == 0
    assert B.band_log_permanent(M, 1) == -math.inf
    # an entry outside the declared band is rejected, not silently dropped
    M = G.from_coo(3, [0, 1, 2, 0], [0, 1, 2, 2])
    with pytest.raises(ValueError):
        B.band_permanent_exact(M, 1)
    with pytest.raises(ValueError):
        B.band_log_permanent(M, 1)


@pytest.mark.parametrize("n,name", [(60, "plain"), (60, "local_threshold"), (200, "local_nodm")])
def test_estimator_mean_within_ci_of_band_permanent(n, name):
    M, band = G.banded(n, 3, 0.8, 7)
    lp = B.band_log_permanent(band, 3)
    out = O.run(O.OMatrix(M), O.preset(name), seed=9, count=20000, nthreads=8)
    st = O.stats(out["logw"], out["alive"])
    assert abs(math.exp(st["log_estimate"] - lp) - 1.0) <= 4.5 * st["rse"], (st, lp)


@pytest.mark.parametrize("tag,n", [("1e3", 1000), ("1e4", 10_000), ("1e5", 100_000)])
def test_stored_band_permanents(tag, n):
    """The stored ln per(A) of the band workloads is what the dynamic
    program gives for the matrices the generator builds today."""
    with open(os.path.join(os.path.dirname(__file__), "golden", f"band_n{tag}_hw4.json")) as f:
        g = json.load(f)
    M, band = G.config_band(1, n=n)
    h = hashlib.sha256()
    for a in (M.row_ptr, M.col_idx, M.col_ptr, M.row_idx):
        h.update(a.astype("<i4").tobytes())
    assert g["n"] == M.n and g["nnz"] == M.nnz and g["index_sha256"] == h.hexdigest()
    assert B.band_log_permanent(band, 4) == g["log_permanent"]
