"""Pins of the oracle's subset expansion of the permanent (the references of
the hidden-block study) and of the stored block-set references."""
from __future__ import annotations

import hashlib
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_15390_amd import inputs as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "blocks50.json")


def _brute(D):
    n = D.shape[0]
    return sum(math.prod(D[i, p[i]] for i in range(n)) for p in itertools.permutations(range(n)))


@pytest.mark.parametrize("n", range(1, 9))
def test_subset_expansion_matches_brute_force(n):
    g = np.random.default_rng(n)
    for _ in range(3):
        D = g.uniform(0.5, 2.0, size=(n, n)) * (g.random((n, n)) < 0.6)
        assert O.perm_subset_dp(D) == pytest.approx(_brute(D), rel=1e-13, abs=1e-300)


def test_subset_expansion_matches_exact_ryser_on_01():
    g = np.random.default_rng(5)
    for n in (10, 14, 18, 20):
        A = (g.random((n, n)) < 0.4) | np.eye(n, dtype=bool)
        assert O.perm_subset_dp(A.astype(np.float64)) == pytest.approx(float(O.ryser(A)), rel=1e-14)


def test_subset_expansion_closed_forms():
    for n in (5, 12, 20, 25):
        assert O.perm_subset_dp(np.ones((n, n))) == pytest.approx(math.factorial(n), rel=1e-14)
    for n in (6, 11, 16):
        d = round(math.factorial(n) / math.e)
        assert O.perm_subset_dp(np.ones((n, n)) - np.eye(n)) == pytest.approx(d, rel=1e-14)
    assert O.perm_subset_dp(np.eye(25)) == 1.0


def test_stored_block_references():
    """The stored set still matches the generator, and two of its matrices'
    references are recomputed block by block."""
    with open(GOLDEN) as f:
        ref = {m["name"]: m for m in json.load(f)["matrices"]}
    assert len(ref) == 50
    checked = 0
    for name, M, blocks in G.config_blocks(orders=(100,)):
        r = ref[name]
        h = hashlib.sha256()
        for a in (M.row_ptr, M.col_idx, M.col_ptr, M.row_idx):
            h.update(a.astype("<i4").tobytes())
        assert h.hexdigest() == r["index_sha256"], name
        if name in ("n100_p0.5_b", "n100_p0.7_w"):
            lp = sum(math.log(O.perm_subset_dp(b)) for b in blocks)
            assert lp == pytest.approx(r["log_permanent"], rel=1e-13)
            checked += 1
    assert checked == 2
