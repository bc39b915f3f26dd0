"""Writes band_n1e3_hw4.json, band_n1e4_hw4.json and band_n1e5_hw4.json: the
exact ln per(A) of the band matrices of mean degree 8 at n = 1e3, 1e4, 1e5
(half-width 4, inner band full, outermost diagonals kept with probability
1/2, rows and columns permuted; generator seed 1), computed by the oracle's
dynamic program over the band.  The index arrays' digest is stored with
each, so that a reader can tell that the generator still builds the same
matrix.

Run from the repository root:  python tests/golden/make_band_golden.py
"""
from __future__ import annotations

import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import band as B  # noqa: E402
from paper_2608_15390_amd import inputs as G  # noqa: E402


def digest(M) -> str:
    h = hashlib.sha256()
    for a in (M.row_ptr, M.col_idx, M.col_ptr, M.row_idx):
        h.update(a.astype("<i4").tobytes())
    return h.hexdigest()


SIZES = {"1e3": 1000, "1e4": 10_000, "1e5": 100_000}


def main() -> None:
    for tag, n in SIZES.items():
        M, band = G.config_band(1, n=n)
        out = {
            "matrix": f"inputs.config_band(seed=1, n={n}): band half-width 4, outer diagonals kept with "
                      "probability 1/2, permuted",
            "n": M.n,
            "nnz": M.nnz,
            "index_sha256": digest(M),
            "log_permanent": B.band_log_permanent(band, 4),
            "method": "oracle/band.py band_log_permanent (float64, rescaled per row)",
        }
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"band_n{tag}_hw4.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")
        print(json.dumps(out))


if __name__ == "__main__":
    main()
