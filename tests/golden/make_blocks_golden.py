"""Writes blocks50.json: the exact ln per(A) of the 50 matrices of the
hidden-block study set (inputs.config_blocks: orders 100..2000, deletion
probabilities 0.1..0.9, binary and weighted, blocks of order 20 or 25),
each the sum of ln per(block) with every block permanent computed by the
oracle's subset expansion (FP64, no cancellation).  The index digest (and
for weighted matrices the value digest) is stored with each, so a reader
can tell that the generator still builds the same matrix.

Run from the repository root:  python tests/golden/make_blocks_golden.py
(about two minutes on 8 cores).
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2608_15390_amd import inputs as G  # noqa: E402


def digest(M) -> str:
    h = hashlib.sha256()
    for a in (M.row_ptr, M.col_idx, M.col_ptr, M.row_idx):
        h.update(a.astype("<i4").tobytes())
    return h.hexdigest()


def value_digest(M) -> str:
    return hashlib.sha256(M.val.astype("<f4").tobytes()).hexdigest() if M.val is not None else ""


def _log_per(block):
    return math.log(O.perm_subset_dp(block))


def main() -> None:
    sets = list(G.config_blocks())
    jobs = [(i, b) for i, (_, _, blocks) in enumerate(sets) for b in blocks]
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        logs = pool.map(_log_per, [b for _, b in jobs], chunksize=4)
    per = [0.0] * len(sets)
    for (i, _), lp in zip(jobs, logs):
        per[i] += lp
    out = {"set": "inputs.config_blocks(): hidden block-diagonal, blocks of order 20/25, permuted",
           "method": "oracle perm_subset_dp per block (float64), ln summed over blocks",
           "matrices": []}
    for (name, M, blocks), lp in zip(sets, per):
        out["matrices"].append({"name": name, "n": M.n, "nnz": M.nnz, "p": M.meta["p"],
                                "weighted": M.val is not None, "blocks": len(blocks),
                                "index_sha256": digest(M), "value_sha256": value_digest(M),
                                "log_permanent": lp})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "blocks50.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"wrote {path}: {len(sets)} matrices")


if __name__ == "__main__":
    main()
