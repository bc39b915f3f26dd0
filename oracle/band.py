"""Exact permanent of a band matrix by dynamic programming over the band.

Test infrastructure: only the test suite, the smoke check and the stored
reference values under ``tests/golden`` use this module; the HIP library
never does.

The permanent is the sum, over perfect matchings of rows to columns, of the
product of the matched entries (Sec. 2).  When every entry of row i lies in
the columns i - w .. i + w, the rows can be matched in order 0, 1, ..., n-1
while remembering only which columns of the sliding window are taken:

* before row i is matched, columns < i - w are all taken (no later row can
  reach them) and columns >= i + w are all free, so the state is the set of
  taken columns among i - w .. i + w - 1, a 2w-bit mask (bit k is column
  i - w + k; columns left of 0 count as taken);
* row i takes one free column j = i - w + k with a nonzero entry: the mask
  gains bit k (bit 2w is column i + w), column i - w must then be taken, and
  the window slides right by one;
* after the last row the columns n - w .. n - 1 must all be taken: the mask
  is the low w bits.

``band_permanent_exact`` carries Python integers (0/1 matrices, any n);
``band_log_permanent`` carries float64 values rescaled after every row and
returns ln per(A) (weighted or 0/1, any n).  Both take the unpermuted band
matrix; per(A) is unchanged by permuting rows and columns.  Parity is
pinned against Ryser's formula, brute force, the Fibonacci closed form of
the full tridiagonal matrix, and each other.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np


def _rows(M) -> List[List[Tuple[int, float]]]:
    out = []
    for i in range(M.n):
        a, b = int(M.row_ptr[i]), int(M.row_ptr[i + 1])
        cols = M.col_idx[a:b]
        vals = np.ones(b - a) if M.val is None else M.val[a:b].astype(np.float64)
        out.append([(int(j), float(v)) for j, v in zip(cols, vals)])
    return out


def _half_width(M) -> int:
    w = 0
    for i, row in enumerate(_rows(M)):
        for j, _ in row:
            w = max(w, abs(j - i))
    return w


def band_permanent_exact(M, half_width: int = None) -> int:
    """per(A) as an exact integer for a 0/1 band matrix."""
    if M.val is not None:
        raise ValueError("exact integer permanent needs a 0/1 matrix")
    w = _half_width(M) if half_width is None else int(half_width)
    n = M.n
    state: Dict[int, int] = {(1 << w) - 1: 1}
    for i, row in enumerate(_rows(M)):
        nxt: Dict[int, int] = {}
        for mask, cnt in state.items():
            for j, _ in row:
                k = j - i + w
                if k < 0 or k > 2 * w:
                    raise ValueError(f"entry ({i},{j}) outside the band of half-width {w}")
                if mask >> k & 1:
                    continue
                m2 = mask | (1 << k)
                if not m2 & 1:
                    continue
                m2 >>= 1
                nxt[m2] = nxt.get(m2, 0) + cnt
        state = nxt
    return state.get((1 << w) - 1, 0) if n > 0 else 1


def band_log_permanent(M, half_width: int = None) -> float:
    """ln per(A) in float64 for a band matrix (0/1 or weighted); -inf when
    there is no perfect matching."""
    w = _half_width(M) if half_width is None else int(half_width)
    n = M.n
    if n == 0:
        return 0.0
    S = 1 << (2 * w)
    # for each band offset k: the masks that can take column i - w + k, and
    # where the window lands after sliding
    src, dst = [], []
    for k in range(2 * w + 1):
        s = np.array([m for m in range(S) if not (m >> k) & 1 and ((m | (1 << k)) & 1)], dtype=np.int64)
        src.append(s)
        dst.append((s | (1 << k)) >> 1)
    val = np.zeros(S)
    val[(1 << w) - 1] = 1.0
    log_scale = 0.0
    for i, row in enumerate(_rows(M)):
        nxt = np.zeros(S)
        for j, a in row:
            k = j - i + w
            if k < 0 or k > 2 * w:
                raise ValueError(f"entry ({i},{j}) outside the band of half-width {w}")
            nxt[dst[k]] += a * val[src[k]]
        top = nxt.max()
        if top <= 0.0:
            return -math.inf
        val = nxt / top
        log_scale += math.log(top)
    last = val[(1 << w) - 1]
    return log_scale + math.log(last) if last > 0 else -math.inf
