"""Seeded synthetic sparse 0/1 (and weighted) square matrices.

This module only *builds inputs*: sparsity patterns, planted permutations,
random entry values and the CSR/CSC index arrays.  It contains none of the
estimator's arithmetic (no scaling, no sampling, no permanent), so both the
HIP path and the CPU oracle's tests draw their inputs from here.

Families (matrix order n, rows and columns both indexed 0..n-1):

* ``identity``, ``permutation``, ``all_ones`` (J_n), ``derangement`` (J_n - I),
  ``upper_triangular`` (full upper triangle incl. diagonal): closed-form
  permanents.
* ``grid``: bipartite adjacency of an a x b grid graph (black cells are rows,
  white cells are columns); its permanent counts domino tilings
  (Kasteleyn / Temperley-Fisher product formula, Sec. 4 "Matrices used").
* ``planted_bernoulli``: identity or random planted permutation plus
  independent Bernoulli(p) off-planted entries (the small-n workloads).
* ``planted_uniform``: planted permutation plus exactly ``extra`` distinct
  off-planted positions chosen uniformly (the paper's Uniform(n,k)
  construction of Sec. 3.1, with a random permutation in place of the
  diagonal) -- the large-n workload, n = 1e5 with 7 extra entries per row.
* ``power_law``: row degrees with P(d) ~ d^-2.5 on [2, 200], distinct uniform
  columns, plus a planted permutation (the stress workload).
* ``hidden_block_diagonal``: randomly permuted block-diagonal matrix with full
  blocks of order 20 or 25 whose off-diagonal entries are deleted with
  probability p while the diagonal is kept (Sec. 4, "Matrices used"); the
  blocks are returned so a test can multiply exact block permanents.
* ``banded``: entries within a band |i - j| <= w (diagonal always, the rest
  -- or only the outermost diagonals -- kept with a given probability), rows
  and columns then randomly permuted;
  the unpermuted band is returned so that a test or a stored reference can
  compute the exact permanent by dynamic programming over the band, at any n.

Everything is deterministic in the seed (numpy PCG64).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "SparseMatrix", "from_coo", "from_dense", "to_dense",
    "identity", "permutation", "all_ones", "derangement", "upper_triangular",
    "grid", "planted_bernoulli", "planted_uniform", "power_law",
    "hidden_block_diagonal", "banded", "uniform_nk", "bernoulli_nk", "with_weights",
    "config_small", "config_batch", "config_large", "config_train", "config_band",
    "config_stress",
]


@dataclass
class SparseMatrix:
    """Square sparse matrix in both CSR and CSC form (int32 indices).

    Lists are sorted ascending and duplicate free.  ``val`` holds float32
    entry values in CSR order, or ``None`` for a 0/1 matrix.
    """

    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    col_ptr: np.ndarray
    row_idx: np.ndarray
    val: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def csc_val(self) -> Optional[np.ndarray]:
        """Entry values in CSC order (None for 0/1 matrices)."""
        if self.val is None:
            return None
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        key_csr = rows * self.n + self.col_idx
        cols = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.col_ptr))
        key_csc = self.row_idx.astype(np.int64) * self.n + cols
        pos = np.searchsorted(key_csr, key_csc)
        return self.val[pos]


def from_coo(n: int, rows, cols, vals=None, meta: Optional[dict] = None) -> SparseMatrix:
    """Build sorted, de-duplicated CSR + CSC arrays from coordinates."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= n or cols.min() < 0 or cols.max() >= n):
        raise ValueError("coordinate out of range")
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    keep = np.ones(key.size, dtype=bool)
    keep[1:] = key[1:] != key[:-1]
    key = key[keep]
    v = None
    if vals is not None:
        v = np.asarray(vals, dtype=np.float32)[order][keep]
    r = key // n
    c = key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    # CSC: sort by (col, row)
    key_t = c * n + r
    order_t = np.argsort(key_t, kind="stable")
    col_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(col_ptr, c + 1, 1)
    col_ptr = np.cumsum(col_ptr)
    return SparseMatrix(
        n=n,
        row_ptr=row_ptr.astype(np.int32),
        col_idx=c.astype(np.int32),
        col_ptr=col_ptr.astype(np.int32),
        row_idx=r[order_t].astype(np.int32),
        val=v,
        meta=dict(meta or {}),
    )


def from_dense(A, weighted: bool = False, meta: Optional[dict] = None) -> SparseMatrix:
    A = np.asarray(A)
    n = A.shape[0]
    assert A.shape == (n, n)
    r, c = np.nonzero(A)
    vals = A[r, c].astype(np.float32) if weighted else None
    return from_coo(n, r, c, vals, meta)


def to_dense(M: SparseMatrix, dtype=np.float64) -> np.ndarray:
    A = np.zeros((M.n, M.n), dtype=dtype)
    rows = np.repeat(np.arange(M.n), np.diff(M.row_ptr))
    A[rows, M.col_idx] = 1.0 if M.val is None else M.val
    return A


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed) & 0xFFFFFFFF, int(seed) >> 32, stream])


# ---------------------------------------------------------------- closed forms
def identity(n: int) -> SparseMatrix:
    i = np.arange(n)
    return from_coo(n, i, i, meta={"family": "identity"})


def permutation(n: int, seed: int = 0) -> SparseMatrix:
    p = _rng(seed, 1).permutation(n)
    return from_coo(n, np.arange(n), p, meta={"family": "permutation"})


def all_ones(n: int) -> SparseMatrix:
    r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return from_coo(n, r.ravel(), c.ravel(), meta={"family": "J"})


def derangement(n: int) -> SparseMatrix:
    r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    m = r != c
    return from_coo(n, r[m], c[m], meta={"family": "J-I"})


def upper_triangular(n: int) -> SparseMatrix:
    r, c = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    m = c >= r
    return from_coo(n, r[m], c[m], meta={"family": "triu"})


def grid(a: int, b: int) -> SparseMatrix:
    """Bipartite adjacency matrix of the a x b grid graph (a*b even)."""
    if (a * b) % 2:
        raise ValueError("grid needs an even number of cells")
    black = {}
    white = {}
    for i in range(a):
        for j in range(b):
            d = black if (i + j) % 2 == 0 else white
            d[(i, j)] = len(d)
    rows, cols = [], []
    for (i, j), ri in black.items():
        for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            w = white.get((i + di, j + dj))
            if w is not None:
                rows.append(ri)
                cols.append(w)
    return from_coo(len(black), rows, cols, meta={"family": "grid", "a": a, "b": b})


# ---------------------------------------------------------- random families
def planted_bernoulli(n: int, p: float, seed: int, planted: str = "identity") -> SparseMatrix:
    """Planted perfect matching plus i.i.d. Bernoulli(p) off-planted entries."""
    g = _rng(seed, 2)
    pi = np.arange(n) if planted == "identity" else g.permutation(n)
    mask = g.random((n, n)) < p
    mask[np.arange(n), pi] = True
    r, c = np.nonzero(mask)
    return from_coo(n, r, c, meta={"family": "planted_bernoulli", "p": p, "seed": seed})


def planted_uniform(n: int, extra: int, seed: int) -> SparseMatrix:
    """Random planted permutation plus exactly ``extra`` distinct uniform
    off-planted positions."""
    g = _rng(seed, 3)
    pi = g.permutation(n).astype(np.int64)
    planted = np.arange(n, dtype=np.int64) * n + pi
    total = n * n - n
    if extra > total:
        raise ValueError("too many extra entries")
    chosen = np.empty(0, dtype=np.int64)
    planted_sorted = np.sort(planted)
    while chosen.size < extra:
        need = extra - chosen.size
        cand = g.integers(0, n * n, size=int(need * 1.1) + 16, dtype=np.int64)
        pos = np.searchsorted(planted_sorted, cand)
        pos[pos >= n] = n - 1
        cand = cand[planted_sorted[pos] != cand]
        cand = np.unique(cand)
        cand = cand[~np.isin(cand, chosen, assume_unique=True)]
        cand = g.permutation(cand)[:need]
        chosen = np.concatenate([chosen, cand])
    keys = np.concatenate([planted, chosen])
    return from_coo(n, keys // n, keys % n,
                    meta={"family": "planted_uniform", "extra": extra, "seed": seed})


def power_law(n: int, seed: int, exponent: float = 2.5, dmin: int = 2, dmax: int = 200) -> SparseMatrix:
    """Row degrees with P(d) ~ d^-exponent on [dmin, dmax], distinct uniform
    columns per row, plus a planted random permutation."""
    g = _rng(seed, 4)
    pi = g.permutation(n).astype(np.int64)
    d = np.arange(dmin, min(dmax, n) + 1)
    pd = d.astype(np.float64) ** (-exponent)
    pd /= pd.sum()
    deg = g.choice(d, size=n, p=pd)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    cols = np.empty(rows.size, dtype=np.int64)
    off = 0
    # distinct columns per row: sample with a per-row rejection of duplicates
    for i in range(n):
        k = int(deg[i])
        s = set()
        while len(s) < k:
            s.update(int(x) for x in g.integers(0, n, size=k - len(s)))
        cols[off:off + k] = sorted(s)[:k]
        off += k
    rows = np.concatenate([rows, np.arange(n, dtype=np.int64)])
    cols = np.concatenate([cols, pi])
    return from_coo(n, rows, cols, meta={"family": "power_law", "seed": seed})


def uniform_nk(n: int, k: int, seed: int) -> SparseMatrix:
    """Uniform(n,k) of Sec. 3.1 before filtering: k*n distinct uniform
    positions plus the full diagonal."""
    g = _rng(seed, 5)
    pos = g.choice(n * n, size=k * n, replace=False)
    r = np.concatenate([pos // n, np.arange(n)])
    c = np.concatenate([pos % n, np.arange(n)])
    return from_coo(n, r, c, meta={"family": "uniform_nk", "k": k})


def bernoulli_nk(n: int, k: int, seed: int) -> SparseMatrix:
    """Bernoulli(n,k) of Sec. 3.1: every position with probability k/n, plus
    the diagonal."""
    g = _rng(seed, 6)
    mask = g.random((n, n)) < k / n
    mask[np.arange(n), np.arange(n)] = True
    r, c = np.nonzero(mask)
    return from_coo(n, r, c, meta={"family": "bernoulli_nk", "k": k})


def hidden_block_diagonal(n: int, p: float, seed: int, weighted: bool = False,
                          block_orders: Sequence[int] = (20, 25)):
    """Randomly permuted block-diagonal matrix (Sec. 4, "Matrices used").

    Returns ``(matrix, blocks)`` where ``blocks`` is a list of dense float64
    block matrices (before permutation) whose permanents multiply to the
    permanent of the whole matrix.
    """
    g = _rng(seed, 7)
    lo, hi = min(block_orders), max(block_orders)
    splits = [(a, (n - a * lo) // hi) for a in range(n // lo + 1) if (n - a * lo) % hi == 0]
    if not splits:
        raise ValueError(f"cannot split {n} into blocks of orders {block_orders}")
    a, bcount = splits[int(g.integers(len(splits)))]
    orders: List[int] = [lo] * a + [hi] * bcount
    orders = [int(x) for x in g.permutation(orders)]
    rows, cols, vals, blocks = [], [], [], []
    base = 0
    for b in orders:
        keep = g.random((b, b)) >= p
        keep[np.arange(b), np.arange(b)] = True
        blk = keep.astype(np.float64)
        if weighted:
            w = g.uniform(1.0, 1.5, size=(b, b)).astype(np.float32).astype(np.float64)
            blk = blk * w
        r, c = np.nonzero(keep)
        rows.append(r + base)
        cols.append(c + base)
        vals.append(blk[r, c])
        blocks.append(blk)
        base += b
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    prow = g.permutation(n)
    pcol = g.permutation(n)
    M = from_coo(n, prow[rows], pcol[cols], vals if weighted else None,
                 meta={"family": "hidden_block_diagonal", "p": p, "orders": orders})
    return M, blocks


def banded(n: int, half_width: int, keep: float, seed: int, weighted: bool = False,
           outer_only: bool = False):
    """Band pattern |i - j| <= half_width with the diagonal always present and
    band positions kept with probability ``keep`` (every off-diagonal band
    position, or with ``outer_only`` only those with |i - j| = half_width,
    the rest of the band being full), values uniform in [1, 1.5] as float32
    when ``weighted``; then rows and columns permuted uniformly at random.

    Returns ``(matrix, band)``: ``band`` is the same matrix before the
    permutation (row i holds only columns i - w .. i + w), and both have the
    same permanent.
    """
    g = _rng(seed, 12)
    w = int(half_width)
    off = np.arange(-w, w + 1, dtype=np.int64)
    i = np.repeat(np.arange(n, dtype=np.int64), off.size)
    j = i + np.tile(off, n)
    draw = g.random(i.size)
    vals = g.uniform(1.0, 1.5, size=i.size).astype(np.float32)
    full = np.abs(j - i) < w if outer_only else j == i
    sel = (j >= 0) & (j < n) & (full | (draw < keep))
    i, j, vals = i[sel], j[sel], vals[sel]
    meta = {"family": "banded", "half_width": w, "keep": keep, "outer_only": outer_only, "seed": seed}
    band = from_coo(n, i, j, vals if weighted else None, meta=dict(meta, permuted=False))
    prow = g.permutation(n)
    pcol = g.permutation(n)
    M = from_coo(n, prow[i], pcol[j], vals if weighted else None, meta=meta)
    return M, band


def config_band(seed: int = 1, n: int = 100_000):
    """n = 1e5 band of half-width 4 whose inner band (|i - j| <= 3) is full
    and whose outermost diagonals keep each entry with probability 1/2 (mean
    degree 8), randomly permuted: a matrix of the large workload's size and
    degree whose permanent is known exactly.  (Thinning the whole band
    instead leaves vertices that lose all their neighbours, and at this n
    every trajectory dies.)"""
    return banded(n, 4, 0.5, seed, outer_only=True)


BLOCK_ORDERS = (100, 250, 500, 1000, 2000)
BLOCK_DELETION = (0.1, 0.3, 0.5, 0.7, 0.9)


def block_set_seed(i_order: int, i_p: int, weighted: bool) -> int:
    """Generator seed of one matrix of the hidden-block study set."""
    return 5000 + 100 * i_order + 10 * i_p + (1 if weighted else 0)


def config_blocks(orders: Sequence[int] = BLOCK_ORDERS, deletion: Sequence[float] = BLOCK_DELETION):
    """The hidden-block study set (Sec. 4, "Matrices used"): for every order
    n in {100, 250, 500, 1000, 2000} and deletion probability p in {0.1, 0.3,
    0.5, 0.7, 0.9} one binary and one weighted (entries U[1, 1.5], support
    drawn independently) randomly permuted block-diagonal matrix with
    blocks of order 20 or 25: 50 matrices.  Yields (name, matrix, blocks)."""
    for i, n in enumerate(orders):
        for j, p in enumerate(deletion):
            for w in (False, True):
                M, blocks = hidden_block_diagonal(n, p, block_set_seed(BLOCK_ORDERS.index(n), j, w), weighted=w)
                yield f"n{n}_p{p:g}_{'w' if w else 'b'}", M, blocks


def with_weights(M: SparseMatrix, seed: int, lo: float = 1.0, hi: float = 1.5) -> SparseMatrix:
    """Same pattern with entry values uniform in [lo, hi] (float32)."""
    g = _rng(seed, 8)
    v = g.uniform(lo, hi, size=M.nnz).astype(np.float32)
    return SparseMatrix(M.n, M.row_ptr, M.col_idx, M.col_ptr, M.row_idx, v, dict(M.meta, weighted=True))


# ------------------------------------------------------- network parameters
def network_params(seed: int = 0, scale: float = 1.0) -> np.ndarray:
    """Random initial parameters of the 8-64-64-1 proposal network (float64,
    packed W1[8][64], b1[64], W2[64][64], b2[64], w3[64], b3): He-normal
    weights scaled by `scale`, inputs 6 and 7 (unused features) zero, biases
    0.05 and 0.  A seeded generator like the matrices above, shared by the
    trainer's start and the tests."""
    IN, H = 8, 64
    g = np.random.default_rng(seed)
    W1 = g.normal(0.0, scale * np.sqrt(2.0 / 6), (IN, H))
    W1[6:, :] = 0.0
    W2 = g.normal(0.0, scale * np.sqrt(2.0 / H), (H, H))
    w3 = g.normal(0.0, scale * np.sqrt(1.0 / H), H)
    return np.concatenate([W1.ravel(), np.full(H, 0.05), W2.ravel(), np.full(H, 0.05), w3, np.zeros(1)])


# ------------------------------------------------------------ workloads
def config_small(seed: int = 1) -> SparseMatrix:
    """n = 20: identity plus Bernoulli(0.2) off-diagonal entries."""
    return planted_bernoulli(20, 0.2, seed, planted="identity")


def config_batch(seed: int = 1, count: int = 256, nmin: int = 30, nmax: int = 400,
                 dmin: float = 3.0, dmax: float = 12.0) -> List[SparseMatrix]:
    """Batch of matrices with n ~ U{nmin..nmax}, mean row degree
    ~ U[dmin, dmax], planted random permutation plus Bernoulli entries with
    p = (d - 1) / (n - 1)."""
    g = _rng(seed, 9)
    out = []
    for b in range(count):
        n = int(g.integers(nmin, nmax + 1))
        d = float(g.uniform(dmin, dmax))
        p = (d - 1.0) / (n - 1.0)
        sub = int(g.integers(0, 2**62))
        out.append(planted_bernoulli(n, p, sub, planted="random"))
    return out


def config_large(seed: int = 1, n: int = 100_000, extra_per_row: int = 7) -> SparseMatrix:
    """n = 1e5, planted permutation plus 7n uniform extra entries."""
    return planted_uniform(n, extra_per_row * n, seed)


def config_train(seed: int = 1, count: int = 512, n: int = 1000, extra_per_row: int = 5) -> List[SparseMatrix]:
    g = _rng(seed, 10)
    return [planted_uniform(n, extra_per_row * n, int(g.integers(0, 2**62))) for _ in range(count)]


def config_stress(seed: int = 1, count: int = 64, lo: float = 4.0, hi: float = 6.0) -> List[SparseMatrix]:
    g = _rng(seed, 11)
    out = []
    for _ in range(count):
        n = int(round(10 ** g.uniform(lo, hi)))
        out.append(power_law(n, int(g.integers(0, 2**62))))
    return out
