"""Helpers shared by the tests: exact trajectory-tree enumeration through the
oracle's probe interface, and dense-matrix utilities that recompute graph
quantities independently of the oracle's own bookkeeping."""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

from oracle import oracle as O


def enumerate_tree(A: "O.OMatrix", sched: "O.Schedule", pre: "O.Prep") -> Tuple[float, float, int]:
    """Exact E[X], P(X > 0) and the number of completed paths, by walking the
    whole trajectory tree: every node asks the oracle for its candidates and
    their sampling probabilities, every leaf contributes P(path) * X(path)."""
    total = 0.0
    p_alive = 0.0
    n_paths = 0
    stack = [([], 0.0)]
    while stack:
        prefix, logp = stack.pop()
        r = O.probe(A, sched, pre, seed=7, k=0, forced=prefix, stop_at=len(prefix))
        if r["stopped"] == 1:
            for u, p in zip(r["cand"].tolist(), r["prob"].tolist()):
                assert p > 0.0
                stack.append((prefix + [u], logp + math.log(p)))
        elif r["stopped"] == -1:
            raise AssertionError("forced vertex was not a candidate")
        elif r["alive"]:
            total += math.exp(logp + r["logw"])
            p_alive += math.exp(logp)
            n_paths += 1
    return total, p_alive, n_paths


def residual_adjacency(M, act: np.ndarray, removed: np.ndarray) -> np.ndarray:
    """Dense 0/1 adjacency of the residual: active rows x active columns,
    edges not removed."""
    n = M.n
    B = np.zeros((n, n), dtype=np.int64)
    rows = np.repeat(np.arange(n), np.diff(M.row_ptr))
    keep = removed[: M.nnz] == 0
    B[rows[keep], M.col_idx[keep]] = 1
    B[act[:n] == 0, :] = 0
    B[:, act[n:] == 0] = 0
    return B


def dense_values(M) -> np.ndarray:
    n = M.n
    D = np.zeros((n, n), dtype=np.float64)
    rows = np.repeat(np.arange(n), np.diff(M.row_ptr))
    D[rows, M.col_idx] = 1.0 if M.val is None else M.val.astype(np.float64)
    return D


def stats_by_hand(M, o, u, v):
    """S_u and the degree-<=2 count from the oracle's state snapshot, written
    out independently of the oracle."""
    n = M.n
    act, deg, removed = o["act"].astype(bool), o["deg"], o["removed"].astype(bool)
    if u < n:
        lo, hi = M.row_ptr[u], M.row_ptr[u + 1]
        nb, edges = M.col_idx[lo:hi] + n, np.arange(lo, hi)
    else:
        lo, hi = M.col_ptr[u - n], M.col_ptr[u - n + 1]
        nb = M.row_idx[lo:hi]
        edges = np.array([M.row_ptr[i] + np.searchsorted(M.col_idx[M.row_ptr[i]:M.row_ptr[i + 1]], u - n)
                          for i in nb], dtype=np.int64)
    S, c2 = 0, 0
    for w, e in zip(nb, edges):
        if act[w] and not removed[e]:
            S += (1 << 20) // int(deg[w])
            c2 += int(w != v and deg[w] <= 2)
    return S, c2
