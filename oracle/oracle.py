"""ctypes front end of the CPU oracle (``perm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the product path never imports this module; only
the tests, the smoke check and the benchmark's CPU-baseline leg do.

The oracle is the plain, sequential statement of the estimator of "The
Quick and the Dead" (Alg. 2 with Eq. (q), Eq. (local) and the DM policies
of Sec. 3.3), plus Ryser's exact permanent (Sec. 2) used to pin it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "perm_oracle.c")
_LIB = os.path.join(_HERE, "libperm_oracle.so")

GCC_FLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU code involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


class _Mat(C.Structure):
    _fields_ = [
        ("n", C.c_int32),
        ("m", C.c_int64),
        ("row_ptr", C.c_void_p),
        ("col_idx", C.c_void_p),
        ("col_ptr", C.c_void_p),
        ("row_idx", C.c_void_p),
        ("val", C.c_void_p),
        ("csc2csr", C.c_void_p),
    ]


class _Sched(C.Structure):
    _fields_ = [
        ("vertex_rule", C.c_int32),
        ("sk_policy", C.c_int32),
        ("dm_policy", C.c_int32),
        ("initial_dm", C.c_int32),
        ("K0", C.c_int32),
        ("K", C.c_int32),
        ("theta_th", C.c_double),
        ("theta_tr", C.c_double),
        ("precision", C.c_int32),
        ("local_gate", C.c_int32),
        ("model", C.c_void_p),
        ("mix_alpha", C.c_double),
        ("local_cap", C.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_rng64.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.or_rng64.restype = C.c_uint64
        L.or_uniform_below.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64]
        L.or_uniform_below.restype = C.c_uint64
        L.or_splitmix_fold.argtypes = [C.c_uint64, C.c_uint64]
        L.or_splitmix_fold.restype = C.c_uint64
        L.or_ryser_u01.argtypes = [C.c_int32, P, P]
        L.or_ryser_f64.argtypes = [C.c_int32, P]
        L.or_ryser_f64.restype = C.c_double
        L.or_perm_subset_dp.argtypes = [C.c_int32, P]
        L.or_perm_subset_dp.restype = C.c_double
        L.or_mat_init.argtypes = [P, P]
        L.or_mat_init.restype = C.c_int
        L.or_support_filter.argtypes = [P, P, P]
        L.or_support_filter.restype = C.c_int
        L.or_prep.argtypes = [P, C.c_int32, C.c_int32, C.c_int32, P, P, P]
        L.or_prep.restype = C.c_int
        L.or_run.argtypes = [P, P, P, P, P, C.c_int32, C.c_uint64, C.c_uint32, C.c_int64, C.c_int64,
                             C.c_int32, P, P, P, P, P]
        L.or_run.restype = C.c_int
        L.or_probe.argtypes = [P, P, P, P, P, C.c_int32, C.c_uint64, C.c_uint32, C.c_uint32,
                               P, P, C.c_int32, C.c_int32, P, P, P, P, P, P, P, P, P, P, P, P]
        L.or_probe.restype = C.c_int
        L.or_stats.argtypes = [P, P, C.c_int64, P]
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


# ---------------------------------------------------------------- schedules
VR_MD, VR_ROW = 0, 1
SK_NONE, SK_FIXED, SK_ADAPTIVE, SK_LOCAL, SK_LEARNED = 0, 1, 2, 3, 4
MLP_IN, MLP_H = 8, 64
MLP_NPARAM = MLP_IN * MLP_H + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1
DM_NONE, DM_ALL, DM_THRS, DM_TRCK = 0, 1, 2, 3
CONTRACT, PAPER = 0, 1


@dataclass
class Schedule:
    vertex_rule: int = VR_MD
    sk_policy: int = SK_NONE
    dm_policy: int = DM_NONE
    initial_dm: int = 0
    K0: int = 0
    K: int = 10
    theta_th: float = 0.33
    theta_tr: float = 0.33
    precision: int = CONTRACT
    model: Optional[np.ndarray] = None   # quantised MLP parameters (float64, MLP_NPARAM)
    mix_alpha: float = 0.05
    local_gate: int = 0                  # learned only: gated local-repair fallback
    local_cap: int = 0                   # local repair: 0 = exact, B > 0 = lists longer than B sampled

    def c(self) -> _Sched:
        if self.sk_policy == SK_LEARNED:
            if self.model is None or self.model.size != MLP_NPARAM:
                raise ValueError("the learned proposal needs a model of MLP_NPARAM parameters")
            self._model_buf = np.ascontiguousarray(self.model, dtype=np.float64)
            mp = self._model_buf.ctypes.data
        else:
            mp = None
        return _Sched(self.vertex_rule, self.sk_policy, self.dm_policy, self.initial_dm, self.K0,
                      self.K, self.theta_th, self.theta_tr, self.precision, self.local_gate, mp,
                      self.mix_alpha, self.local_cap)

    def replace(self, **kw) -> "Schedule":
        d = {k: v for k, v in self.__dict__.items() if not k.startswith("_")}
        d.update(kw)
        return Schedule(**d)


def preset(name: str) -> Schedule:
    """The paper's five variants (Sec. 4: two-sided MD, K0 = 100, K = 10,
    shared initial DM, theta = 0.33) plus the unscaled estimators."""
    both = dict(vertex_rule=VR_MD, initial_dm=1, K0=100, K=10, theta_th=0.33, theta_tr=0.33)
    table: Dict[str, Schedule] = {
        "plain": Schedule(vertex_rule=VR_MD),
        "rasmussen": Schedule(vertex_rule=VR_ROW),
        "fixed_all": Schedule(sk_policy=SK_FIXED, dm_policy=DM_ALL, **both),
        "adaptive_threshold": Schedule(sk_policy=SK_ADAPTIVE, dm_policy=DM_THRS, **both),
        "local_threshold": Schedule(sk_policy=SK_LOCAL, dm_policy=DM_THRS, **both),
        "adaptive_tracked": Schedule(sk_policy=SK_ADAPTIVE, dm_policy=DM_TRCK, **both),
        "local_tracked": Schedule(sk_policy=SK_LOCAL, dm_policy=DM_TRCK, **both),
        # local repair every step, no inner filtering (large-n workload)
        "local_nodm": Schedule(sk_policy=SK_LOCAL, dm_policy=DM_NONE, **both),
        # learned proposal (the network goes in Schedule.model)
        "learned": Schedule(sk_policy=SK_LEARNED, dm_policy=DM_NONE, **both),
        "learned_threshold": Schedule(sk_policy=SK_LEARNED, dm_policy=DM_THRS, **both),
        # the same with the gated local-repair fallback
        "learned_gated": Schedule(sk_policy=SK_LEARNED, dm_policy=DM_NONE, local_gate=1, **both),
        "learned_threshold_gated": Schedule(sk_policy=SK_LEARNED, dm_policy=DM_THRS, local_gate=1, **both),
    }
    if name not in table:
        raise KeyError(name)
    return table[name]


# ------------------------------------------------------------------ matrix
class OMatrix:
    """A SparseMatrix bound to the oracle (keeps the numpy buffers alive)."""

    def __init__(self, M):
        self.M = M
        self.n = int(M.n)
        self.m = int(M.nnz)
        self.row_ptr = np.ascontiguousarray(M.row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(M.col_idx, dtype=np.int32)
        self.col_ptr = np.ascontiguousarray(M.col_ptr, dtype=np.int32)
        self.row_idx = np.ascontiguousarray(M.row_idx, dtype=np.int32)
        self.val = None if M.val is None else np.ascontiguousarray(M.val, dtype=np.float32)
        self.csc2csr = np.zeros(max(self.m, 1), dtype=np.int32)
        self.s = _Mat(self.n, self.m, _p(self.row_ptr), _p(self.col_idx), _p(self.col_ptr),
                      _p(self.row_idx), _p(self.val), None)
        rc = lib().or_mat_init(C.byref(self.s), _p(self.csc2csr))
        if rc != 0:
            raise ValueError("CSR and CSC disagree")

    @property
    def ref(self):
        return C.byref(self.s)


@dataclass
class Prep:
    removed: np.ndarray
    r: np.ndarray
    c: np.ndarray
    ok: int


def prep(A: OMatrix, sched: Schedule) -> Prep:
    removed = np.zeros(max(A.m, 1), dtype=np.uint8)
    r = np.ones(A.n, dtype=np.float64)
    c = np.ones(A.n, dtype=np.float64)
    ok = lib().or_prep(A.ref, sched.initial_dm, sched.K0, sched.precision, _p(removed), _p(r), _p(c))
    if ok < 0:
        raise MemoryError("oracle prep failed")
    return Prep(removed, r, c, ok)


def support_filter(A: OMatrix, act: Optional[np.ndarray] = None, removed: Optional[np.ndarray] = None):
    """Returns (ok, removed) where removed marks CSR edges in no perfect matching."""
    rem = np.zeros(max(A.m, 1), dtype=np.uint8) if removed is None else removed.astype(np.uint8).copy()
    a = None if act is None else np.ascontiguousarray(act, dtype=np.uint8)
    ok = lib().or_support_filter(A.ref, _p(a), _p(rem))
    if ok < 0:
        raise MemoryError
    return ok, rem


def run(A: OMatrix, sched: Schedule, seed: int, first: int = 0, count: int = 1, b: int = 0,
        nthreads: int = 1, want_path: bool = False, pre: Optional[Prep] = None) -> Dict[str, np.ndarray]:
    pre = pre or prep(A, sched)
    s = sched.c()
    logw = np.zeros(count, dtype=np.float64)
    alive = np.zeros(count, dtype=np.uint8)
    ph = np.zeros(count, dtype=np.uint64)
    cnt = np.zeros((count, 4), dtype=np.int32)
    path = np.zeros((count, 2 * A.n), dtype=np.int32) if want_path else None
    rc = lib().or_run(A.ref, C.byref(s), _p(pre.removed), _p(pre.r), _p(pre.c), pre.ok,
                      C.c_uint64(seed), b, first, count, nthreads,
                      _p(logw), _p(alive), _p(path), _p(ph), _p(cnt))
    if rc != 0:
        raise MemoryError("oracle run failed")
    out = {"logw": logw, "alive": alive, "path_hash": ph, "counters": cnt}
    if want_path:
        out["path"] = path
    return out


def probe(A: OMatrix, sched: Schedule, pre: Prep, seed: int, k: int, forced, stop_at: int,
          forced_events=None, b: int = 0):
    """One trajectory with forced candidate choices; see or_probe."""
    s = sched.c()
    fc = np.ascontiguousarray(np.asarray(forced, dtype=np.int32)) if len(forced) else np.zeros(1, np.int32)
    fe = None if forced_events is None else np.ascontiguousarray(np.asarray(forced_events, dtype=np.int32))
    ncand = np.zeros(1, dtype=np.int32)
    cand = np.zeros(A.n, dtype=np.int32)
    prob = np.zeros(A.n, dtype=np.float64)
    path = np.zeros(2 * A.n, dtype=np.int32)
    events = np.zeros(2 * A.n, dtype=np.int32)
    counters = np.zeros(4, dtype=np.int32)
    res = np.zeros(4, dtype=np.float64)
    act = np.zeros(2 * A.n, dtype=np.uint8)
    removed = np.zeros(max(A.m, 1), dtype=np.uint8)
    r = np.zeros(A.n, dtype=np.float64)
    c = np.zeros(A.n, dtype=np.float64)
    deg = np.zeros(2 * A.n, dtype=np.int32)
    rc = lib().or_probe(A.ref, C.byref(s), _p(pre.removed), _p(pre.r), _p(pre.c), pre.ok,
                        C.c_uint64(seed), b, k, _p(fc), _p(fe), len(forced), stop_at,
                        _p(ncand), _p(cand), _p(prob), _p(path), _p(events), _p(counters), _p(res),
                        _p(act), _p(removed), _p(r), _p(c), _p(deg))
    if rc != 0:
        raise MemoryError
    return {
        "logw": res[0], "alive": int(res[1]), "stopped": int(res[2]), "steps": int(res[3]),
        "cand": cand[: ncand[0]].copy(), "prob": prob[: ncand[0]].copy(),
        "path": path, "events": events, "counters": counters,
        "act": act, "removed": removed[: A.m], "r": r, "c": c, "deg": deg,
    }


def stats(logw: np.ndarray, alive: np.ndarray) -> Dict[str, float]:
    out = np.zeros(8, dtype=np.float64)
    lw = np.ascontiguousarray(logw, dtype=np.float64)
    al = np.ascontiguousarray(alive, dtype=np.uint8)
    lib().or_stats(_p(lw), _p(al), lw.size, _p(out))
    keys = ["log_estimate", "p_match", "rel_spread", "rse", "ess", "var_logw", "max_logw", "n_alive"]
    return dict(zip(keys, out.tolist()))


# ------------------------------------------------------------ primitives
def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def rng64(seed: int, k: int, b: int, t: int, d: int) -> int:
    return int(lib().or_rng64(C.c_uint64(seed), k, b, t, d))


def uniform_below(seed: int, k: int, b: int, t: int, d0: int, W: int) -> int:
    return int(lib().or_uniform_below(C.c_uint64(seed), k, b, t, d0, C.c_uint64(W)))


def splitmix_fold(h: int, x: int) -> int:
    return int(lib().or_splitmix_fold(C.c_uint64(h), C.c_uint64(x)))


def ryser(dense) -> int:
    """Exact permanent of a 0/1 matrix (n <= 20) by Ryser's formula."""
    A = np.ascontiguousarray(np.asarray(dense) != 0, dtype=np.uint8)
    n = A.shape[0]
    if n == 0:
        return 1
    if n > 24:
        raise ValueError("n too large for exact Ryser")
    out = np.zeros(2, dtype=np.uint64)
    lib().or_ryser_u01(n, _p(A), _p(out))
    v = int(out[0]) | (int(out[1]) << 64)
    if v >= 1 << 127:
        v -= 1 << 128
    return v


def ryser_f64(dense) -> float:
    A = np.ascontiguousarray(dense, dtype=np.float64)
    n = A.shape[0]
    if n == 0:
        return 1.0
    return float(lib().or_ryser_f64(n, _p(A)))


def perm_subset_dp(dense) -> float:
    """Permanent of a dense nonnegative matrix (n <= 26) by the subset
    expansion (no cancellation; FP64)."""
    A = np.ascontiguousarray(dense, dtype=np.float64)
    n = A.shape[0]
    if n > 26:
        raise ValueError("n too large for the subset expansion")
    if (A < 0).any():
        raise ValueError("the subset expansion is for nonnegative matrices")
    v = float(lib().or_perm_subset_dp(n, _p(A)))
    if v < 0:
        raise MemoryError("workspace of 2^n doubles")
    return v


def plog2(s: float) -> float:
    lib().or_plog2.argtypes = [C.c_double]
    lib().or_plog2.restype = C.c_double
    return float(lib().or_plog2(s))


def learned_logit(model: np.ndarray, x) -> int:
    L = lib()
    L.or_learned_logit.argtypes = [C.c_void_p, C.c_void_p]
    L.or_learned_logit.restype = C.c_int32
    m = np.ascontiguousarray(model, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    return int(L.or_learned_logit(m.ctypes.data, xx.ctypes.data))


def learned_features(deg_rho, deg_gam, r0_rho, c0_gam, t, n, v_is_row, s_u, c2_u) -> np.ndarray:
    """Features of a candidate edge; s_u = sum of floor(2^20 / deg w) over
    the candidate's residual neighbours w, c2_u = how many of them other
    than v have degree <= 2."""
    L = lib()
    L.or_learned_features.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                      C.c_int32, C.c_int32, C.c_int64, C.c_int32, C.c_void_p]
    x = np.zeros(MLP_IN, dtype=np.float64)
    L.or_learned_features(deg_rho, deg_gam, r0_rho, c0_gam, t, n, v_is_row, s_u, c2_u, x.ctypes.data)
    return x


def learned_weights(logits, alpha: float) -> np.ndarray:
    L = lib()
    L.or_learned_weights.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_void_p]
    lg = np.ascontiguousarray(logits, dtype=np.int32)
    w = np.zeros(lg.size, dtype=np.uint64)
    L.or_learned_weights(lg.ctypes.data, lg.size, alpha, w.ctypes.data)
    return w
