"""MI355X-native estimator of sparse-matrix permanents.

Runs very many independent sequential-importance-sampling trajectories of
the adaptive estimator of "The Quick and the Dead" (Alg. 2: two-sided
minimum-degree selection, scaled proposal with importance correction,
scheduled Sinkhorn-Knopp scaling and support filtering) as hand-written
HIP kernels for gfx950 behind the C ABI of ``include/perm_est.h``.

This module only marshals arguments: torch provides device memory and the
current stream, the library does the work.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional

import numpy as np

from . import _native as N
from .inputs import SparseMatrix

__all__ = ["PermEst", "PermEstBatch", "preset", "Schedule", "PermEstError"]

PermEstError = N.PermEstError
Schedule = N.Schedule

VR_MD, VR_ROW_ORDER = 0, 1
SK_NONE, SK_FIXED, SK_ADAPTIVE, SK_LOCAL = 0, 1, 2, 3
DM_NONE, DM_ALL, DM_THRS, DM_TRCK = 0, 1, 2, 3


def preset(name: str, **overrides) -> N.Schedule:
    """A named schedule from the library (see perm_est_schedule_preset),
    optionally with fields overridden."""
    s = N.Schedule()
    N.check(N.load().perm_est_schedule_preset(name.encode(), C.byref(s)))
    for k, v in overrides.items():
        setattr(s, k, v)
    return s


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


class PermEst:
    """One sparse matrix resident on one GPU."""

    def __init__(self, M: SparseMatrix, device: int = 0, force_hbm: bool = False):
        import torch  # noqa: F401  (initialises the HIP runtime the library shares)

        self._lib = N.load()
        self.n = int(M.n)
        self.m = int(M.nnz)
        self.device = device
        self._h = C.c_void_p()
        rp = np.ascontiguousarray(M.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(M.col_idx, dtype=np.int32)
        cp = np.ascontiguousarray(M.col_ptr, dtype=np.int32)
        ri = np.ascontiguousarray(M.row_idx, dtype=np.int32)
        val = None if M.val is None else np.ascontiguousarray(M.val, dtype=np.float32)
        opts = N.Options(device, 1 if force_hbm else 0)
        N.check(self._lib.perm_est_create(
            self.n, self.m, rp.ctypes.data, ci.ctypes.data, cp.ctypes.data, ri.ctypes.data,
            None if val is None else val.ctypes.data, C.byref(opts), C.byref(self._h)))

    def close(self):
        if self._h:
            self._lib.perm_est_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, first: int, count: int, seed: int, schedule: N.Schedule, *, want_logw=True,
            want_alive=True, want_hash=False, want_path=False, want_counters=False,
            stream=None) -> Dict:
        """Run trajectories first..first+count-1; returns the statistics and
        the requested per-trajectory device tensors."""
        import torch

        dev = torch.device("cuda", self.device)
        out = {}
        logw = torch.empty(count, dtype=torch.float64, device=dev) if want_logw else None
        alive = torch.empty(count, dtype=torch.uint8, device=dev) if want_alive else None
        ph = torch.empty(count, dtype=torch.int64, device=dev) if want_hash else None
        path = torch.empty((count, 2 * self.n), dtype=torch.int32, device=dev) if want_path else None
        cnt = torch.empty((count, 4), dtype=torch.int32, device=dev) if want_counters else None
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        res = N.Result()
        N.check(self._lib.perm_est_run_range(
            self._h, first, count, C.c_uint64(seed), C.byref(schedule), C.byref(res),
            _ptr(logw), _ptr(alive), _ptr(ph), _ptr(path), _ptr(cnt), C.c_void_p(st.cuda_stream)))
        out["result"] = res.as_dict()
        for k, v in (("logw", logw), ("alive", alive), ("path_hash", ph), ("path", path), ("counters", cnt)):
            if v is not None:
                out[k] = v
        return out


class PermEstBatch:
    """Many matrices of uneven order resident on one GPU; every run executes
    all their trajectories in one persistent launch."""

    def __init__(self, mats, device: int = 0, force_hbm: bool = False):
        import torch  # noqa: F401

        self._lib = N.load()
        self.count = len(mats)
        self.n = [int(M.n) for M in mats]
        self.device = device
        keep = []

        def arr(a, dt):
            x = np.ascontiguousarray(a, dtype=dt)
            keep.append(x)
            return x.ctypes.data

        weighted = [M.val is not None for M in mats]
        if any(weighted) and not all(weighted):
            raise ValueError("a batch must be all 0/1 or all weighted")
        ns = np.array(self.n, dtype=np.int32)
        zs = np.array([M.nnz for M in mats], dtype=np.int64)
        ptr_arr = lambda xs: (C.c_void_p * self.count)(*xs)  # noqa: E731
        rp = ptr_arr([arr(M.row_ptr, np.int32) for M in mats])
        ci = ptr_arr([arr(M.col_idx, np.int32) for M in mats])
        cp = ptr_arr([arr(M.col_ptr, np.int32) for M in mats])
        ri = ptr_arr([arr(M.row_idx, np.int32) for M in mats])
        vals = ptr_arr([arr(M.val, np.float32) for M in mats]) if all(weighted) else None
        self._h = C.c_void_p()
        opts = N.Options(device, N.PE_FLAG_FORCE_HBM if force_hbm else 0)
        cast = lambda x: C.cast(x, C.POINTER(C.c_void_p))  # noqa: E731
        N.check(self._lib.perm_est_create_batch(
            self.count, ns.ctypes.data, zs.ctypes.data, cast(rp), cast(ci), cast(cp), cast(ri),
            None if vals is None else cast(vals), C.byref(opts), C.byref(self._h)))

    def close(self):
        if self._h:
            self._lib.perm_est_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, n_traj, seed: int, schedule: N.Schedule, *, want_logw=True, want_alive=True,
            want_hash=False, autotune=False, stream=None) -> Dict:
        """n_traj: an int (same for every matrix) or one count per matrix.
        Returns per-matrix statistics and the concatenated device outputs."""
        import torch

        counts = np.array([n_traj] * self.count if np.isscalar(n_traj) else list(n_traj), dtype=np.int64)
        total = int(counts.sum())
        dev = torch.device("cuda", self.device)
        logw = torch.empty(total, dtype=torch.float64, device=dev) if want_logw else None
        alive = torch.empty(total, dtype=torch.uint8, device=dev) if want_alive else None
        ph = torch.empty(total, dtype=torch.int64, device=dev) if want_hash else None
        res = (N.Result * self.count)()
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        N.check(self._lib.perm_est_run_batch(
            self._h, counts.ctypes.data, C.c_uint64(seed), C.byref(schedule), res,
            _ptr(logw), _ptr(alive), _ptr(ph), N.PE_RUN_AUTOTUNE if autotune else 0,
            C.c_void_p(st.cuda_stream)))
        out = {"results": [r.as_dict() for r in res], "offsets": np.concatenate([[0], np.cumsum(counts)])}
        for k, v in (("logw", logw), ("alive", alive), ("path_hash", ph)):
            if v is not None:
                out[k] = v
        return out
