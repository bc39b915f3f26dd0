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
import os
from typing import Dict, Optional

import numpy as np

from . import _native as N
from .inputs import SparseMatrix

__all__ = ["PermEst", "PermEstBatch", "ProposalNet", "preset", "Schedule", "PermEstError", "save_model",
           "load_model", "consensus"]

PermEstError = N.PermEstError
Schedule = N.Schedule

VR_MD, VR_ROW_ORDER = 0, 1
SK_NONE, SK_FIXED, SK_ADAPTIVE, SK_LOCAL, SK_LEARNED = 0, 1, 2, 3, 4
MLP_NPARAM = N.PE_MLP_NPARAM
DM_NONE, DM_ALL, DM_THRS, DM_TRCK = 0, 1, 2, 3


def preset(name: str, **overrides) -> N.Schedule:
    """A named schedule from the library (see perm_est_schedule_preset),
    optionally with fields overridden."""
    s = N.Schedule()
    N.check(N.load().perm_est_schedule_preset(name.encode(), C.byref(s)))
    for k, v in overrides.items():
        setattr(s, k, v)
    return s


def save_model(path: str, params, mix_alpha: float) -> None:
    """Write a network (MLP_NPARAM float values, host array or tensor) and
    its uniform share to `path` (perm_est_model_save)."""
    if hasattr(params, "detach"):
        params = params.detach().cpu().numpy()
    p = np.ascontiguousarray(params, dtype=np.float32)
    if p.size != MLP_NPARAM:
        raise ValueError(f"expected {MLP_NPARAM} parameters")
    N.check(N.load().perm_est_model_save(os.fsencode(path), p.ctypes.data, float(mix_alpha)))


def load_model(path: str):
    """(params as a float32 numpy array, mix_alpha) from a file written by
    save_model (perm_est_model_load)."""
    p = np.empty(MLP_NPARAM, dtype=np.float32)
    a = C.c_double()
    N.check(N.load().perm_est_model_load(os.fsencode(path), p.ctypes.data, C.byref(a)))
    return p, a.value


_CHECK_NAMES = {N.PE_CON_ALL_RUNS: "all_runs_present", N.PE_CON_T_INTERVALS: "t_intervals_intersect",
                N.PE_CON_BONFERRONI: "d_max_within_bonferroni", N.PE_CON_ALIVE: "alive_at_least_1000",
                N.PE_CON_ESS: "ess_at_least_1000", N.PE_CON_HALF_WIDTH: "half_width_within_10pct"}
_RESULT_KEYS = ("log_estimate", "rse", "n_traj", "n_alive", "ess")


def consensus(runs, alpha: float = 0.05) -> Dict:
    """Multi-seed consensus diagnostics (perm_est_consensus) of runs given as
    a list over variants of lists over seeds of result dicts (the `result`
    of PermEst.run: log_estimate, rse, n_traj, n_alive, ess are used)."""
    V, R = len(runs), len(runs[0])
    if any(len(r) != R for r in runs):
        raise ValueError("every variant needs the same number of seeds")
    arr = (N.Result * (V * R))()
    for p in range(V):
        for r in range(R):
            for k in _RESULT_KEYS:
                setattr(arr[p * R + r], k, runs[p][r][k])
    out = N.ConsensusResult()
    ly = np.zeros(V)
    re = np.zeros(V)
    N.check(N.load().perm_est_consensus(V, R, arr, float(alpha), C.byref(out), ly.ctypes.data, re.ctypes.data))
    d = out.as_dict()
    d["checks"] = {name: bool(out.checks & bit) for bit, name in _CHECK_NAMES.items()}
    d["provisional"] = bool(out.provisional)
    d["log_ybar"] = ly.tolist()
    d["rel_e"] = re.tolist()
    return d


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


class _ModelMixin:
    def set_model(self, params, mix_alpha: float = 0.05, stream=None):
        """Install the learned proposal's network: params is a float32
        device tensor of MLP_NPARAM values (snapped to the inference grid by
        the library)."""
        import torch

        if params.dtype != torch.float32 or not params.is_cuda or params.numel() != MLP_NPARAM:
            raise ValueError("params must be a float32 device tensor of MLP_NPARAM values")
        params = params.contiguous()
        st = stream if stream is not None else torch.cuda.current_stream(params.device)
        N.check(self._lib.perm_est_set_model(self._h, _ptr(params), float(mix_alpha), C.c_void_p(st.cuda_stream)))


class PermEst(_ModelMixin):
    """One sparse matrix resident on one GPU."""

    def __init__(self, M: SparseMatrix, device: int = 0, force_hbm: bool = False, wave_per_trajectory: bool = False):
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
        opts = N.Options(device, (N.PE_FLAG_FORCE_HBM if force_hbm else 0) |
                         (N.PE_FLAG_WAVE_PER_TRAJECTORY if wave_per_trajectory else 0))
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
            stream=None, noalloc=False) -> Dict:
        """Run trajectories first..first+count-1; returns the statistics and
        the requested per-trajectory device tensors.  noalloc: through
        perm_est_run_range_noalloc (the library allocates nothing; the
        schedule's preprocessing must have run on this handle before)."""
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
        fn = self._lib.perm_est_run_range_noalloc if noalloc else self._lib.perm_est_run_range
        N.check(fn(
            self._h, first, count, C.c_uint64(seed), C.byref(schedule), C.byref(res),
            _ptr(logw), _ptr(alive), _ptr(ph), _ptr(path), _ptr(cnt), C.c_void_p(st.cuda_stream)))
        out["result"] = res.as_dict()
        for k, v in (("logw", logw), ("alive", alive), ("path_hash", ph), ("path", path), ("counters", cnt)):
            if v is not None:
                out[k] = v
        return out


class PermEstBatch(_ModelMixin):
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
            want_hash=False, autotune=False, graph=False, stream=None) -> Dict:
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
            _ptr(logw), _ptr(alive), _ptr(ph),
            (N.PE_RUN_AUTOTUNE if autotune else 0) | (N.PE_RUN_GRAPH if graph else 0),
            C.c_void_p(st.cuda_stream)))
        out = {"results": [r.as_dict() for r in res], "offsets": np.concatenate([[0], np.cumsum(counts)])}
        for k, v in (("logw", logw), ("alive", alive), ("path_hash", ph)):
            if v is not None:
                out[k] = v
        return out

    def record(self, n_traj, seed: int, schedule: N.Schedule, *, rec_cap: int, group_cap: int,
               stride: int = 1, stream=None) -> Dict:
        """Run the batch and record training pairs (features, proposal of the
        running schedule) at every stride-th step; returns the statistics and
        the written prefix of the recording as device tensors."""
        import torch

        counts = np.array([n_traj] * self.count if np.isscalar(n_traj) else list(n_traj), dtype=np.int64)
        dev = torch.device("cuda", self.device)
        x = torch.empty((rec_cap, 8), dtype=torch.float32, device=dev)
        y = torch.empty(rec_cap, dtype=torch.float32, device=dev)
        gs = torch.empty(group_cap, dtype=torch.int64, device=dev)
        gi = torch.empty((group_cap, 4), dtype=torch.int32, device=dev)
        buf = N.RecordBuffers(_ptr(x), _ptr(y), _ptr(gs), _ptr(gi), rec_cap, group_cap, stride, 0)
        res = (N.Result * self.count)()
        nr, ng = C.c_int64(), C.c_int64()
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        N.check(self._lib.perm_est_record(self._h, counts.ctypes.data, C.c_uint64(seed), C.byref(schedule),
                                          C.byref(buf), res, C.byref(nr), C.byref(ng),
                                          C.c_void_p(st.cuda_stream)))
        nr, ng = nr.value, ng.value
        return {"results": [r.as_dict() for r in res], "x": x[:nr], "y": y[:nr], "gstart": gs[:ng],
                "ginfo": gi[:ng], "n_records": nr, "n_groups": ng}


class ProposalNet:
    """Trainer of the learned proposal's network on one GPU (float master
    parameters, Adam moments), driving the library's matrix-core kernels."""

    def __init__(self, params, device: int = 0):
        import torch  # noqa: F401

        self._lib = N.load()
        self.device = device
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != MLP_NPARAM:
            raise ValueError(f"expected {MLP_NPARAM} parameters")
        self._h = C.c_void_p()
        N.check(self._lib.perm_est_mlp_create(device, p.ctypes.data, C.byref(self._h)))

    def close(self):
        if self._h:
            self._lib.perm_est_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self, stream=None):
        """A float32 device tensor copy of the current parameters."""
        import torch

        out = torch.empty(MLP_NPARAM, dtype=torch.float32, device=torch.device("cuda", self.device))
        N.check(self._lib.perm_est_mlp_get_params(self._h, _ptr(out), self._stream(stream)))
        return out

    def _stream(self, stream):
        import torch

        st = stream if stream is not None else torch.cuda.current_stream(torch.device("cuda", self.device))
        return C.c_void_p(st.cuda_stream)

    def forward(self, x, stream=None):
        import torch

        x = x.contiguous()
        out = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        N.check(self._lib.perm_est_mlp_forward(self._h, _ptr(x), x.shape[0], _ptr(out), self._stream(stream)))
        return out

    def loss_grad(self, rec: Dict, g0: int = 0, g1: Optional[int] = None, stream=None):
        import torch

        g1 = rec["n_groups"] if g1 is None else g1
        grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device=rec["x"].device)
        loss = C.c_double()
        N.check(self._lib.perm_est_mlp_loss_grad(
            self._h, _ptr(rec["x"]), _ptr(rec["y"]), _ptr(rec["gstart"]), _ptr(rec["ginfo"]), g0, g1,
            C.byref(loss), _ptr(grad), self._stream(stream)))
        return loss.value, grad

    def train(self, rec: Dict, epochs: int, batch_groups: int, lr: float, seed: int = 0, stream=None):
        losses = (C.c_double * max(epochs, 1))()
        N.check(self._lib.perm_est_mlp_train(
            self._h, _ptr(rec["x"]), _ptr(rec["y"]), _ptr(rec["gstart"]), _ptr(rec["ginfo"]),
            rec["n_groups"], epochs, batch_groups, float(lr), C.c_uint64(seed), losses, self._stream(stream)))
        return [losses[i] for i in range(epochs)]
