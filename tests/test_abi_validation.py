"""perm_est_create rejects malformed input on the host, before any GPU
work, with PE_EINVAL / PE_ENOTSUP (runs without a GPU)."""
import ctypes as C

import numpy as np
import pytest

from paper_2608_15390_amd import _native as N
from paper_2608_15390_amd import inputs as G


def _create(n, nnz, rp, ci, cp, ri, val=None):
    L = N.load()
    h = C.c_void_p()
    arr = [np.ascontiguousarray(a, dtype=np.int32) for a in (rp, ci, cp, ri)]
    v = None if val is None else np.ascontiguousarray(val, dtype=np.float32)
    rc = L.perm_est_create(n, nnz, *[a.ctypes.data for a in arr],
                           None if v is None else v.ctypes.data, None, C.byref(h))
    return rc, L.perm_est_last_error().decode()


def test_rejects_bad_matrices():
    M = G.config_small(1)
    base = [M.row_ptr, M.col_idx, M.col_ptr, M.row_idx]
    assert _create(0, 0, *base)[0] == N.PE_EINVAL
    ci = M.col_idx.copy(); ci[3] = M.n  # out of range
    assert _create(M.n, M.nnz, M.row_ptr, ci, M.col_ptr, M.row_idx)[0] == N.PE_EINVAL
    ci = M.col_idx.copy(); ci[[0, 1]] = ci[[1, 0]]  # unsorted row
    assert _create(M.n, M.nnz, M.row_ptr, ci, M.col_ptr, M.row_idx)[0] == N.PE_EINVAL
    rp = M.row_ptr.copy(); rp[-1] -= 1  # ptr[n] != nnz
    assert _create(M.n, M.nnz, rp, M.col_idx, M.col_ptr, M.row_idx)[0] == N.PE_EINVAL
    val = np.ones(M.nnz, dtype=np.float32); val[5] = 0.0  # non-positive value
    rc, msg = _create(M.n, M.nnz, *base, val=val)
    assert rc == N.PE_EINVAL and "values" in msg
    val[5] = np.nan
    assert _create(M.n, M.nnz, *base, val=val)[0] == N.PE_EINVAL


def test_rejects_degree_beyond_u16():
    n = 70000
    rows = np.zeros(n, dtype=np.int64)
    cols = np.arange(n)
    M = G.from_coo(n, np.concatenate([rows, np.arange(n)]), np.concatenate([cols, np.arange(n)]))
    rc, msg = _create(M.n, M.nnz, M.row_ptr, M.col_idx, M.col_ptr, M.row_idx)
    assert rc == N.PE_ENOTSUP


def test_learned_and_training_entry_points_reject_bad_arguments():
    """Argument checks that run before any device work."""
    L = N.load()
    P = C.c_void_p
    out = P()
    # trainer: NULL output, NULL or non-finite parameters
    assert L.perm_est_mlp_create(0, None, None) == N.PE_EINVAL
    assert L.perm_est_mlp_create(0, None, C.byref(out)) == N.PE_EINVAL
    bad = np.zeros(N.PE_MLP_NPARAM, dtype=np.float32)
    bad[100] = np.inf
    assert L.perm_est_mlp_create(0, bad.ctypes.data, C.byref(out)) == N.PE_EINVAL
    assert not out.value
    # NULL handles
    assert L.perm_est_set_model(None, None, 0.05, None) == N.PE_EINVAL
    assert L.perm_est_mlp_forward(None, None, 1, None, None) == N.PE_EINVAL
    assert L.perm_est_mlp_get_params(None, None, None) == N.PE_EINVAL
    loss = C.c_double()
    assert L.perm_est_mlp_loss_grad(None, None, None, None, None, 0, 1, C.byref(loss), None, None) == N.PE_EINVAL
    assert L.perm_est_mlp_train(None, None, None, None, None, 1, 1, 1, 1e-3, 0, None, None) == N.PE_EINVAL
    nr, ng = C.c_int64(), C.c_int64()
    counts = np.ones(1, dtype=np.int64)
    assert L.perm_est_record(None, counts.ctypes.data, 0, None, None, None, C.byref(nr), C.byref(ng),
                             None) == N.PE_EINVAL
    L.perm_est_mlp_destroy(None)


def test_learned_presets():
    import paper_2608_15390_amd as Pk
    s = Pk.preset("learned")
    assert (s.sk_policy, s.dm_policy, s.initial_dm, s.K0) == (4, 0, 1, 100)
    assert Pk.preset("learned_threshold").dm_policy == 2
