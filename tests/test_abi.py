"""The C ABI library loads and exports every entry point that
include/perm_est.h declares (no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "perm_est.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*[\s\*]+(perm_est_[a-z_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("perm_est_create", "perm_est_run", "perm_est_run_range", "perm_est_destroy",
                     "perm_est_schedule_preset", "perm_est_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2608_15390_amd import _native as N
    if not os.path.exists(N.LIB_PATH):
        pytest.fail("libpermest.so is not built (python -m paper_2608_15390_amd.build)")
    lib = ctypes.CDLL(N.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(N.EXPORTS) == sorted(declared_functions())


def test_presets_and_errors_without_gpu():
    from paper_2608_15390_amd import _native as N
    import paper_2608_15390_amd as P
    s = P.preset("local_threshold")
    assert (s.sk_policy, s.dm_policy, s.initial_dm, s.K0, s.K) == (3, 2, 1, 100, 10)
    assert abs(s.theta_th - 0.33) < 1e-15
    with pytest.raises(N.PermEstError) as ei:
        P.preset("no_such_variant")
    assert ei.value.code == N.PE_EINVAL


def test_model_file_round_trip_and_rejections(tmp_path):
    """perm_est_model_save / perm_est_model_load (host only): the values
    come back bit for bit; a flipped byte, a truncated file, another
    parameter count or a missing file are rejected with the stated codes."""
    import numpy as np
    import paper_2608_15390_amd as P
    from paper_2608_15390_amd import _native as N
    g = np.random.default_rng(3)
    th = g.normal(0, 1, P.MLP_NPARAM).astype(np.float32)
    th[5] = -0.0
    f = str(tmp_path / "net.pemlp")
    P.save_model(f, th, 0.01)
    got, a = P.load_model(f)
    assert a == 0.01 and got.tobytes() == th.tobytes()
    raw = bytearray(open(f, "rb").read())
    assert raw[:8] == b"PEMLP001" and len(raw) == 8 + 4 + 4 + 8 + 4 * P.MLP_NPARAM + 8
    for pos in (3, 9, 20, 100, len(raw) - 1):
        bad = bytearray(raw)
        bad[pos] ^= 0x10
        open(f, "wb").write(bytes(bad))
        with pytest.raises(N.PermEstError) as ei:
            P.load_model(f)
        assert ei.value.code == N.PE_EINVAL, pos
    open(f, "wb").write(bytes(raw[:-3]))
    with pytest.raises(N.PermEstError) as ei:
        P.load_model(f)
    assert ei.value.code == N.PE_EINVAL
    with pytest.raises(N.PermEstError) as ei:
        P.load_model(str(tmp_path / "missing"))
    assert ei.value.code == N.PE_EIO
    bad = th.copy()
    bad[0] = np.inf
    with pytest.raises(N.PermEstError) as ei:
        P.save_model(f, bad, 0.01)
    assert ei.value.code == N.PE_EINVAL
    with pytest.raises(N.PermEstError) as ei:
        P.save_model(f, th, 1.5)
    assert ei.value.code == N.PE_EINVAL
