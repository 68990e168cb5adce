"""The C-ABI library without a GPU: it loads, exports every entry point that
include/sublabel.h declares, and its host-only calls (status strings, argument checks and
workspace sizing, which touch no device) behave as the header documents. CPU only: no
call here launches or allocates anything on a device.
"""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sublabel.h")
LIB_PATH = os.path.join(ROOT, "paper_1512_01383_amd", "libsublabel.so")


def _declared():
    """Function names declared in the header (comments stripped)."""
    txt = re.sub(r"/\*.*?\*/", " ", open(HEADER).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(sl_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB_PATH):
        pytest.fail(f"{LIB_PATH} is missing: build it with `python -m paper_1512_01383_amd.build`")
    import paper_1512_01383_amd as S
    return S.lib()


@pytest.fixture(scope="module")
def S():
    import paper_1512_01383_amd as mod
    return mod


def test_library_exports_every_declared_entry_point(lib):
    names = _declared()
    assert len(names) == 36, names   # the entry points of include/sublabel.h
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    want = {0: "ok", 1: "invalid argument", 2: "unsupported", 3: "device error",
            4: "workspace error", 5: "numeric error"}
    for code, text in want.items():
        assert lib.sl_status_string(code).decode() == text
    assert lib.sl_status_string(99).decode() == "unknown status"


def _desc(S, H=8, W=9, L=5, rho=None, storage=0):
    gamma = np.linspace(0.0, 1.0, L)
    d = S.Desc()
    d.H, d.W, d.L = H, W, L
    d._gamma = gamma   # keep alive
    d.gamma = gamma.ctypes.data_as(C.POINTER(C.c_double))
    d.rho = S.RHO_QUAD if rho is None else rho
    d.f = 16           # never dereferenced by the host-only calls
    d.a, d.nu, d.lam = 1.0, 0.025, 0.2
    d.tv = S.TV_ISO
    d.storage = storage
    d.check_every = 50
    d.normalize_labels = 1
    return d


def _size(lib, d):
    n = C.c_size_t()
    st = lib.sl_workspace_size(C.byref(d), C.byref(n))
    return st, n.value


def test_workspace_size_covers_the_state_and_grows(lib, S):
    for H, W, L in [(1, 1, 2), (8, 9, 5), (37, 130, 11), (256, 256, 20)]:
        st, n = _size(lib, _desc(S, H, W, L))
        assert st == 0
        k = L - 1
        ps = -(-(H * W) // 64) * 64
        assert n >= (11 * k + 2) * ps * 4          # the FP32 state planes alone
    s_small = _size(lib, _desc(S, 64, 64, 8))[1]
    assert _size(lib, _desc(S, 64, 128, 8))[1] > s_small
    assert _size(lib, _desc(S, 64, 64, 16))[1] > s_small
    # BF16 dual storage keeps float-sized dual planes (widened in place for the FP32
    # finishing phase), so it needs the same workspace as FP32
    assert _size(lib, _desc(S, 64, 64, 8, storage=1))[1] == s_small


def test_argument_checks(lib, S):
    def status(d):
        return _size(lib, d)[0]
    assert status(_desc(S, H=0)) == 1
    d = _desc(S)
    d._gamma = np.array([0.0, 0.5, 0.5, 0.7, 1.0])
    d.gamma = d._gamma.ctypes.data_as(C.POINTER(C.c_double))
    assert status(d) == 1 and "increasing" in lib.sl_last_error().decode()
    max_labels = int(re.search(r"#define SL_MAX_LABELS (\d+)", open(HEADER).read()).group(1))
    assert status(_desc(S, L=max_labels)) == 0
    assert status(_desc(S, L=max_labels + 1)) == 2
    d = _desc(S)
    d.f = None
    assert status(d) == 1 and "f is NULL" in lib.sl_last_error().decode()
    d = _desc(S, rho=S.RHO_TRUNC_QUAD)
    d.nu = 0.0
    assert status(d) == 1
    d = _desc(S, rho=S.RHO_PERIODIC_QUAD)
    assert status(d) == 0
    d.nu = 0.0
    assert status(d) == 1 and "nu" in lib.sl_last_error().decode()
    assert status(_desc(S, rho=4)) == 1
    d = _desc(S)
    d.tv = S.TV_ANISO
    assert status(d) == 0
    d.tv = 2
    assert status(d) == 1 and "TV kind" in lib.sl_last_error().decode()
    # H*W = 2^29: one FP32 plane would reach 2 GiB
    assert status(_desc(S, H=1 << 15, W=1 << 14)) == 2
    assert "2^29" in lib.sl_last_error().decode()
    assert status(_desc(S, H=(1 << 15) - 1, W=1 << 14)) == 0


def test_temporal_calls_need_a_handle(lib):
    n = C.c_size_t(0)
    assert lib.sl_temporal_workspace_size(None, C.byref(n)) == 1
    assert lib.sl_set_temporal(None, None, 0) == 1
    assert lib.sl_set_temporal(None, C.c_void_p(256), 1 << 20) == 1


def test_batch_workspace_size(lib, S):
    ds = (S.Desc * 2)(_desc(S, 8, 9, 5), _desc(S, 30, 70, 9))
    # the gamma arrays of the copies must stay alive
    keep = [np.linspace(0.0, 1.0, 5), np.linspace(0.0, 1.0, 9)]
    for i in range(2):
        ds[i].gamma = keep[i].ctypes.data_as(C.POINTER(C.c_double))
    n = C.c_size_t()
    assert lib.sl_batch_workspace_size(ds, 2, C.byref(n)) == 0
    singles = sum(_size(lib, _desc(S, *hwl))[1] for hwl in [(8, 9, 5), (30, 70, 9)])
    assert n.value >= singles
    assert lib.sl_batch_workspace_size(ds, 0, C.byref(n)) == 1


def test_stereo_cost_argument_checks(lib):
    """Every rejected call fails before anything is launched (the pointers are dummies)."""
    f = lib.sl_stereo_costs
    f.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                  C.c_void_p, C.c_void_p]
    p = C.c_void_p(256)
    assert f(None, p, 8, 8, 4, 1.0, p, None) == 1
    assert f(p, p, 8, 8, 4, 1.0, None, None) == 1
    assert f(p, p, 0, 8, 4, 1.0, p, None) == 1
    assert f(p, p, 8, 8, 0, 1.0, p, None) == 1
    assert f(p, p, 8, 8, 1025, 1.0, p, None) == 2
    assert f(p, p, 1 << 15, 1 << 14, 4, 1.0, p, None) == 2
    assert f(p, p, 8, 8, 4, -1.0, p, None) == 1
    assert f(p, p, 8, 8, 4, float("nan"), p, None) == 1


def test_static_solve_argument_checks(lib, S):
    """The allocation-free solve rejects bad arguments, and problems whose workspace exceeds
    its fixed array, before any device work (the output pointers are dummies)."""
    f = lib.sl_solve_static
    p = C.c_void_p(256)
    limit = int(re.search(r"#define SL_STATIC_WORKSPACE_BYTES \((\d+)u \* 1024u \* 1024u\)",
                          open(HEADER).read()).group(1)) << 20
    assert limit == S.STATIC_WORKSPACE_BYTES
    big = _desc(S, 256, 256, 28)
    assert _size(lib, big)[1] > limit
    assert f(C.byref(big), 0.0, 10, p, p, None, None) == 2
    assert "allocation-free" in lib.sl_last_error().decode()
    ok = _desc(S, 64, 64, 8)
    assert _size(lib, ok)[1] <= limit
    assert f(C.byref(ok), 0.0, -1, p, p, None, None) == 1
    assert f(C.byref(ok), -1e-3, 10, p, p, None, None) == 1
    assert f(C.byref(ok), float("nan"), 10, p, p, None, None) == 1
    assert f(None, 0.0, 10, p, p, None, None) == 1
    bad = _desc(S, H=0)
    assert f(C.byref(bad), 0.0, 10, p, p, None, None) == 1


def test_binding_fails_loudly_without_the_library(S, monkeypatch):
    """No CPU fallback: with the library absent every entry point of the binding raises."""
    monkeypatch.setattr(S, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "libsublabel.so"))
    monkeypatch.setattr(S, "_lib", None)
    with pytest.raises(ImportError, match="missing"):
        S.lib()
