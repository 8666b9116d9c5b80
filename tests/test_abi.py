"""The C ABI: the built library loads on a host without a GPU, exports every
function include/lbm.h declares, the Python binding names exactly those, and
the argument checks that run before any device work reject bad calls."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[A-Za-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lbm():
    from paper_2512_12213_amd import lbm as L
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("liblbm.so is not built (run __graft_entry__.build())")
    L.lib()
    return L


def test_header_declares_the_hot_path():
    names = declared()
    for n in ("lbm_create", "lbm_step", "lbm_stress", "lbm_wall_force", "lbm_force_balance"):
        assert n in names


def test_every_declared_symbol_is_exported(lbm):
    raw = C.CDLL(lbm.LIB_PATH)
    missing = [n for n in declared() if not hasattr(raw, n)]
    assert not missing, missing


def test_binding_matches_header(lbm):
    assert sorted(lbm.EXPORTED) == declared()


def test_enum_values_match_header(lbm):
    src = open(HEADER).read()
    for name in ("LBM_D2Q9", "LBM_D3Q19", "LBM_FORCE_HE", "LBM_FORCE_LUO", "LBM_FORCE_SHANCHEN", "LBM_FORCE_EDM",
                 "LBM_FORCE_GUO", "LBM_F64", "LBM_F32", "LBM_F16", "LBM_BF16", "LBM_OK", "LBM_EINVAL",
                 "LBM_ENOMEM", "LBM_EHIP", "LBM_ESTATE", "LBM_EUNSTABLE", "LBM_MAX_GROUPS", "LBM_NREC",
                 "LBM_EQ_NS", "LBM_EQ_STOKES"):
        m = re.search(r"\b%s\s*=\s*(-?\d+)" % name, src)
        assert m, name
        assert getattr(lbm, name) == int(m.group(1)), name


def test_null_context_is_rejected_without_device_work(lbm):
    L = lbm.lib()
    L.lbm_destroy(None)
    for name, _res, args in lbm._SIGS:
        if name in ("lbm_create", "lbm_destroy", "lbm_last_error"):
            continue
        call = [None] + [None if (a is C.c_void_p or hasattr(a, "contents")) else 0 for a in args[1:]]
        rc = getattr(L, name)(*call)
        assert rc == lbm.LBM_EINVAL, name
        assert "null" in lbm.last_error()


@pytest.mark.parametrize("args,msg", [
    ((7, 64, 32, 1, 0.8, 1.0, 1.0, 4), "lattice"),
    ((0, 64, 32, 2, 0.8, 1.0, 1.0, 4), "nz"),
    ((1, 0, 32, 32, 0.8, 1.0, 1.0, 4), "size"),
    ((1, 64, 32, 32, 0.5, 1.0, 1.0, 4), "tau"),
    ((1, 64, 32, 32, 0.8, -1.0, 1.0, 4), "dx"),
    ((1, 64, 32, 32, 0.8, 1.0, 1.0, 9), "force"),
    ((1, 70000, 32, 32, 0.8, 1.0, 1.0, 4), "size"),
    ((1, 4096, 4096, 256, 0.8, 1.0, 1.0, 4), "too large"),
])
def test_create_rejects_bad_arguments(lbm, args, msg):
    L = lbm.lib()
    assert not L.lbm_create(*args)
    assert msg in lbm.last_error().lower()


def test_binding_fails_loudly_without_the_library(monkeypatch):
    from paper_2512_12213_amd import lbm as L
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", os.path.join(ROOT, "no_such_dir", "liblbm.so"))
    with pytest.raises(ImportError):
        L.lib()
    with pytest.raises(ImportError):
        L.Lattice(L.LBM_D2Q9, 8, 8, 1, 0.8)
