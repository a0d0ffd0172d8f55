"""Host-side checks of the C-ABI library (no GPU needed, no device work)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1301_3460_amd as lgf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_built():
    assert os.path.exists(lgf.LIB_PATH), "run python -m paper_1301_3460_amd.build"


def test_every_declared_symbol_is_exported():
    declared = lgf.EXPORTS
    assert "lgf_fix" in declared and "lgf_create" in declared and len(declared) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", lgf.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(lgf_\w+)$", out, re.M))
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    lib = lgf.load()
    for s in declared:
        assert getattr(lib, s) is not None


def test_library_has_gfx950_code_object():
    with open(lgf.LIB_PATH, "rb") as f:
        blob = f.read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def _create(L, prec=0):
    lib = lgf.load()
    h = ctypes.c_void_p()
    arr = (ctypes.c_int * 4)(*L)
    rc = lib.lgf_create(ctypes.byref(h), ctypes.byref(arr), prec, None)
    return rc, lib.lgf_last_error(None).decode(), h


@pytest.mark.parametrize("L", [(5, 4, 4, 4), (4, 4, 4, 0), (4, 4, 4, 7), (4, 4, 4, 512),
                               (4, 4, 4, 384), (1, 4, 4, 4), (4, -4, 4, 4), (10, 4, 4, 4)])
def test_create_rejects_unsupported_extents_before_touching_the_device(L):
    rc, msg, h = _create(L)
    assert rc == lgf.LGF_ERR_ARG
    assert "extent" in msg
    assert not h.value


def test_create_rejects_bad_precision():
    rc, msg, _ = _create((4, 4, 4, 4), prec=7)
    assert rc == lgf.LGF_ERR_ARG and "precision" in msg


def test_null_context_calls_are_argument_errors():
    lib = lgf.load()
    r = lgf._Result()
    assert lib.lgf_fix(None, None, 0.08, 1e-15, 10, ctypes.byref(r)) == lgf.LGF_ERR_ARG
    assert lib.lgf_iterate(None, None, 0.08, 1, ctypes.byref(r)) == lgf.LGF_ERR_ARG
    d = ctypes.c_double()
    assert lib.lgf_theta(None, None, ctypes.byref(d)) == lgf.LGF_ERR_ARG
    assert lib.lgf_set_theta_switch(None, 1e-8) == lgf.LGF_ERR_ARG
    lib.lgf_destroy(None)  # no-op
    assert isinstance(lib.lgf_last_error(None), bytes)


def test_header_documents_every_entry_point():
    with open(os.path.join(ROOT, "include", "lgf.h")) as f:
        text = f.read()
    for name in lgf.EXPORTS:
        # every declaration is preceded by a comment block
        m = re.search(r"^(?:int|void|const char)\s*\*?\s*" + name + r"\(", text, re.M)
        assert m, name
        idx = m.start()
        assert "*/" in text[max(0, idx - 1200):idx], name


def test_measure_noalloc_rejects_arguments_before_touching_the_device():
    lib = lgf.load()
    out = ctypes.c_void_p(16)  # never dereferenced: the call fails its argument checks
    big = (ctypes.c_int * 4)(128, 128, 64, 64)  # 2^26 sites, beyond the fixed scratch
    assert lib.lgf_measure_noalloc(ctypes.byref(big), out, out, None) == lgf.LGF_ERR_ARG
    assert b"sites" in lib.lgf_last_error(None)
    bad = (ctypes.c_int * 4)(5, 4, 4, 4)
    assert lib.lgf_measure_noalloc(ctypes.byref(bad), out, out, None) == lgf.LGF_ERR_ARG
    ok = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert lib.lgf_measure_noalloc(ctypes.byref(ok), None, out, None) == lgf.LGF_ERR_ARG


@pytest.mark.parametrize("L", [(9, 18, 27, 36), (72, 144, 2, 2), (192, 4, 4, 4), (256, 2, 2, 2),
                               (243, 81, 2, 2), (54, 108, 162, 2), (216, 3, 3, 3)])
def test_create_accepts_every_2a3b_extent_up_to_256(L):
    """Every 2^a 3^b extent from 2 to 256 passes the argument checks (on a host
    without a GPU the call then stops at the device lookup)."""
    rc, msg, h = _create(L)
    assert rc != lgf.LGF_ERR_ARG, msg
    if h.value:
        lgf.load().lgf_destroy(h)
