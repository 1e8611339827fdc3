"""The C-ABI library loads and exports every function include/aoresp.h
declares; host-side argument checks behave as documented.  No GPU needed: none
of the calls below reaches a device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aoresp.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "return")))


@pytest.fixture(scope="module")
def lib():
    from paper_2502_06337_amd import _lib
    return _lib.load()


def test_header_parsed():
    names = declared_functions()
    for must in ("est_rotation", "est_rotations_topk", "est_rotation_batch", "aoresp_server_create",
                 "aoresp_submit", "aoresp_poll", "aoresp_server_stats", "aoresp_server_destroy"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2502_06337_amd import _lib
    names = declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding covers every declared entry point
    assert set(names) <= set(_lib.SIGNATURES), set(names) - set(_lib.SIGNATURES)


def test_grid_for_n_is_pure_and_in_range(lib):
    vals = [lib.aoresp_grid_for_n(n) for n in (0, 10, 1000, 5000, 50000, 500000, 10 ** 7)]
    assert vals == [lib.aoresp_grid_for_n(n) for n in (0, 10, 1000, 5000, 50000, 500000, 10 ** 7)]
    assert all(v in (128, 256, 512, 1024) for v in vals)
    assert vals == sorted(vals)


def test_strerror(lib):
    for st in range(-6, 1):
        assert lib.aoresp_strerror(st)
    assert b"gfx950" in lib.aoresp_version()


@pytest.mark.parametrize("field,val", [("grid", 100), ("grid", 32), ("grid", 8192), ("refine_grid", 3),
                                       ("refine_grid", 256), ("angle_bins", 1), ("angle_bins", 9000),
                                       ("angle_gate", 2), ("angle_refine", 257), ("angle_refine", 200),
                                       ("vote_rule", 2), ("circle_samples", 3), ("circle_samples", 65537)])
def test_invalid_params_rejected_on_host(lib, field, val):
    from paper_2502_06337_amd import _lib
    prm = _lib.SolveParams(grid=256, angle_bins=360)
    setattr(prm, field, val)
    P = np.zeros((3, 4), dtype=np.float32)
    res = _lib.Result()
    st = lib.est_rotation(P.ctypes.data, P.ctypes.data, 4, C.byref(prm.c()), C.byref(res), None)
    assert st == _lib.EINVAL


def test_null_and_tiny_inputs_on_host(lib):
    from paper_2502_06337_amd import _lib
    res = _lib.Result()
    prm = _lib.SolveParams(grid=64).c()
    assert lib.est_rotation(None, None, 5, C.byref(prm), C.byref(res), None) == _lib.EINVAL
    assert lib.est_rotation(None, None, 5, C.byref(prm), None, None) == _lib.EINVAL
    P = np.ones((3, 1), dtype=np.float32)
    m = np.full(1, 7, dtype=np.uint8)
    assert lib.est_rotation(P.ctypes.data, P.ctypes.data, 1, C.byref(prm), C.byref(res), m.ctypes.data) == \
        _lib.ENODATA
    assert np.array_equal(np.array(res.R[:]).reshape(3, 3), np.eye(3)) and m[0] == 0
    found = C.c_uint32(9)
    out = (_lib.Result * 9)()
    assert lib.est_rotations_topk(P.ctypes.data, P.ctypes.data, 1, 9, C.byref(prm), out, None,
                                  C.byref(found)) == _lib.EINVAL
    assert lib.est_rotations_topk(P.ctypes.data, P.ctypes.data, 1, 0, C.byref(prm), out, None,
                                  C.byref(found)) == _lib.EINVAL
