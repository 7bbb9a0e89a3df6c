"""The C ABI library loads and exports every symbol include/bse.h declares.

No compute calls are made (there may be no GPU); only host-side arithmetic
and argument checks that return before touching the device.
"""

import ctypes
import os
import re

import pytest

import paper_1501_03830_amd as pkg
from paper_1501_03830_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bse.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\*?\s*(bse_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libbse.so is not built (python -m paper_1501_03830_amd.build)")
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["bse_ctx_create", "bse_ctx_destroy", "bse_footprint_bytes", "bse_solve",
                 "bse_last_error", "bse_version"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in bse.h but not exported"
    bound = {n for n, _, _ in _lib.SIGNATURES}
    assert set(names) <= bound, f"binding lacks {set(names) - bound}"


def test_version(lib):
    assert lib.bse_version() >= 100


def test_footprint_is_host_only_and_monotone(lib):
    assert lib.bse_footprint_bytes(0, 0, 0) == 0
    assert lib.bse_footprint_bytes(-3, 0, 0) == 0
    assert lib.bse_footprint_bytes(64, 99, 0) == 0
    prev = 0
    for n in [1, 2, 63, 64, 65, 1000, 2048, 8192]:
        f = lib.bse_footprint_bytes(n, 0, 0)
        assert f > prev
        prev = f
    # about 40 N^2 bytes of FP64 workspace (L, W, Z, V and inverse-iteration factors)
    n = 8192
    N = 2 * n
    f = lib.bse_footprint_bytes(n, 0, 0)
    assert 30 * N * N < f < 60 * N * N


def test_null_context_rejected_without_device(lib):
    rc = lib.bse_solve(None, 4, None, 4, None, 4, 0, 0, None, None, 8, None, None, None, None)
    assert rc == -1
    assert lib.bse_ctx_create(None, 0, None, 0, None) == -1
    assert lib.bse_ctx_destroy(None) == 0
    assert "ctx" in _lib.last_error()


def test_package_import_does_not_load_library():
    import importlib
    import sys
    mod = importlib.reload(sys.modules["paper_1501_03830_amd"])
    assert hasattr(mod, "Context")


def test_tile_table_host_validation(lib):
    """The tile table accessors are host-only; invalid tables are rejected
    before any device call (a NULL context is argument 1)."""
    import ctypes
    t = (ctypes.c_int * 18)()
    assert lib.bse_get_tile_table(t) == 0
    row64, row32 = list(t[:9]), list(t[9:])
    assert row64[:4] == sorted(row64[:4], reverse=True)
    assert all(1 <= v <= 16 for v in row64[4:] + row32[4:])
    assert lib.bse_set_tile_table(None, t) == -1
