"""The C-ABI library loads and exports every symbol include/sqh.h declares
(no device needed; no compute calls)."""
import ctypes
import os
import re

import pytest

from paper_1501_04706_amd import sqh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sqh.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sqh_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for s in ["sqh_create", "sqh_destroy", "sqh_hull", "sqh_hull_batched", "sqh_workspace_bytes",
              "sqh_set_precision", "sqh_get_stats", "sqh_strerror"]:
        assert s in syms


def test_library_exports_all_declared_symbols():
    lib = sqh.load()
    for s in declared_symbols():
        assert hasattr(lib, s), f"libsqh.so does not export {s}"
    # no stray C++ mangling of the ABI
    lib2 = ctypes.CDLL(sqh.LIB_PATH)
    for s in declared_symbols():
        getattr(lib2, s)


def test_workspace_bytes_host_only():
    a = sqh.sqh_workspace_bytes(100_000, 1)
    b = sqh.sqh_workspace_bytes(20_000_000, 1)
    assert 0 < a < b
    # survivor buffers (2 x 12 B/pt) at least
    assert b >= 24 * 20_000_000
    assert sqh.sqh_workspace_bytes(-1, 1) == 0
    assert sqh.sqh_workspace_bytes(10, 0) == 0
    assert sqh.sqh_workspace_bytes(2 ** 31, 1) == 0
    assert sqh.sqh_workspace_bytes(0, 1) > 0


def test_strerror():
    assert "workspace" in sqh.sqh_strerror(sqh.SQH_ENOMEM)
    assert sqh.sqh_strerror(12345) == "unknown error"
