"""CPU checks of the boundary: the library loads and exports every function the
header declares; host-side argument checks need no GPU."""
from __future__ import annotations

import ctypes
import os

import pytest

import paper_2503_20286_amd as nsga3


def test_header_declares_expected_entry_points():
    names = nsga3.header_symbols()
    for n in ("nsga3_create", "nsga3_destroy", "nsga3_reserve", "nsga3_select",
              "nsga3_status_string", "nsga3_workspace_size", "nsga3_profile",
              "nsga3_phase_times", "nsga3_version"):
        assert n in names


def test_library_exports_every_declared_symbol():
    exp = nsga3.exported_symbols()
    missing = [k for k, v in exp.items() if not v]
    assert not missing, f"not exported: {missing}"


def test_status_strings_and_version():
    L = nsga3.load()
    for code in (0, -1, -2, -3, -4, -5):
        assert L.nsga3_status_string(code)
    assert nsga3.version() >= 100


def test_workspace_size_query_and_argument_checks():
    L = nsga3.load()
    sz = ctypes.c_size_t()
    assert L.nsga3_workspace_size(200000, 5, 210, ctypes.byref(sz)) == 0
    assert 10_000_000 < sz.value < 2_000_000_000
    small = ctypes.c_size_t()
    assert L.nsga3_workspace_size(200, 3, 91, ctypes.byref(small)) == 0
    assert small.value < sz.value
    for args in ((0, 5, 10), (10, 1, 10), (10, 17, 10), (10, 3, 0), (10, 3, 65536), (2**31, 3, 5)):
        assert L.nsga3_workspace_size(*args, ctypes.byref(sz)) == -1
    # null context / pointers are rejected before anything touches a device
    assert L.nsga3_select(None, None, 10, 3, None, 5, 5, None, None, None, None, None, None,
                          None, None) == -1
    assert L.nsga3_reserve(None, 10, 3, 5) == -1
    assert L.nsga3_profile(None, 1) == -1
    L.nsga3_destroy(None)


def test_library_missing_fails_loudly(monkeypatch, tmp_path):
    import importlib
    from paper_2503_20286_amd import _native
    monkeypatch.setenv("NSGA3_LIB", str(tmp_path / "nope.so"))
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(ImportError):
        _native.load()
    monkeypatch.delenv("NSGA3_LIB")
    monkeypatch.setattr(_native, "_lib", None)
    importlib.reload(_native)


def test_plan_stage_names_match_header():
    """The binding names one stage per entry of the header's stage arrays."""
    import re
    from paper_2503_20286_amd import _native
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "nsga3.h")
    with open(hdr) as fh:
        m = re.search(r"#define NSGA3_PLAN_STAGES (\d+)", fh.read())
    assert m and int(m.group(1)) == len(_native.PLAN_STAGES)
    assert _native.PLAN_STAGES[-1] == "done"
