"""The C-ABI library loads on the CPU and exports every function include/aroam.h declares
(no compute calls: those need the GPU)."""
import ctypes
import os
import re

import pytest

import paper_2009_10173_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "aroam.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aroam_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["aroam_build_model", "aroam_forward", "aroam_adjoint", "aroam_solve_lsqr",
              "aroam_solve_l1", "aroam_model_query", "aroam_model_export_table",
              "aroam_model_destroy", "aroam_last_error", "aroam_forward_batch",
              "aroam_adjoint_batch"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(P.library_path())
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_mirrors_every_entry_point():
    for n in _declared():
        assert callable(getattr(P, n)), n


def test_struct_layouts_match_header():
    # field order and C sizes of the public structs
    assert ctypes.sizeof(P.binding.Sensor) == 48
    assert ctypes.sizeof(P.binding.Grid) == 64
    assert ctypes.sizeof(P.binding.SolveOpts) == 56
    assert ctypes.sizeof(P.binding.SolveInfo) == 48


def test_host_side_argument_errors_without_gpu():
    """Calls that fail argument validation return before touching the device."""
    lib = P.load_library()
    assert lib.aroam_model_query(None, None) == -1
    assert "NULL" in P.aroam_last_error()
    assert lib.aroam_forward(None, 1, None, None, None) == -1
    assert lib.aroam_solve_lsqr(None, None, None, None, None, None) == -1
    lib.aroam_model_destroy(None)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setenv("AROAM_LIB", str(tmp_path / "nope.so"))
    monkeypatch.setattr(P.binding, "_LIB", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        P.binding.load_library()
