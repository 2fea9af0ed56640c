"""The C-ABI library loads on the CPU and exports every function include/aroam.h declares
(no compute calls: those need the GPU)."""
import ctypes
import os
import re
import subprocess

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


_STRUCTS = {"aroam_sensor": "Sensor", "aroam_grid": "Grid", "aroam_model_info": "ModelInfo",
            "aroam_filter": "Filter",
            "aroam_solve_opts": "SolveOpts", "aroam_solve_info": "SolveInfo"}
_RENAMED = {"lambda_": "lambda"}


def test_struct_layouts_match_header(tmp_path):
    """Sizes and field offsets of the binding's ctypes structs equal what a C compiler makes of
    include/aroam.h."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "aroam.h"', "int main(void) {"]
    for cname, pyname in _STRUCTS.items():
        st = getattr(P.binding, pyname)
        lines.append(f'printf("{pyname} size %zu\\n", sizeof({cname}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{pyname} {f} %zu\\n", offsetof({cname}, {_RENAMED.get(f, f)}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    for line in filter(None, out):
        pyname, field, value = line.split()
        st = getattr(P.binding, pyname)
        got = ctypes.sizeof(st) if field == "size" else getattr(st, field).offset
        assert got == int(value), (pyname, field, got, value)


def test_import_model_rejects_bad_tables_without_gpu():
    """aroam_import_model validates the grid, the windows and the values before any device
    call."""
    import numpy as np
    lib = P.load_library()
    g = P.binding._grid(dict(c_mps=1500.0, fs_hz=250e6, nx=4, ny=4, step_m=1e-5, nz=3,
                             dz_m=1e-5, nt=8, k_half=1, footprint_mode=0))
    H = np.zeros((3, 3, 3, 8))
    lo = np.full((3, 3, 3), -1, dtype=np.int32)
    hi = lo.copy()
    h = ctypes.c_void_p()
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert lib.aroam_import_model(None, ptr(H), None, None, 0, None, ctypes.byref(h)) == -1
    assert lib.aroam_import_model(ctypes.byref(g), ptr(H), ptr(lo), None, 0, None,
                                  ctypes.byref(h)) == -1
    lo[1, 1, 0], hi[1, 1, 0] = 5, 8          # window beyond nt
    assert lib.aroam_import_model(ctypes.byref(g), ptr(H), ptr(lo), ptr(hi), 0, None,
                                  ctypes.byref(h)) == -1
    assert "window" in P.aroam_last_error()
    H[1, 1, 0, 3] = np.nan                   # non-finite value inside a derived window
    H[1, 1, 0, 2] = 1.0
    assert lib.aroam_import_model(ctypes.byref(g), ptr(H), None, None, 0, None,
                                  ctypes.byref(h)) == -4
    assert not h.value


def test_host_side_argument_errors_without_gpu():
    """Calls that fail argument validation return before touching the device."""
    lib = P.load_library()
    assert lib.aroam_model_query(None, None) == -1
    assert "NULL" in P.aroam_last_error()
    assert lib.aroam_forward(None, 1, None, None, None) == -1
    assert lib.aroam_solve_lsqr(None, None, None, None, None, None) == -1
    assert lib.aroam_server_set_large(None, 1.0, 0) == -1
    assert lib.aroam_server_held(None, None, None) == -1
    assert "NULL" in P.aroam_last_error()
    lib.aroam_model_destroy(None)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setenv("AROAM_LIB", str(tmp_path / "nope.so"))
    monkeypatch.setattr(P.binding, "_LIB", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        P.binding.load_library()


def test_filtered_build_rejects_bad_filters_without_gpu():
    import workloads as W
    lib = P.load_library()
    cfg = W.config("tiny")
    sen, g = P.binding._sensor(cfg["sensor"]), P.binding._grid(cfg["grid"])
    h = ctypes.c_void_p()
    for f in [(80e6, 0.5e6, 32), (0.5e6, 200e6, 32), (-1.0, 80e6, 32), (0.5e6, 80e6, -1),
              (0.5e6, 80e6, 128)]:                  # 128 >= nt of the tiny grid
        filt = P.binding.Filter(*f)
        assert lib.aroam_build_model_filtered(ctypes.byref(sen), ctypes.byref(g),
                                              ctypes.byref(filt), 0, None, ctypes.byref(h)) == -1
        assert not h.value
    assert lib.aroam_build_model_filtered(ctypes.byref(sen), ctypes.byref(g), None, 0, None,
                                          ctypes.byref(h)) == -1
    assert lib.aroam_filter_signals(None, 1, None, None, None) == -1


def test_build_rejects_bad_discretisation_without_gpu():
    import workloads as W
    lib = P.load_library()
    cfg = W.config("tiny")
    sen = P.binding._sensor(cfg["sensor"])
    h = ctypes.c_void_p()
    for bad in (dict(voxel_basis=2), dict(time_derivative=-1), dict(basis_quad=9)):
        g = P.binding._grid(dict(cfg["grid"], **bad))
        assert lib.aroam_build_model(ctypes.byref(sen), ctypes.byref(g), 0, None,
                                     ctypes.byref(h)) == -1
        assert not h.value


def test_batch_rejects_fp64_without_gpu():
    """The batch's vectors are FP32, so an FP64 batch (which would read and write doubles) is
    rejected before anything is looked at or enqueued, for any n; FP32 with n = 0 succeeds."""
    lib = P.load_library()
    for fn in (lib.aroam_forward_batch, lib.aroam_adjoint_batch):
        assert fn(0, None, P.AROAM_FP64, None, None, None) == -1
        assert "FP32, BF16 or FP8" in P.aroam_last_error()
        assert fn(0, None, 7, None, None, None) == -1
        assert fn(0, None, P.AROAM_FP32, None, None, None) == 0


def test_k_half_limit_is_the_lds_stage_limit(tmp_path):
    """The largest k_half the header allows is the largest whose staged row ring (9 rows x
    (32 + 2 k_half) columns x 80 bytes) fits the 160 KiB LDS of a compute unit; the build
    rejects one more before any device call."""
    src = tmp_path / "k.cc"
    src.write_text('#include <cstdio>\n#include "aroam.h"\n#include "staging.h"\n'
                   "int main() { std::printf(\"%d %d %lld %lld %lld\\n\", AROAM_MAX_K_HALF, "
                   "aroam::max_k_half(), aroam::staged_lds_bytes(AROAM_MAX_K_HALF), "
                   "aroam::staged_lds_bytes(AROAM_MAX_K_HALF + 1), aroam::kLdsBytes); }\n")
    exe = tmp_path / "k"
    subprocess.run(["g++", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I",
                    os.path.join(ROOT, "paper_2009_10173_amd", "csrc"), str(src), "-o", str(exe)],
                   check=True)
    kmax, kcalc, lds, lds_next, cap = map(int, subprocess.run(
        [str(exe)], check=True, capture_output=True, text=True).stdout.split())
    assert kmax == kcalc
    assert cap == 160 * 1024
    assert lds == 9 * (32 + 2 * kmax) * 80 <= cap < lds_next
    import workloads as W
    lib = P.load_library()
    cfg = W.config("tiny")
    sen = P.binding._sensor(cfg["sensor"])
    h = ctypes.c_void_p()
    g = P.binding._grid(dict(cfg["grid"], k_half=kmax + 1))
    assert lib.aroam_build_model(ctypes.byref(sen), ctypes.byref(g), 0, None, ctypes.byref(h)) == -1
    assert "k_half" in P.aroam_last_error() and not h.value
    H = __import__("numpy").zeros(1)
    assert lib.aroam_import_model(ctypes.byref(g), H.ctypes.data_as(ctypes.c_void_p), None, None,
                                  0, None, ctypes.byref(h)) == -1
