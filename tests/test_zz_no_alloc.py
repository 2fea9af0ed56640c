"""The allocation-free forward (aroam_forward_noalloc, stage buffer in a static device array)
against aroam_forward through the C ABI: the same kernels, so the same result bit for bit, on
two calls in a row (the second on a smaller grid, so it reuses the array a larger call left
behind), and a clear error for an apply that needs more scratch than the array holds."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2009_10173_amd as P  # noqa: E402


def _raw(fn, m, dtype, x, s):
    lib = P.load_library()
    return getattr(lib, fn)(m.handle, P.DTYPES[dtype], ctypes.c_void_p(x.data_ptr()),
                            ctypes.c_void_p(s.data_ptr()), P.binding._stream(None))


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "bf16", "fp8"])
def test_noalloc_forward_equals_forward(dtype):
    dev = torch.device("cuda:0")
    tdt = torch.float64 if dtype == "fp64" else torch.float32
    models = []
    try:
        for name in ("mid", "tiny"):                   # the second grid is the smaller one
            cfg = W.config(name)
            print(f"[no-alloc forward {name} {dtype}]", flush=True)
            m = P.Model(cfg["sensor"], cfg["grid"], dtypes=("fp64", "fp32", "bf16", "fp8"))
            models.append(m)
            x = torch.from_numpy(W.random_image(cfg, 41)).to(dev, tdt)
            ref = torch.empty(m.signal_shape, device=dev, dtype=tdt)
            got = torch.full(m.signal_shape, float("nan"), device=dev, dtype=tdt)
            assert _raw("aroam_forward", m, dtype, x, ref) == 0
            assert _raw("aroam_forward_noalloc", m, dtype, x, got) == 0, P.aroam_last_error()
            torch.cuda.synchronize()
            assert torch.equal(got, ref), name
            assert torch.isfinite(got).all()
    finally:
        for m in models:
            m.close()


def test_noalloc_forward_rejects_an_apply_beyond_the_static_array():
    """A 600x600 scan with 64 depths stages 608 x 616 x 64 FP32 values (95.9 MB) for its
    forward, more than the 64 MiB array: AROAM_EINVAL with the size in the message, and the
    output is not touched."""
    dev = torch.device("cuda:0")
    cfg = W.config("tiny")
    g = dict(cfg["grid"], nx=600, ny=600, nz=64, nt=64)
    with P.Model(cfg["sensor"], g, dtypes=("fp32",)) as m:
        x = torch.zeros(m.image_shape, device=dev)
        s = torch.full(m.signal_shape, 7.0, device=dev)
        assert _raw("aroam_forward_noalloc", m, "fp32", x, s) == -1
        assert "static buffer" in P.aroam_last_error()
        torch.cuda.synchronize()
        assert bool((s == 7.0).all())
