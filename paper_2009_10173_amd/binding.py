"""ctypes binding of libaroam.so: argument marshalling only.

Functions named `aroam_*` mirror the C entry points of include/aroam.h one to one.  Vectors
are torch tensors on the GPU (their data pointers are passed through); streams are torch
CUDA (HIP) streams.  Every call raises `AroamError` on a non-zero status.  There is no CPU
fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))

AROAM_FP64, AROAM_FP32, AROAM_BF16, AROAM_FP8E4M3 = 0, 1, 2, 3
DTYPES = {"fp64": AROAM_FP64, "fp32": AROAM_FP32, "bf16": AROAM_BF16, "fp8": AROAM_FP8E4M3}
STATUS = {0: "AROAM_OK", -1: "AROAM_EINVAL", -2: "AROAM_ENOMEM", -3: "AROAM_EDEVICE",
          -4: "AROAM_ENONFINITE", -5: "AROAM_EUNSUPPORTED"}


class AroamError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Sensor(C.Structure):
    _fields_ = [("radius_m", C.c_double), ("aperture_m", C.c_double), ("hole_m", C.c_double),
                ("n_rings", C.c_int), ("f0_hz", C.c_double), ("frac_bw", C.c_double)]


class Grid(C.Structure):
    _fields_ = [("c_mps", C.c_double), ("fs_hz", C.c_double), ("nx", C.c_int), ("ny", C.c_int),
                ("step_m", C.c_double), ("nz", C.c_int), ("dz_m", C.c_double), ("nt", C.c_int),
                ("k_half", C.c_int), ("footprint_mode", C.c_int), ("voxel_basis", C.c_int),
                ("time_derivative", C.c_int), ("basis_quad", C.c_int)]


class Filter(C.Structure):
    _fields_ = [("f_lo_hz", C.c_double), ("f_hi_hz", C.c_double), ("half_taps", C.c_int)]


class ModelInfo(C.Structure):
    _fields_ = [("n_columns", C.c_longlong), ("nnz", C.c_longlong), ("mac_alg", C.c_longlong),
                ("mac_exec", C.c_longlong * 4), ("mac_exec_adj", C.c_longlong * 4),
                ("device_bytes", C.c_size_t), ("n_elements", C.c_int),
                ("dtype_mask", C.c_uint), ("stored_columns", C.c_longlong),
                ("stored_nnz", C.c_longlong), ("row_tiles", C.c_int * 4),
                ("row_tiles_adj", C.c_int * 4), ("pieces", C.c_int * 4),
                ("pieces_adj", C.c_int * 4)]


class SolveOpts(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("iters", C.c_int), ("refine_sweeps", C.c_int),
                ("anchor_period", C.c_int), ("power_iters", C.c_int), ("lipschitz", C.c_double),
                ("inner", C.c_int), ("outer", C.c_int), ("anchor_warmup", C.c_int),
                ("power_start", C.c_void_p)]


class SolveInfo(C.Structure):
    _fields_ = [("iters_done", C.c_int), ("status", C.c_int), ("lambda_", C.c_double),
                ("lipschitz", C.c_double), ("rnorm", C.c_double), ("alpha", C.c_double),
                ("beta", C.c_double)]


_LIB = None
_SYMBOLS = {
    "aroam_build_model": ([C.POINTER(Sensor), C.POINTER(Grid), C.c_uint, C.c_void_p,
                           C.POINTER(C.c_void_p)], C.c_int),
    "aroam_build_model_filtered": ([C.POINTER(Sensor), C.POINTER(Grid), C.POINTER(Filter),
                                    C.c_uint, C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "aroam_filter_signals": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p],
                             C.c_int),
    "aroam_import_model": ([C.POINTER(Grid), C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint,
                            C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "aroam_model_query": ([C.c_void_p, C.POINTER(ModelInfo)], C.c_int),
    "aroam_model_export_table": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "aroam_model_export_quantized": ([C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p],
                                     C.c_int),
    "aroam_forward": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "aroam_forward_noalloc": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p],
                              C.c_int),
    "aroam_adjoint": ([C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "aroam_solve_lsqr": ([C.c_void_p, C.POINTER(SolveOpts), C.c_void_p, C.c_void_p,
                          C.POINTER(SolveInfo), C.c_void_p], C.c_int),
    "aroam_solve_l1": ([C.c_void_p, C.POINTER(SolveOpts), C.c_void_p, C.c_void_p,
                        C.POINTER(SolveInfo), C.c_void_p], C.c_int),
    "aroam_forward_batch": ([C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p],
                            C.c_int),
    "aroam_adjoint_batch": ([C.c_int, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p],
                            C.c_int),
    "aroam_model_destroy": ([C.c_void_p], None),
    "aroam_solve_footprint": ([C.c_void_p, C.c_int, C.POINTER(SolveOpts),
                               C.POINTER(C.c_size_t)], C.c_int),
    "aroam_server_create": ([C.c_size_t, C.c_int, C.c_int, C.POINTER(C.c_void_p)], C.c_int),
    "aroam_server_set_large": ([C.c_void_p, C.c_double, C.c_int], C.c_int),
    "aroam_server_held": ([C.c_void_p, C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)],
                          C.c_int),
    "aroam_server_submit": ([C.c_void_p, C.c_void_p, C.c_int, C.POINTER(SolveOpts), C.c_void_p,
                             C.c_void_p, C.POINTER(C.c_longlong)], C.c_int),
    "aroam_server_poll": ([C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)], C.c_int),
    "aroam_server_collect": ([C.c_void_p, C.c_int, C.POINTER(C.c_longlong),
                              C.POINTER(SolveInfo), C.POINTER(C.c_int)], C.c_int),
    "aroam_server_destroy": ([C.c_void_p], None),
    "aroam_last_error": ([], C.c_char_p),
}


def library_path():
    return os.environ.get("AROAM_LIB", os.path.join(PKG, "libaroam.so"))


def load_library():
    """Load libaroam.so (built by `python -m paper_2009_10173_amd.build`).

    PyTorch's HIP runtime is brought up first, so that the library and the tensors it works
    on share one runtime in the process (the library's HIP dependency then resolves to the
    runtime already loaded)."""
    global _LIB
    if _LIB is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build the HIP library first "
                               "(python -m paper_2009_10173_amd.build); there is no fallback")
        try:
            import torch
            torch.cuda.is_available()
        except ImportError:
            pass
        lib = C.CDLL(path)
        for name, (args, res) in _SYMBOLS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _LIB = lib
    return _LIB


def _check(rc):
    if rc != 0:
        raise AroamError(rc, aroam_last_error())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _sensor(d):
    return Sensor(d["radius_m"], d["aperture_m"], d.get("hole_m", 0.0), int(d.get("n_rings", 0)),
                  d["f0_hz"], d["frac_bw"])


def _grid(d):
    return Grid(d["c_mps"], d["fs_hz"], d["nx"], d["ny"], d["step_m"], d["nz"], d["dz_m"],
                d["nt"], d["k_half"], d["footprint_mode"], int(d.get("voxel_basis", 0)),
                int(d.get("time_derivative", 0)), int(d.get("basis_quad", 0)))


# --- one function per C entry point ---------------------------------------------------------

def aroam_last_error():
    return load_library().aroam_last_error().decode(errors="replace")


def aroam_build_model(sensor, grid, dtype_mask, stream=None):
    h = C.c_void_p()
    _check(load_library().aroam_build_model(C.byref(_sensor(sensor)), C.byref(_grid(grid)),
                                            dtype_mask, _stream(stream), C.byref(h)))
    return h


def _filter(f):
    return Filter(float(f["f_lo_hz"]), float(f["f_hi_hz"]), int(f["half_taps"]))


def aroam_build_model_filtered(sensor, grid, filt, dtype_mask, stream=None):
    h = C.c_void_p()
    _check(load_library().aroam_build_model_filtered(
        C.byref(_sensor(sensor)), C.byref(_grid(grid)), C.byref(_filter(filt)), dtype_mask,
        _stream(stream), C.byref(h)))
    return h


def aroam_filter_signals(h, dtype, s_in, s_out, stream=None):
    _check(load_library().aroam_filter_signals(h, dtype, _ptr(s_in), _ptr(s_out),
                                               _stream(stream)))


def aroam_import_model(grid, dense, col_lo=None, col_hi=None, dtype_mask=0, stream=None):
    """dense: host float64 array [2K+1][2K+1][nz][nt]; col_lo / col_hi: int32 [2K+1][2K+1][nz]
    or None.  Returns the model handle."""
    import numpy as np
    K, nz, nt = grid["k_half"], grid["nz"], grid["nt"]
    W = 2 * K + 1
    H = np.ascontiguousarray(dense, dtype=np.float64)
    if H.shape != (W, W, nz, nt):
        raise ValueError(f"table shape {H.shape} != {(W, W, nz, nt)}")
    lo = hi = None
    if col_lo is not None or col_hi is not None:
        lo = np.ascontiguousarray(col_lo, dtype=np.int32)
        hi = np.ascontiguousarray(col_hi, dtype=np.int32)
        if lo.shape != (W, W, nz) or hi.shape != (W, W, nz):
            raise ValueError("window arrays must have shape [2K+1][2K+1][nz]")
    h = C.c_void_p()
    _check(load_library().aroam_import_model(
        C.byref(_grid(grid)), H.ctypes.data_as(C.c_void_p),
        None if lo is None else lo.ctypes.data_as(C.c_void_p),
        None if hi is None else hi.ctypes.data_as(C.c_void_p), dtype_mask, _stream(stream),
        C.byref(h)))
    return h


def aroam_model_query(h):
    info = ModelInfo()
    _check(load_library().aroam_model_query(h, C.byref(info)))
    return dict(n_columns=info.n_columns, nnz=info.nnz, mac_alg=info.mac_alg,
                mac_exec=list(info.mac_exec), mac_exec_adj=list(info.mac_exec_adj),
                device_bytes=info.device_bytes, n_elements=info.n_elements,
                dtype_mask=info.dtype_mask, stored_columns=info.stored_columns,
                stored_nnz=info.stored_nnz, row_tiles=list(info.row_tiles),
                row_tiles_adj=list(info.row_tiles_adj), pieces=list(info.pieces),
                pieces_adj=list(info.pieces_adj))


def aroam_model_export_table(h, grid, dense=True):
    """Returns (H [2K+1][2K+1][nz][nt] float64 or None, col_lo, col_hi) as numpy arrays."""
    import numpy as np
    K, nz, nt = grid["k_half"], grid["nz"], grid["nt"]
    W = 2 * K + 1
    lo = np.empty((W, W, nz), dtype=np.int32)
    hi = np.empty((W, W, nz), dtype=np.int32)
    H = np.empty((W, W, nz, nt), dtype=np.float64) if dense else None
    _check(load_library().aroam_model_export_table(
        h, H.ctypes.data_as(C.c_void_p) if dense else None, lo.ctypes.data_as(C.c_void_p),
        hi.ctypes.data_as(C.c_void_p)))
    return H, lo, hi


def aroam_model_export_quantized(h, grid, dtype, adjoint=False):
    """Returns (H [2K+1][2K+1][nz][nt] float64 of the values the dtype's apply multiplies,
    block scales [2K+1][2K+1][ceil(nz/16)] float32 for FP8 else None)."""
    import numpy as np
    K, nz, nt = grid["k_half"], grid["nz"], grid["nt"]
    W = 2 * K + 1
    dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    H = np.empty((W, W, nz, nt), dtype=np.float64)
    sc = np.empty((W, W, (nz + 15) // 16), dtype=np.float32) if dtype == AROAM_FP8E4M3 else None
    _check(load_library().aroam_model_export_quantized(
        h, dtype, int(bool(adjoint)), H.ctypes.data_as(C.c_void_p),
        None if sc is None else sc.ctypes.data_as(C.c_void_p)))
    return H, sc


def aroam_forward(h, dtype, x, s, stream=None):
    _check(load_library().aroam_forward(h, dtype, _ptr(x), _ptr(s), _stream(stream)))


def aroam_forward_noalloc(h, dtype, x, s, stream=None):
    _check(load_library().aroam_forward_noalloc(h, dtype, _ptr(x), _ptr(s), _stream(stream)))


def aroam_adjoint(h, dtype, s, x, stream=None):
    _check(load_library().aroam_adjoint(h, dtype, _ptr(s), _ptr(x), _stream(stream)))


def _opts(lam, iters, refine_sweeps=0, anchor_period=0, power_iters=0, lipschitz=0.0,
          inner=AROAM_FP32, outer=None, anchor_warmup=-1, power_start=None):
    return SolveOpts(float(lam), int(iters), int(refine_sweeps), int(anchor_period),
                     int(power_iters), float(lipschitz), int(inner),
                     int(inner if outer is None else outer), int(anchor_warmup),
                     _ptr(power_start))


def _info(i):
    return dict(iters_done=i.iters_done, status=i.status, lam=i.lambda_, lipschitz=i.lipschitz,
                rnorm=i.rnorm, alpha=i.alpha, beta=i.beta)


def aroam_solve_lsqr(h, s, x, stream=None, **opts):
    info = SolveInfo()
    _check(load_library().aroam_solve_lsqr(h, C.byref(_opts(**opts)), _ptr(s), _ptr(x),
                                           C.byref(info), _stream(stream)))
    return _info(info)


def aroam_solve_l1(h, s, x, stream=None, **opts):
    info = SolveInfo()
    _check(load_library().aroam_solve_l1(h, C.byref(_opts(**opts)), _ptr(s), _ptr(x),
                                         C.byref(info), _stream(stream)))
    return _info(info)


def _batch(fn, hs, dtype, ins, outs, stream):
    n = len(hs)
    harr = (C.c_void_p * n)(*[h.value for h in hs])
    iarr = (C.c_void_p * n)(*[t.data_ptr() for t in ins])
    oarr = (C.c_void_p * n)(*[t.data_ptr() for t in outs])
    _check(fn(n, harr, dtype, iarr, oarr, _stream(stream)))


def aroam_forward_batch(hs, dtype, xs, ss, stream=None):
    _batch(load_library().aroam_forward_batch, hs, dtype, xs, ss, stream)


def aroam_adjoint_batch(hs, dtype, ss, xs, stream=None):
    _batch(load_library().aroam_adjoint_batch, hs, dtype, ss, xs, stream)


def aroam_model_destroy(h):
    if h is not None and h.value:
        load_library().aroam_model_destroy(h)


def aroam_solve_footprint(h, kind, **opts):
    b = C.c_size_t()
    _check(load_library().aroam_solve_footprint(h, int(kind), C.byref(_opts(**opts)), C.byref(b)))
    return b.value


def aroam_server_create(hbm_budget_bytes, max_slots=8, tick_iters=2):
    h = C.c_void_p()
    _check(load_library().aroam_server_create(int(hbm_budget_bytes), int(max_slots),
                                              int(tick_iters), C.byref(h)))
    return h


def aroam_server_set_large(server, large_macs, large_alone=False):
    _check(load_library().aroam_server_set_large(server, float(large_macs), int(bool(large_alone))))


def aroam_server_held(server):
    """(polls held by the budget, polls held by the large-request policy)."""
    b, l = C.c_longlong(), C.c_longlong()
    _check(load_library().aroam_server_held(server, C.byref(b), C.byref(l)))
    return b.value, l.value


def aroam_server_submit(server, model_h, kind, s, x, **opts):
    """Queue one reconstruction (kind 0 = LSQR, 1 = FISTA); s and x must stay alive until the
    request is collected.  Returns the request id."""
    rid = C.c_longlong()
    _check(load_library().aroam_server_submit(server, model_h, int(kind), C.byref(_opts(**opts)),
                                              _ptr(s), _ptr(x), C.byref(rid)))
    return rid.value


def aroam_server_poll(server):
    nr, nq = C.c_int(), C.c_int()
    _check(load_library().aroam_server_poll(server, C.byref(nr), C.byref(nq)))
    return nr.value, nq.value


def aroam_server_collect(server, max_n=256):
    ids = (C.c_longlong * max_n)()
    infos = (SolveInfo * max_n)()
    n = C.c_int()
    _check(load_library().aroam_server_collect(server, max_n, ids, infos, C.byref(n)))
    return [(ids[i], _info(infos[i])) for i in range(n.value)]


def aroam_server_destroy(server):
    if server is not None and server.value:
        load_library().aroam_server_destroy(server)


# --- convenience wrapper -----------------------------------------------------------------

def _mask(dtypes):
    mask = 0
    for d in dtypes:
        mask |= 1 << (DTYPES[d] if isinstance(d, str) else int(d))
    return mask


class Model:
    """A built model (device-resident tables) plus its grid; frees itself on close()."""

    def __init__(self, sensor, grid, dtypes=("fp64", "fp32"), stream=None, filter=None,
                 _handle=None):
        self.sensor, self.grid = (None if sensor is None else dict(sensor)), dict(grid)
        self.filter = None if filter is None else dict(filter)
        if _handle is not None:
            self.handle = _handle
        elif filter is None:
            self.handle = aroam_build_model(sensor, grid, _mask(dtypes), stream)
        else:
            self.handle = aroam_build_model_filtered(sensor, grid, filter, _mask(dtypes), stream)

    @classmethod
    def from_table(cls, grid, dense, col_lo=None, col_hi=None, dtypes=("fp64", "fp32"),
                   stream=None):
        """A model from a table given on the host (aroam_import_model)."""
        h = aroam_import_model(grid, dense, col_lo, col_hi, _mask(dtypes), stream)
        return cls(None, grid, _handle=h)

    def info(self):
        return aroam_model_query(self.handle)

    def export_table(self, dense=True):
        return aroam_model_export_table(self.handle, self.grid, dense)

    def export_quantized(self, dtype, adjoint=False):
        return aroam_model_export_quantized(self.handle, self.grid, dtype, adjoint)

    @property
    def image_shape(self):
        g = self.grid
        return (g["ny"], g["nx"], g["nz"])

    @property
    def signal_shape(self):
        g = self.grid
        return (g["ny"], g["nx"], g["nt"])

    def _vec_dtype(self, dtype):
        import torch
        return torch.float64 if dtype == AROAM_FP64 else torch.float32

    def forward(self, x, dtype=AROAM_FP32, out=None, stream=None):
        import torch
        dtype = DTYPES.get(dtype, dtype) if isinstance(dtype, str) else dtype
        if out is None:
            out = torch.empty(self.signal_shape, dtype=self._vec_dtype(dtype), device=x.device)
        _expect(x, self.image_shape, self._vec_dtype(dtype))
        _expect(out, self.signal_shape, self._vec_dtype(dtype))
        aroam_forward(self.handle, dtype, x, out, stream)
        return out

    def adjoint(self, s, dtype=AROAM_FP32, out=None, stream=None):
        import torch
        dtype = DTYPES.get(dtype, dtype) if isinstance(dtype, str) else dtype
        if out is None:
            out = torch.empty(self.image_shape, dtype=self._vec_dtype(dtype), device=s.device)
        _expect(s, self.signal_shape, self._vec_dtype(dtype))
        _expect(out, self.image_shape, self._vec_dtype(dtype))
        aroam_adjoint(self.handle, dtype, s, out, stream)
        return out

    def filter_signals(self, s, out=None, stream=None):
        """F s with the model's band-pass filter, in the tensor's precision (FP64 or FP32)."""
        import torch
        if s.dtype not in (torch.float64, torch.float32):
            raise ValueError(f"signals are filtered in float64 or float32, not {s.dtype}")
        d = AROAM_FP64 if s.dtype == torch.float64 else AROAM_FP32
        _expect(s, self.signal_shape, s.dtype)
        if out is None:
            out = torch.empty_like(s)
        aroam_filter_signals(self.handle, d, s, out, stream)
        return out

    def solve_lsqr(self, s, lam=-1.0, iters=50, inner="fp32", outer=None, refine_sweeps=0,
                   out=None, stream=None):
        import torch
        inner = DTYPES[inner] if isinstance(inner, str) else inner
        outer = inner if outer is None else (DTYPES[outer] if isinstance(outer, str) else outer)
        if out is None:
            out = torch.empty(self.image_shape, dtype=self._vec_dtype(inner), device=s.device)
        _expect(s, self.signal_shape, self._vec_dtype(inner))
        _expect(out, self.image_shape, self._vec_dtype(inner))
        info = aroam_solve_lsqr(self.handle, s, out, stream, lam=lam, iters=iters,
                                refine_sweeps=refine_sweeps, inner=inner, outer=outer)
        return out, info

    def solve_l1(self, s, lam=-1.0, iters=200, inner="fp32", outer=None, lipschitz=0.0,
                 power_iters=50, anchor_period=0, anchor_warmup=-1, power_start=None, out=None,
                 stream=None):
        import torch
        inner = DTYPES[inner] if isinstance(inner, str) else inner
        outer = inner if outer is None else (DTYPES[outer] if isinstance(outer, str) else outer)
        if out is None:
            out = torch.empty(self.image_shape, dtype=self._vec_dtype(inner), device=s.device)
        _expect(s, self.signal_shape, self._vec_dtype(inner))
        _expect(out, self.image_shape, self._vec_dtype(inner))
        if power_start is not None:
            _expect(power_start, self.image_shape, self._vec_dtype(inner))
        info = aroam_solve_l1(self.handle, s, out, stream, lam=lam, iters=iters,
                              lipschitz=lipschitz, power_iters=power_iters,
                              anchor_period=anchor_period, anchor_warmup=anchor_warmup,
                              inner=inner, outer=outer, power_start=power_start)
        return out, info

    def close(self):
        aroam_model_destroy(self.handle)
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _expect(t, shape, dtype):
    if tuple(t.shape) != tuple(shape) or t.dtype != dtype or not t.is_contiguous() \
            or not t.is_cuda:
        raise ValueError(f"expected a contiguous GPU tensor {tuple(shape)} {dtype}, got "
                         f"{tuple(t.shape)} {t.dtype} on {t.device}")
