"""MI355X-native model-based AR-OAM reconstruction (HIP kernels for gfx950 behind a C ABI).

The compute path lives in `libaroam.so` (built from `csrc/` by `build.py`); this package only
marshals arguments to it.  See `include/aroam.h` for the ABI.
"""
from .binding import (  # noqa: F401
    AROAM_BF16, AROAM_FP32, AROAM_FP64, AROAM_FP8E4M3, DTYPES, AroamError, Model, aroam_adjoint,
    aroam_adjoint_batch, aroam_build_model, aroam_build_model_filtered, aroam_filter_signals,
    aroam_forward, aroam_forward_batch, aroam_forward_noalloc, aroam_import_model,
    aroam_last_error, aroam_model_destroy, aroam_model_export_quantized, aroam_model_export_table,
    aroam_model_query,
    aroam_server_collect, aroam_server_create, aroam_server_destroy, aroam_server_poll,
    aroam_server_held, aroam_server_set_large, aroam_server_submit, aroam_solve_footprint, aroam_solve_l1, aroam_solve_lsqr, library_path,
    load_library)
