// C ABI entry points (declared and documented in include/aroam.h).
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <vector>

#include "internal.h"

namespace aroam {

namespace {
thread_local char g_err[512] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = 0; }

int pool_alloc(void** p, size_t bytes, hipStream_t st) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static hipMemPool_t pools[kMaxDevices] = {};
  int dev = 0;
  AROAM_HIP(hipGetDevice(&dev));
  AROAM_CHECK(dev >= 0 && dev < kMaxDevices, AROAM_EDEVICE, "device %d out of range", dev);
  hipMemPool_t pool = nullptr;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (!pools[dev]) {
      hipMemPoolProps props = {};
      props.allocType = hipMemAllocationTypePinned;
      props.handleTypes = hipMemHandleTypeNone;
      props.location.type = hipMemLocationTypeDevice;
      props.location.id = dev;
      hipMemPool_t created = nullptr;
      AROAM_HIP(hipMemPoolCreate(&created, &props));
      uint64_t keep = UINT64_MAX;  // keep every freed block for reuse
      AROAM_HIP(hipMemPoolSetAttribute(created, hipMemPoolAttrReleaseThreshold, &keep));
      pools[dev] = created;
    }
    pool = pools[dev];
  }
  AROAM_HIP(hipMallocFromPoolAsync(p, bytes, pool, st));
  return AROAM_OK;
}

}  // namespace aroam

struct aroam_model {
  aroam::Model* m;
};

using aroam::Model;

namespace {

int build_handle(const aroam_sensor* sensor, const aroam_grid* grid, const aroam_filter* filter,
                 unsigned dtype_mask, void* stream, aroam_model** out) {
  aroam::clear_error();
  if (!out) {
    aroam::set_error("NULL output handle");
    return AROAM_EINVAL;
  }
  *out = nullptr;
  Model* m = nullptr;
  int rc = aroam::build_model(sensor, grid, filter, dtype_mask, (hipStream_t)stream, &m);
  if (rc != AROAM_OK) return rc;
  aroam_model* h = new (std::nothrow) aroam_model{m};
  if (!h) {
    aroam::destroy_model(m);
    aroam::set_error("host allocation failed");
    return AROAM_ENOMEM;
  }
  *out = h;
  return AROAM_OK;
}

}  // namespace

extern "C" {


int aroam_build_model(const aroam_sensor* sensor, const aroam_grid* grid, unsigned dtype_mask,
                      void* stream, aroam_model** out) {
  return build_handle(sensor, grid, nullptr, dtype_mask, stream, out);
}

int aroam_build_model_filtered(const aroam_sensor* sensor, const aroam_grid* grid,
                               const aroam_filter* filter, unsigned dtype_mask, void* stream,
                               aroam_model** out) {
  if (!filter) {
    aroam::clear_error();
    aroam::set_error("NULL filter");
    return AROAM_EINVAL;
  }
  return build_handle(sensor, grid, filter, dtype_mask, stream, out);
}

int aroam_filter_signals(const aroam_model* model, int dtype, const void* s_in, void* s_out,
                         void* stream) {
  aroam::clear_error();
  if (!model) {
    aroam::set_error("NULL model");
    return AROAM_EINVAL;
  }
  return aroam::filter_signals(*model->m, dtype, s_in, s_out, (hipStream_t)stream);
}

int aroam_import_model(const aroam_grid* grid, const double* dense, const int* col_lo,
                       const int* col_hi, unsigned dtype_mask, void* stream, aroam_model** out) {
  aroam::clear_error();
  if (!out) {
    aroam::set_error("NULL output handle");
    return AROAM_EINVAL;
  }
  *out = nullptr;
  Model* m = nullptr;
  int rc = aroam::import_model(grid, dense, col_lo, col_hi, dtype_mask, (hipStream_t)stream, &m);
  if (rc != AROAM_OK) return rc;
  aroam_model* h = new (std::nothrow) aroam_model{m};
  if (!h) {
    aroam::destroy_model(m);
    aroam::set_error("host allocation failed");
    return AROAM_ENOMEM;
  }
  *out = h;
  return AROAM_OK;
}

int aroam_model_query(const aroam_model* model, aroam_model_info* info) {
  aroam::clear_error();
  if (!model || !info) {
    aroam::set_error("NULL argument to aroam_model_query");
    return AROAM_EINVAL;
  }
  const Model& m = *model->m;
  info->n_columns = m.n_columns;
  info->nnz = m.nnz;
  info->mac_alg = m.mac_alg;
  for (int d = 0; d < 4; ++d) {
    const bool packed = (m.dtype_mask >> d) & 1u;
    info->mac_exec[d] = packed ? aroam::layout_for(m, false, d).mac_exec : 0;
    info->mac_exec_adj[d] = packed ? aroam::layout_for(m, true, d).mac_exec : 0;
  }
  info->device_bytes = m.device_bytes;
  info->n_elements = m.M;
  info->dtype_mask = m.dtype_mask;
  info->stored_columns = m.n_stored;
  info->stored_nnz = m.nnz_stored;
  for (int d = 0; d < 4; ++d) {
    const bool packed = (m.dtype_mask >> d) & 1u;
    const aroam::Layout& f = aroam::layout_for(m, false, d);
    const aroam::Layout& a = aroam::layout_for(m, true, d);
    info->row_tiles[d] = packed ? f.n_tiles : 0;
    info->row_tiles_adj[d] = packed ? a.n_tiles : 0;
    info->pieces[d] = packed ? (f.staged ? f.n_pieces : f.n_tiles) : 0;
    info->pieces_adj[d] = packed ? (a.staged ? a.n_pieces : a.n_tiles) : 0;
  }
  return AROAM_OK;
}

int aroam_model_export_table(const aroam_model* model, double* dense, int* col_lo, int* col_hi) {
  aroam::clear_error();
  if (!model) {
    aroam::set_error("NULL model");
    return AROAM_EINVAL;
  }
  const Model& m = *model->m;
  const int nz = m.grid.nz, nt = m.grid.nt;
  const size_t ncol = (size_t)m.n_off * nz;
  if (col_lo)
    for (size_t i = 0; i < ncol; ++i) col_lo[i] = m.h_lo[i];
  if (col_hi)
    for (size_t i = 0; i < ncol; ++i) col_hi[i] = m.h_hi[i];
  if (dense) {
    std::vector<double> band((size_t)std::max<long long>(1, m.nnz_stored));
    if (m.nnz_stored > 0 &&
        hipMemcpy(band.data(), m.d_band, m.nnz_stored * sizeof(double), hipMemcpyDeviceToHost) !=
            hipSuccess) {
      aroam::set_error("table download failed");
      return AROAM_EDEVICE;
    }
    for (size_t i = 0; i < ncol * nt; ++i) dense[i] = 0.0;
    for (size_t key = 0; key < ncol; ++key) {
      const int c = m.h_colidx[key];
      if (c < 0) continue;
      const long long o = m.h_off[c], len = m.h_off[c + 1] - o;
      double* dst = dense + key * nt + m.h_lo[key];
      for (long long i = 0; i < len; ++i) dst[i] = band[o + i];
    }
  }
  return AROAM_OK;
}

int aroam_model_export_quantized(const aroam_model* model, int dtype, int adjoint, double* dense,
                                 float* block_scales) {
  aroam::clear_error();
  if (!model) {
    aroam::set_error("NULL model");
    return AROAM_EINVAL;
  }
  return aroam::export_quantized(*model->m, dtype, adjoint != 0, dense, block_scales);
}

int aroam_forward(const aroam_model* model, int dtype, const void* x, void* s, void* stream) {
  aroam::clear_error();
  if (!model) {
    aroam::set_error("NULL model");
    return AROAM_EINVAL;
  }
  return aroam::apply(*model->m, false, dtype, x, s, nullptr, (hipStream_t)stream);
}

int aroam_forward_noalloc(const aroam_model* model, int dtype, const void* x, void* s,
                          void* stream) {
  aroam::clear_error();
  if (!model) {
    aroam::set_error("NULL model");
    return AROAM_EINVAL;
  }
  return aroam::apply_noalloc(*model->m, false, dtype, x, s, (hipStream_t)stream);
}

int aroam_adjoint(const aroam_model* model, int dtype, const void* s, void* x, void* stream) {
  aroam::clear_error();
  if (!model) {
    aroam::set_error("NULL model");
    return AROAM_EINVAL;
  }
  return aroam::apply(*model->m, true, dtype, s, x, nullptr, (hipStream_t)stream);
}

int aroam_solve_lsqr(const aroam_model* model, const aroam_solve_opts* opts, const void* s,
                     void* x, aroam_solve_info* info, void* stream) {
  aroam::clear_error();
  if (!model || !opts) {
    aroam::set_error("NULL model or options");
    return AROAM_EINVAL;
  }
  return aroam::solve_lsqr(*model->m, *opts, s, x, info, (hipStream_t)stream);
}

int aroam_solve_l1(const aroam_model* model, const aroam_solve_opts* opts, const void* s, void* x,
                   aroam_solve_info* info, void* stream) {
  aroam::clear_error();
  if (!model || !opts) {
    aroam::set_error("NULL model or options");
    return AROAM_EINVAL;
  }
  return aroam::solve_l1(*model->m, *opts, s, x, info, (hipStream_t)stream);
}

static int batch(int n, const aroam_model* const* models, bool adjoint, int dtype,
                 const float* const* in, float* const* out, void* stream) {
  aroam::clear_error();
  // the batch's vectors are FP32, so FP64 (double vectors) is not a batch dtype
  if (dtype != AROAM_FP32 && dtype != AROAM_BF16 && dtype != AROAM_FP8E4M3) {
    aroam::set_error("batched applies take FP32, BF16 or FP8 (dtype %d)", dtype);
    return AROAM_EINVAL;
  }
  if (n < 0 || (n > 0 && (!models || !in || !out))) {
    aroam::set_error("bad batch arguments");
    return AROAM_EINVAL;
  }
  std::vector<const Model*> ms(n);
  for (int i = 0; i < n; ++i) {
    if (!models[i]) {
      aroam::set_error("NULL model in batch entry %d", i);
      return AROAM_EINVAL;
    }
    ms[i] = models[i]->m;
  }
  return aroam::apply_batch(n, ms.data(), adjoint, dtype, in, out, (hipStream_t)stream);
}

int aroam_forward_batch(int n, const aroam_model* const* models, int dtype, const float* const* x,
                        float* const* s, void* stream) {
  return batch(n, models, false, dtype, x, s, stream);
}

int aroam_adjoint_batch(int n, const aroam_model* const* models, int dtype, const float* const* s,
                        float* const* x, void* stream) {
  return batch(n, models, true, dtype, s, x, stream);
}

int aroam_solve_footprint(const aroam_model* model, int kind, const aroam_solve_opts* opts,
                          size_t* bytes) {
  aroam::clear_error();
  if (!model || !opts || !bytes || (kind != 0 && kind != 1)) {
    aroam::set_error("bad arguments to aroam_solve_footprint");
    return AROAM_EINVAL;
  }
  *bytes = aroam::solver_footprint(*model->m, kind, *opts);
  return AROAM_OK;
}

struct aroam_server {
  aroam::Server* s;
};

int aroam_server_create(size_t hbm_budget_bytes, int max_slots, int tick_iters,
                        aroam_server** out) {
  aroam::clear_error();
  if (!out) {
    aroam::set_error("NULL output handle");
    return AROAM_EINVAL;
  }
  *out = nullptr;
  aroam::Server* s = nullptr;
  const int rc = aroam::server_create(hbm_budget_bytes, max_slots, tick_iters, &s);
  if (rc != AROAM_OK) return rc;
  *out = new (std::nothrow) aroam_server{s};
  if (!*out) {
    aroam::server_destroy(s);
    aroam::set_error("host allocation failed");
    return AROAM_ENOMEM;
  }
  return AROAM_OK;
}

int aroam_server_set_large(aroam_server* server, double large_macs, int large_alone) {
  aroam::clear_error();
  if (!server) {
    aroam::set_error("NULL server");
    return AROAM_EINVAL;
  }
  return aroam::server_set_large(*server->s, large_macs, large_alone);
}

int aroam_server_held(const aroam_server* server, long long* by_budget, long long* by_large) {
  aroam::clear_error();
  if (!server) {
    aroam::set_error("NULL server");
    return AROAM_EINVAL;
  }
  return aroam::server_held(*server->s, by_budget, by_large);
}

int aroam_server_submit(aroam_server* server, const aroam_model* model, int kind,
                        const aroam_solve_opts* opts, const void* s, void* x, long long* id) {
  aroam::clear_error();
  if (!server || !model || !opts) {
    aroam::set_error("NULL argument to aroam_server_submit");
    return AROAM_EINVAL;
  }
  return aroam::server_submit(*server->s, *model->m, kind, *opts, s, x, id);
}

int aroam_server_poll(aroam_server* server, int* n_resident, int* n_queued) {
  aroam::clear_error();
  if (!server) {
    aroam::set_error("NULL server");
    return AROAM_EINVAL;
  }
  return aroam::server_poll(*server->s, n_resident, n_queued);
}

int aroam_server_collect(aroam_server* server, int max, long long* ids, aroam_solve_info* infos,
                         int* n) {
  aroam::clear_error();
  if (!server) {
    aroam::set_error("NULL server");
    return AROAM_EINVAL;
  }
  return aroam::server_collect(*server->s, max, ids, infos, n);
}

void aroam_server_destroy(aroam_server* server) {
  if (!server) return;
  aroam::server_destroy(server->s);
  delete server;
}

void aroam_model_destroy(aroam_model* model) {
  if (!model) return;
  aroam::destroy_model(model->m);
  delete model;
}

const char* aroam_last_error(void) { return aroam::g_err; }

}  // extern "C"
