// Internal declarations of the AR-OAM HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "aroam.h"
#include "staging.h"

namespace aroam {

// ------------------------------------------------------------------------------------------
// Errors: a thread-local message plus the status code returned through the C ABI.
void set_error(const char* fmt, ...);
void clear_error();

// Stream-ordered temporaries of the library (stage buffers of single applies, solver state):
// one memory pool per device that keeps freed blocks for reuse (no release threshold), so
// repeated applies and solves do not hand memory back to the driver at every
// synchronisation.  The pools live until the process ends.  Free with hipFreeAsync.
int pool_alloc(void** p, size_t bytes, hipStream_t st);

#define AROAM_HIP(expr)                                                             \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::aroam::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),     \
                         __FILE__, __LINE__);                                       \
      return AROAM_EDEVICE;                                                         \
    }                                                                               \
  } while (0)

#define AROAM_CHECK(cond, code, ...)       \
  do {                                     \
    if (!(cond)) {                         \
      ::aroam::set_error(__VA_ARGS__);     \
      return (code);                       \
    }                                      \
  } while (0)

#define AROAM_TRY(expr)          \
  do {                           \
    int st_ = (expr);            \
    if (st_ != AROAM_OK) return st_; \
  } while (0)

constexpr int kTile = 16;     // output rows per tile (time samples or depths) = MFMA M
constexpr int kLaneGroups = 4; // K-groups per bundle = 64-lane wave / 16
constexpr int kTileRows8 = 32;  // output rows per tile of the G = 8 (BF16 / FP8) layouts
constexpr int kMaxElements = 4096;  // two FP64 values per sub-element fit in 64 KiB of LDS
static_assert(max_k_half() == AROAM_MAX_K_HALF, "the header's k_half limit is the LDS stage's");

// ------------------------------------------------------------------------------------------
// Padded operand geometry.  Inputs of an apply are staged into a zero-padded buffer
// [nyp][nxp][Lp] with a halo of K columns on every lateral side, x rounded up to whole
// 16-position tiles, and the fast axis padded so that every K-group read stays in bounds.
struct PadGeom {
  int K = 0, nx = 0, ny = 0;
  int ntx = 0;        // 16-position tiles per scan row
  int nxp = 0, nyp = 0;
  int L = 0, Lp = 0;  // true and padded length of the fast axis of the input
  long long elems() const { return (long long)nyp * nxp * Lp; }
};

// Staged layouts: bits kMetaMaskShift.. of each K-group's meta word hold its bundle's mask (the
// LDS offset stays below 2^kMetaMaskShift): with two row halves the halves its K-groups reach,
// with one (FP32, runs of 4) the entries of the runs, one MFMA each, that they reach.
constexpr int kMetaMaskShift = 28;

// Band tiles of one operator (forward: rows = time, K = (offset, depth); adjoint: rows =
// depth, K = (offset, time)) at one K-group width G.  A K-group is G consecutive entries of
// one table column block; four K-groups form a bundle, which one MFMA step consumes.
//
// Two forms:
//  * direct (staged == false): meta[q] is the element offset of K-group q's input run
//    relative to the output position, read straight from the padded input;
//  * LDS-staged (staged == true): each tile's bundles are grouped into stage units
//    (dy, chunk of CH inner entries).  A workgroup loads the input rows of its position patch
//    shifted by dy, for the chunk and the unit's dx range, into LDS once, and then sweeps all
//    (dx, G-run) K-groups of the unit from LDS; meta[q] is then the LDS element offset
//    (dx + K) * CS + (run start - chunk start), with the bundle's mask in the top bits.
struct Layout {
  int G = 0;
  int TM = 16;              // output rows per tile (16 or 32: two MFMA row halves)
  int n_tiles = 0;          // output row tiles
  int out_len = 0;          // rows of the output vector (nt or nz)
  long long n_bundles = 0;
  int* d_tile_start = nullptr;   // [n_tiles + 1] bundle range of each tile (direct form)
  int* d_meta = nullptr;         // [n_bundles * 4] per K-group offset (see above)
  int4* d_groups = nullptr;      // [n_bundles * 4] (offset index, start, tile, active)
  std::vector<int> h_tile_start;  // bundle (direct) or stage-unit (staged) range of each tile
  long long mac_exec = 0;        // MACs issued per apply
  PadGeom in;                    // staged input geometry
  // LDS-staged form
  bool staged = false;
  int CH = 0, BR = 0, BC = 0;    // chunk length, patch rows, patch columns
  int CS = 0, NCOL = 0;          // LDS column stride (elements), staged columns BC + 2K
  long long n_units = 0;
  int4* d_units = nullptr;       // [n_units] (dy, chunk start, bundle begin, bundle end)
  int2* d_ucols = nullptr;       // [n_units] padded input rows [lo, hi) the unit loads (ring)
  size_t lds_bytes = 0;
  // Work split of the staged kernel: a tile's stage units may be cut at chunk starts (where
  // the LDS ring is reloaded anyway) into pieces of similar work, so that the workgroups of a
  // launch are many and even, and the pieces may be dispatched heaviest first.  Each piece of a
  // cut tile leaves its partial sums in a slot of the stage buffer, and a second kernel adds
  // a tile's slots in slot order (deterministic).
  int n_pieces = 0;
  int n_slots = 0;               // partial slots (pieces of the tiles cut into several)
  int n_patches = 0;             // position patches of one launch
  int4* d_pieces = nullptr;      // [n_pieces] (tile, unit begin, unit end, slot or -1) in
                                 // dispatch order
  int2* d_tile_split = nullptr;  // [n_tiles] (pieces of the tile, its first slot)
};

struct Pack {
  void* d = nullptr;   // FP32 / BF16: [n_bundles * 4 * TM * G] elements; FP8: [n_bundles][half]
                       // [lane group][row][32] e4m3 bytes (see kFp8Lane)
  size_t bytes = 0;
};

// Operand positions of the FP8 bundles (v_mfma_scale_f32_16x16x128_f8f6f4, measured on
// gfx950): lane (n, g) holds 32 bytes, and the 128 K of one MFMA form four scale blocks of 32.
// Scale block b consists of the 8-byte slots kFp8Slot[b][i] of lane groups kFp8Lane[b][i]
// (i < 4), and takes the scale byte of lane group kFp8ScaleLane[b].
constexpr int kFp8Lane[4][4] = {{0, 0, 1, 1}, {2, 2, 3, 3}, {0, 0, 1, 1}, {2, 2, 3, 3}};
constexpr int kFp8Slot[4][4] = {{0, 1, 0, 1}, {0, 1, 0, 1}, {2, 3, 2, 3}, {2, 3, 2, 3}};
constexpr int kFp8ScaleLane[4] = {0, 1, 2, 3};

struct Model {
  aroam_sensor sensor{};
  aroam_grid grid{};
  int K = 0, n_off = 0;          // n_off = (2K+1)^2
  int M = 0;                     // sub-elements
  double R_mm = 0, cfs = 0;      // focal radius (mm), mm per sample
  double sigma = 0, omega = 0;   // EIR envelope (samples), carrier (rad/sample)
  double step_mm = 0, dz_mm = 0;
  long long n_columns = 0, nnz = 0, mac_alg = 0;  // over all footprint columns
  long long n_stored = 0, nnz_stored = 0;         // columns / band entries held on the device
  std::vector<int> h_lo, h_hi;   // [n_off][nz], -1 where inactive
  std::vector<long long> h_off;  // [n_stored + 1] band offsets of the stored columns
  std::vector<int> h_colidx;     // [n_off][nz] -> stored column index or -1
  // device tables
  double* d_band = nullptr;      // FP64 band values [nnz_stored]
  int* d_colidx = nullptr;       // [n_off][nz]
  int* d_lo = nullptr;           // [n_stored]
  long long* d_off = nullptr;    // [n_stored + 1]
  Layout g4f, g4a;               // direct form, G = 4: FP64 forward / adjoint
  Layout s4f, s4a;               // LDS-staged, G = 4: FP32
  Layout s8f, s8a;               // LDS-staged, G = 8: BF16
  Layout f8f, f8a;               // LDS-staged, G = 8, bundles of the block-scaled FP8 MFMA
  Pack fwd_pack[4], adj_pack[4]; // indexed by aroam_dtype
  // band-pass filter applied along time to the columns (and, by the caller, to the signals)
  bool filtered = false;
  aroam_filter filter{};
  int fir_L = 0;
  std::vector<double> fir_taps;  // h[-L..L]
  double* d_fir_taps = nullptr;  // h[-L..L]
  double* d_fir_pad64 = nullptr; // zero-padded taps for the signal kernel, FP64 and FP32
  float* d_fir_pad32 = nullptr;
  unsigned dtype_mask = 0;
  size_t device_bytes = 0;
  int device = 0;
};

// filter.hip
std::vector<double> fir_taps(const aroam_filter& f, double fs);
int check_filter(const aroam_filter& f, double fs, int nt);
int setup_filter(Model& m, const aroam_filter& f);
int filter_columns(const Model& m, const int* d_rlo, const long long* d_roff,
                   const double* d_raw, hipStream_t st);
int filter_signals(const Model& m, int dtype, const void* in, void* out, hipStream_t st);

// table.hip
int check_grid(const aroam_grid* g);
int finish_model(Model* m, int rc, unsigned mask, hipStream_t st, Model** out);
int import_model(const aroam_grid* g, const double* dense, const int* col_lo,
                 const int* col_hi, unsigned mask, hipStream_t st, Model** out);
int build_model(const aroam_sensor* s, const aroam_grid* g, const aroam_filter* f,
                unsigned mask, hipStream_t st, Model** out);
void destroy_model(Model* m);
// Host copy of the FP32 / BF16 / FP8 pack of one direction in the dense table layout, each
// entry the value that the dtype's apply multiplies (FP8: also the block scales).
int export_quantized(const Model& m, int dtype, bool adjoint, double* dense, float* scales);

// apply.hip
const Layout& layout_for(const Model& m, bool adjoint, int dtype);
size_t stage_bytes(const Model& m, bool adjoint, int dtype);
// Apply A (adjoint = false) or A^T.  `in`/`out` are caller vectors of the dtype's element
// type (double for FP64, float otherwise).  `stage` is a device buffer of at least
// stage_bytes() bytes that the call may overwrite.
int apply(const Model& m, bool adjoint, int dtype, const void* in, void* out, void* stage,
          hipStream_t st);
// apply() with its stage buffer in a static device array of kStaticScratchBytes (no
// allocation); calls that overlap on one device race for that array.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
int apply_noalloc(const Model& m, bool adjoint, int dtype, const void* in, void* out,
                  hipStream_t st);
// Ragged batch of FP32-vector applies (dtype FP32, BF16 or FP8): the single applies of the
// requests, enqueued in index order on one stream.
int apply_batch(int n, const Model* const* ms, bool adjoint, int dtype, const float* const* in,
                float* const* out, hipStream_t st);

// solvers.hip
// A solver whose work is enqueued step by step on its stream (kind 0 = LSQR, 1 = FISTA).
class Solver {
 public:
  virtual ~Solver() {}
  virtual int step(int n_iters) = 0;              // enqueue up to n more iterations
  virtual bool all_enqueued() const = 0;
  virtual long long total_iters() const = 0;      // iterations incl. power method / sweeps
  virtual int finish(aroam_solve_info* info) = 0; // synchronise the stream and report
  hipStream_t stream = nullptr;
};
int solver_create(const Model& m, int kind, const aroam_solve_opts& o, const void* s, void* x,
                  hipStream_t st, Solver** out);
size_t solver_footprint(const Model& m, int kind, const aroam_solve_opts& o);
double solver_work(const Model& m, int kind, const aroam_solve_opts& o);
int solve_lsqr(const Model& m, const aroam_solve_opts& o, const void* s, void* x,
               aroam_solve_info* info, hipStream_t st);
int solve_l1(const Model& m, const aroam_solve_opts& o, const void* s, void* x,
             aroam_solve_info* info, hipStream_t st);

// serve.hip
struct Server;
int server_create(size_t budget, int max_slots, int tick, Server** out);
int server_set_large(Server& sv, double large_work, int large_alone);
int server_held(const Server& sv, long long* by_budget, long long* by_large);
int server_submit(Server& sv, const Model& m, int kind, const aroam_solve_opts& o, const void* s,
                  void* x, long long* id);
int server_poll(Server& sv, int* n_resident, int* n_queued);
int server_collect(Server& sv, int max, long long* ids, aroam_solve_info* infos, int* n);
void server_destroy(Server* sv);

// FP8 e4m3 code (OCP: sign, 4 exponent bits of bias 7, 3 mantissa bits, largest finite 448,
// no infinities) of an FP32 value: nearest with ties to even, finite values beyond 448
// saturate to +-448, and NaN and infinities give the NaN code 0x7f / 0xff.
__device__ inline uint8_t f32_to_e4m3(float f) {
  const uint8_t sign = (uint8_t)((__float_as_uint(f) >> 24) & 0x80u);
  const float a = fabsf(f);
  if (!(a <= 3.402823466e38f)) return (uint8_t)(sign | 0x7f);
  if (a >= 448.0f) return (uint8_t)(sign | 0x7e);
  if (a < 0.015625f) {                     // subnormal range: multiples of 2^-9
    const float q = rintf(a * 512.0f);     // q = 8 is the smallest normal, code 0x08
    return (uint8_t)(sign | (uint8_t)q);
  }
  int e;
  const float mant = frexpf(a, &e);        // a = mant 2^e, mant in [0.5, 1)
  float q = rintf(mant * 16.0f);           // 8..16: implicit bit + 3 fraction bits
  if (q >= 16.0f) {
    q = 8.0f;
    e += 1;
  }
  const int eb = e + 6;                    // a = (q / 8) 2^(e - 1), biased exponent e - 1 + 7
  if (eb > 15 || (eb == 15 && q > 14.0f)) return (uint8_t)(sign | 0x7e);
  return (uint8_t)(sign | (uint8_t)(eb << 3) | (uint8_t)((int)q - 8));
}

inline long long ceil_div(long long a, long long b) { return (a + b - 1) / b; }
inline long long round_up(long long a, long long b) { return ceil_div(a, b) * b; }

}  // namespace aroam
