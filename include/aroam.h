/*
 * aroam.h - C ABI of the MI355X (gfx950) model-based AR-OAM reconstruction library.
 *
 * Model-based inversion for acoustic-resolution optoacoustic microscopy with a raster-scanned
 * spherical sensor (Li, Hofmann et al., "Broadband model-based inversion enables optoacoustic
 * microscopy beyond the acoustic diffraction limit").  The library builds the compressed,
 * scan-symmetric time-domain model, applies it and its transpose, and solves Eq. 5 with LSQR
 * (Tikhonov, Eq. 6) or FISTA (L1, Eq. 7).  Every step runs in hand-written HIP kernels.
 *
 * Conventions shared by all calls
 *   - Return value: AROAM_OK (0) or a negative aroam_status.  aroam_last_error() returns a
 *     message for the calling thread's last failure (valid until that thread's next call).
 *   - Vectors are DEVICE pointers owned by the caller, C-contiguous:
 *       image   x[ny][nx][nz]  (voxel columns; depth fastest)
 *       signals s[ny][nx][nt]  (one time trace per scan position; time fastest)
 *     The voxel lateral grid coincides with the scan grid (Results, first paragraph).
 *     Element type: double for AROAM_FP64, float for every other dtype (AROAM_BF16 and
 *     AROAM_FP8E4M3 name the precision of the model table and operands inside the apply;
 *     the caller's vectors stay FP32).  AROAM_BF16: table and operand rounded to BF16
 *     (nearest, ties to even), products accumulated in FP32.  AROAM_FP8E4M3: OCP e4m3 table
 *     with a power-of-two scale per (offset, 16-depth block) and e4m3 operand with a
 *     power-of-two scale per 64 entries of its fast axis (chosen from that block's largest
 *     |value| over the call's whole input vector, the smallest power of two >= amax / 448),
 *     multiplied on the block-scaled FP8 MFMA, which sums each 128-term product to about
 *     14 bits (measured error below 1e-4 of the sum of absolute products), the sums
 *     accumulated in FP32; NaN and infinities in the operand become e4m3 NaN codes.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Applies are asynchronous; the
 *     solvers enqueue all their work on `stream` and synchronise it once before returning.
 *   - Models are immutable after aroam_build_model and may be shared by concurrent calls on
 *     different streams; a model's scratch buffers are per call, so concurrent calls on the
 *     same model are safe.  Destroying a model while work that uses it is in flight is an
 *     error of the caller.
 *   - Scratch memory of applies and solves (staged inputs, partial sums of cut tiles, solver
 *     vectors) is allocated stream-ordered from one memory pool per device that the library
 *     creates on first use.  The pool keeps freed blocks for reuse and holds the peak of
 *     what was in use until the process ends.
 */
#ifndef AROAM_H
#define AROAM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aroam_model aroam_model; /* opaque; owns the device-resident model tables */

typedef enum {
  AROAM_OK = 0,
  AROAM_EINVAL = -1,      /* bad argument: NULL pointer, size out of range, bad dtype        */
  AROAM_ENOMEM = -2,      /* a device or host allocation failed                              */
  AROAM_EDEVICE = -3,     /* a HIP runtime call or kernel launch failed                      */
  AROAM_ENONFINITE = -4,  /* a solver met a non-finite norm; info->iters_done says where     */
  AROAM_EUNSUPPORTED = -5 /* the model was built without the requested dtype                 */
} aroam_status;

typedef enum { AROAM_FP64 = 0, AROAM_FP32 = 1, AROAM_BF16 = 2, AROAM_FP8E4M3 = 3 } aroam_dtype;

/* Largest lateral model extent k_half (offsets -k_half .. k_half).  The staged applies keep,
 * per workgroup, 9 scan rows x (32 + 2 k_half) columns x 80 bytes of input in the 160 KiB LDS
 * of a compute unit.  At the 5 um step this is about 0.97 mm of lateral extent. */
#define AROAM_MAX_K_HALF 97

/* Spherical-cap sensor (Methods, "Forward modeling", Eq. 3; "AR-OAM set-up").
 *   radius_m   radius of curvature = focal distance
 *   aperture_m chord diameter of the cap (numerical aperture = aperture / (2 radius))
 *   hole_m     diameter of a central hole, 0 for none
 *   n_rings    equal-angle rings of sub-elements (0 selects 20); each ring is cut into a
 *              multiple of 8 patches of equal area, so ~1200 sub-elements at the default
 *   f0_hz      centre frequency of the electrical impulse response (EIR)
 *   frac_bw    its -6 dB amplitude bandwidth as a fraction of f0 (1.0 = 100 %)          */
typedef struct {
  double radius_m, aperture_m, hole_m;
  int n_rings;
  double f0_hz, frac_bw;
} aroam_sensor;

/* Acquisition and reconstruction grid.
 *   c_mps, fs_hz   speed of sound, temporal sampling rate
 *   nx, ny, step_m scan positions (== voxel columns) and their lateral spacing
 *   nz, dz_m       voxel depths z_k = (k - nz/2) dz from the focal plane, + = away from sensor
 *   nt             time samples per scan position; sample nt/2 is the focal arrival R / c
 *   k_half         lateral model extent: offsets -k_half..k_half in x and y,
 *                  0 <= k_half <= AROAM_MAX_K_HALF
 *   footprint_mode 0: full (2 k_half + 1)^2 square at every depth;
 *                  1: also (dx^2 + dy^2) step^2 <= (rho0 + |z| tan(theta_max))^2 with
 *                     rho0 = 2 * 0.71 lambda(f0) / NA (the diffraction-limit rule, Results)
 * Discretisation of the model (Methods, Forward modeling); zero-initialised fields select the
 * point voxel with the analytic derivative:
 *   voxel_basis     0: point absorber at the voxel centre; 1: trilinear (tent) basis of half
 *                   width one voxel spacing in x, y and z, integrated over the voxel by the
 *                   product of basis_quad-point Gauss-Legendre rules on each half axis with
 *                   the tent folded into the weights
 *   time_derivative 0: analytic derivative of the EIR; 1: central difference
 *                   (s(n + 1) - s(n - 1)) / 2 of the band-limited signal
 *   basis_quad      Gauss points per half axis of the trilinear basis, 1..8 (0 = 3)        */
typedef struct {
  double c_mps, fs_hz;
  int nx, ny;
  double step_m;
  int nz;
  double dz_m;
  int nt;
  int k_half;
  int footprint_mode;
  int voxel_basis;
  int time_derivative;
  int basis_quad;
} aroam_grid;

/* Sizes and work figures of a built model. */
typedef struct {
  long long n_columns;   /* (offset, depth) columns kept by the footprint with a non-empty window */
  long long nnz;         /* band entries of the compressed table over all those columns           */
  long long mac_alg;     /* algorithmic multiply-accumulates of one apply of A (or A^T)           */
  long long mac_exec[4]; /* MACs the forward kernel issues per apply, indexed by aroam_dtype      */
  long long mac_exec_adj[4]; /* the same for the adjoint kernel                                   */
  size_t device_bytes;   /* device memory held by the model                                        */
  int n_elements;        /* sensor sub-elements M                                                  */
  unsigned dtype_mask;   /* bit (1 << dtype) set for every dtype the model was packed for          */
  long long stored_columns; /* FP64 columns held on the device: a built model stores one column
                             * per symmetry class of the square (H[dx,dy] = H[+-dx,+-dy] =
                             * H[dy,dx]), an imported one every column it was given */
  long long stored_nnz;  /* FP64 band entries held on the device                                   */
  int row_tiles[4];      /* output row tiles of the forward kernel (time samples), by aroam_dtype  */
  int row_tiles_adj[4];  /* the same for the adjoint (depths)                                      */
  int pieces[4];         /* workgroup rows of the forward launch: row_tiles, or more where the
                          * stage units of heavy tiles are cut into pieces whose partial sums a
                          * second kernel adds (load balance of the launch)                       */
  int pieces_adj[4];     /* the same for the adjoint                                               */
} aroam_model_info;

/* Build the compressed model (Methods, "Efficient reconstruction based on scanning
 * symmetries"): for one scan position, every voxel column within the lateral footprint gets
 *     H[o][n, k] = sum_j dS_j / (2 pi r_j) e'((n - nt/2) - fs (r_j - R) / c)
 * (Eq. 1 for point voxels, summed over sub-elements per Eq. 3-4, convolved with the EIR
 * e(t) = exp(-t^2 / (2 sigma^2)) cos(2 pi f0 t); a term counts iff |tau| <= 5 sigma).  The
 * table is computed on the device in FP64 and packed into band tiles for every dtype whose
 * bit is set in dtype_mask (1 << AROAM_FP32 etc.; FP64 and FP32 are always packed).  The
 * sub-element set and the footprint are invariant under the square's symmetry group (the
 * sensor's axial symmetry), so one column per class {(+-dx, +-dy), (+-dy, +-dx)} is computed
 * and stored, and the offsets of a class share it.
 * On success *out owns the device tables; release with aroam_model_destroy.
 * Errors: AROAM_EINVAL for NULL pointers or sizes out of range (nx, ny, nz, nt >= 1,
 * 0 <= k_half <= AROAM_MAX_K_HALF, at most 4096 sub-elements), AROAM_ENOMEM, AROAM_EDEVICE.
 * Synchronises `stream` before returning. */
int aroam_build_model(const aroam_sensor* sensor, const aroam_grid* grid, unsigned dtype_mask,
                      void* stream, aroam_model** out);

/* Build a model from a table given in HOST memory instead of from the sensor geometry: a
 * model matrix estimated by experiment (Discussion: raster-scanning a small particle through
 * the volume for one transducer position) or computed elsewhere.
 *   grid    scan / voxel grids and k_half; footprint_mode is ignored (the footprint is wherever
 *           a column has a window)
 *   dense   [(2 k_half + 1)][(2 k_half + 1)][nz][nt] doubles, H[dy + K][dx + K][k][n] (the layout
 *           aroam_model_export_table writes); read only, the caller keeps ownership
 *   col_lo, col_hi  [(2 k_half + 1)][(2 k_half + 1)][nz] inclusive sample windows, -1 for an
 *           inactive column (values outside a window are ignored); both NULL: each column's
 *           window is its first..last nonzero sample, all-zero columns are inactive
 * Every column is stored as given (no symmetry folding).  dtype_mask as for
 * aroam_build_model.  Errors: AROAM_EINVAL (NULL pointers, sizes out of range, a window outside
 * [0, nt) or only one of col_lo / col_hi given), AROAM_ENONFINITE (a non-finite value inside a
 * window), AROAM_ENOMEM, AROAM_EDEVICE.  Synchronises `stream` before returning. */
int aroam_import_model(const aroam_grid* grid, const double* dense, const int* col_lo,
                       const int* col_hi, unsigned dtype_mask, void* stream, aroam_model** out);

/* Band-pass filter applied along time to the signals and to every model column before the
 * inversion (Results: 0.5-80 MHz for the simulated sub-diffraction pairs; Methods, in vivo
 * imaging: 1-120 MHz; the filter itself is not specified there).  A zero-phase FIR designed by
 * the window method with 2 half_taps + 1 taps:
 *     h[d] = w[d] ((2 f_hi / fs) sinc(2 f_hi d / fs) - (2 f_lo / fs) sinc(2 f_lo d / fs)),
 *     w[d] = 0.42 + 0.5 cos(pi d / L) + 0.08 cos(2 pi d / L)  (Blackman),  |d| <= L = half_taps,
 * sinc(u) = sin(pi u) / (pi u), applied as y[n] = sum_d h[d] x[n - d] with x = 0 outside
 * [0, nt).  Band edges below about fs / (2 L) are only approximated by so short a filter. */
typedef struct {
  double f_lo_hz, f_hi_hz;  /* band edges, 0 <= f_lo < f_hi <= fs / 2                */
  int half_taps;            /* L, 0 <= L <= min(1024, nt - 1)                       */
} aroam_filter;

/* aroam_build_model for the filtered model F A: every column of the table is filtered along
 * time (its window [lo, hi] grows to [lo - L, hi + L] within [0, nt)).  The model keeps the
 * filter for aroam_filter_signals.  Errors as aroam_build_model, plus AROAM_EINVAL for a NULL
 * or invalid filter. */
int aroam_build_model_filtered(const aroam_sensor* sensor, const aroam_grid* grid,
                               const aroam_filter* filter, unsigned dtype_mask, void* stream,
                               aroam_model** out);

/* s_out = F s_in for all ny * nx signals [ny][nx][nt] (device pointers, FP64 or FP32 as
 * `dtype`, accumulated in that precision) with the filter of a model built by
 * aroam_build_model_filtered.  Asynchronous on `stream`.  s_in and s_out must not overlap.
 * Errors: AROAM_EINVAL (NULL pointers, in == out, a model without a filter, dtype other than
 * FP64 / FP32), AROAM_EDEVICE. */
int aroam_filter_signals(const aroam_model* model, int dtype, const void* s_in, void* s_out,
                         void* stream);

/* Fill *info (host pointer). */
int aroam_model_query(const aroam_model* model, aroam_model_info* info);

/* Copy the FP64 table to HOST memory.
 *   dense   [(2 k_half + 1)][(2 k_half + 1)][nz][nt] doubles, H[dy + K][dx + K][k][n], zero
 *           outside the band and the footprint; may be NULL.
 *   col_lo, col_hi  [(2 k_half + 1)][(2 k_half + 1)][nz] ints: inclusive sample window of each
 *           column, -1 for columns outside the footprint or with an empty window; may be NULL.
 * Synchronous.  Errors: AROAM_EINVAL (model NULL), AROAM_EDEVICE. */
int aroam_model_export_table(const aroam_model* model, double* dense, int* col_lo, int* col_hi);

/* Copy the reduced-precision table of one apply direction to HOST memory, in the layout of
 * aroam_model_export_table, each entry being exactly the value that the dtype's apply
 * multiplies (for error analysis of the quantised table):
 *   dtype    AROAM_FP32: the FP64 table rounded to FP32;  AROAM_BF16: those FP32 values
 *            rounded to BF16 (nearest, ties to even);  AROAM_FP8E4M3: e4m3(v / scale) * scale
 *            with the FP32 value v / scale rounded to the nearest e4m3 code (ties to even) and
 *            scale the smallest power of two >= amax / 448 of the entry's (offset, 16-depth
 *            block), amax the largest |value| of the FP64 table in that block
 *   adjoint  0: the forward pack, 1: the adjoint pack (each is checked on its own)
 *   dense    [(2 k_half + 1)][(2 k_half + 1)][nz][nt] doubles, H[dy + K][dx + K][k][n]; required
 *   block_scales  FP8 only, may be NULL: [(2 k_half + 1)][(2 k_half + 1)][ceil(nz / 16)] floats,
 *            the scale of each (offset, 16-depth block), 0 where the block has no entries
 * Synchronous.  Errors: AROAM_EINVAL (NULL model or dense, dtype not FP32 / BF16 / FP8),
 * AROAM_EUNSUPPORTED (dtype not packed), AROAM_EDEVICE. */
int aroam_model_export_quantized(const aroam_model* model, int dtype, int adjoint, double* dense,
                                 float* block_scales);

/* s = A x  (Eq. 4 with the translational symmetry of the Methods):
 *   s[iy, ix, n] = sum_{o, (iy+dy, ix+dx) in grid} sum_k H[o][n, k] x[iy+dy, ix+dx, k].
 * Every element of s is written (no accumulation into s).  x and s must not overlap.
 * Errors: AROAM_EINVAL, AROAM_EUNSUPPORTED (dtype not packed), AROAM_ENOMEM, AROAM_EDEVICE. */
int aroam_forward(const aroam_model* model, int dtype, const void* x, void* s, void* stream);

/* aroam_forward that allocates nothing, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation).  The same
 * kernels and result as aroam_forward (bit for bit), but the apply's scratch (the zero-padded
 * staged input and the partial sums of cut tiles) lives in a static device array of 64 MiB
 * that the library holds on each GPU it runs on until the process ends, instead of coming from
 * the memory pool.  Every call on one GPU shares that array: calls that overlap on one GPU
 * (on different streams, or from different threads) race and give undefined results;
 * serialise them.  The array needs no clearing: each call writes all of it that it reads.
 * Errors: as aroam_forward, plus AROAM_EINVAL when the apply needs more than the 64 MiB
 * (the message gives the size; the 200x200 workload's forward needs 33 MB, a 400x400 one
 * with 256 depths about 0.25 GB). */
int aroam_forward_noalloc(const aroam_model* model, int dtype, const void* x, void* s,
                          void* stream);

/* x = A^T s:  x[jy, jx, k] = sum_{o, (jy-dy, jx-dx) in grid} sum_n H[o][n, k] s[jy-dy, jx-dx, n].
 * Every element of x is written.  Same errors as aroam_forward. */
int aroam_adjoint(const aroam_model* model, int dtype, const void* s, void* x, void* stream);

/* Solver options.
 *   lambda        Eq. 5 weight; < 0 selects the default rule computed on the device
 *                 (Tikhonov: 1e-2 ||A^T s||_2; L1: 5e-3 max|A^T s|) and reports it in info
 *   iters         iterations (fixed count, x0 = 0, no early stop)
 *   refine_sweeps LSQR: residual-correction sweeps after the first solve (0 = none); sweeps
 *                 need lambda > 0, also when the rule computes it (AROAM_EINVAL otherwise)
 *   anchor_period FISTA with inner != outer: after the warm-up, a high-precision anchor
 *                 gradient every this many iterations (0 = 5)
 *   anchor_warmup FISTA with inner != outer: the first this many iterations take the
 *                 high-precision gradient at every iteration (< 0 = a quarter of iters)
 *   power_iters   FISTA: power-method iterations for the Lipschitz constant (0 = 50)
 *   lipschitz     FISTA: if > 0 use this L instead of the power method
 *   inner, outer  aroam_dtype of the iteration's applies and of the high-precision residuals
 *                 (anchors / refinement residuals); plain solves use inner == outer
 *   power_start   FISTA: optional DEVICE vector of the image's element type holding the power
 *                 method's start vector; NULL uses a vector of ones                         */
typedef struct {
  double lambda;
  int iters, refine_sweeps, anchor_period, power_iters;
  double lipschitz;
  int inner, outer, anchor_warmup;
  const void* power_start;
} aroam_solve_opts;

typedef struct {
  int iters_done, status;
  double lambda, lipschitz;
  double rnorm;  /* LSQR: |phibar| estimate of the stacked residual norm at the end           */
  double alpha, beta; /* LSQR: last bidiagonalisation scalars                                   */
} aroam_solve_info;

/* Tikhonov / least squares (Eq. 5-6): min ||s - A x||^2 + lambda ||x||^2 by LSQR (Paige and
 * Saunders) with damp = sqrt(lambda); lambda = 0 gives plain least squares.  x receives the
 * result (device, image layout).  All norms, dot products and the LSQR scalar recurrences are
 * FP64 on the device.  Takes its work vectors from the per-device memory pool (see
 * Conventions) for the duration of the call; aroam_solve_footprint gives their size.  info
 * (host) may be NULL; on every return it holds the status, and iters_done the iterations
 * completed (0 when the set-up failed).
 * Non-finite values: a non-finite norm (from a NaN or infinity in s, or one that arises)
 * stops the solve with AROAM_ENONFINITE and info->iters_done = the iterations completed
 * before it, counted over all sweeps; the lambda rule of a refined solve on such an s gives
 * AROAM_ENONFINITE with iters_done = 0.  x is then undefined.
 * Errors: AROAM_EINVAL, AROAM_EUNSUPPORTED, AROAM_ENOMEM, AROAM_EDEVICE, AROAM_ENONFINITE. */
int aroam_solve_lsqr(const aroam_model* model, const aroam_solve_opts* opts, const void* s,
                     void* x, aroam_solve_info* info, void* stream);

/* L1 (Eq. 5, 7): min ||s - A x||^2 + lambda ||x||_1 by FISTA (Beck and Teboulle) with step
 * 1 / L, L = 2.02 sigma_max(A)^2 from the power method unless opts->lipschitz > 0, and the
 * soft threshold lambda / L.  Same conventions and errors as aroam_solve_lsqr.  Non-finite
 * values: a non-finite L, lambda (the rule's max|A^T s| carries a NaN through), power-method
 * norm, or gradient step y - g / L (tested before the soft threshold, which would map a NaN
 * to 0) stops the solve with AROAM_ENONFINITE; info->iters_done = the FISTA iterations
 * completed before it (0 when it happened in the power method or the parameters). */
int aroam_solve_l1(const aroam_model* model, const aroam_solve_opts* opts, const void* s,
                   void* x, aroam_solve_info* info, void* stream);

/* Ragged batch of applies: n independent applies, request i using models[i], dtype, x[i]
 * and s[i] (device pointers of FP32 vectors), enqueued on the stream in index order, each
 * with the launches aroam_forward / aroam_adjoint would make for it, so each result equals
 * the single apply's bit for bit.  dtype is AROAM_FP32, AROAM_BF16 or AROAM_FP8E4M3 (the
 * vectors are FP32; AROAM_FP64 is rejected, also when n = 0).  n = 0 with a valid dtype does
 * nothing and succeeds.  A NULL model or a bad dtype is rejected with AROAM_EINVAL before
 * anything is enqueued; any other error
 * of entry i is returned after entries 0 .. i-1 have been enqueued.  Errors as
 * aroam_forward. */
int aroam_forward_batch(int n, const aroam_model* const* models, int dtype,
                        const float* const* x, float* const* s, void* stream);
int aroam_adjoint_batch(int n, const aroam_model* const* models, int dtype,
                        const float* const* s, float* const* x, void* stream);

/* Device bytes a solve allocates for its work vectors, stage buffers and FP64 state (what
 * the request scheduler charges against its budget; the model's tables are not included).
 * kind: 0 = LSQR (aroam_solve_lsqr), 1 = FISTA (aroam_solve_l1). */
int aroam_solve_footprint(const aroam_model* model, int kind, const aroam_solve_opts* opts,
                          size_t* bytes);

/* Continuous-batching request scheduler (a serving loop around the two solvers).
 * A request is one reconstruction: a model (device-resident, shared by requests), a solver
 * kind (0 = LSQR, 1 = FISTA), options, and caller-owned DEVICE vectors s (signals) and x
 * (result), which must stay valid until the request is collected.  Requests are admitted in
 * submission order while one of `max_slots` streams is free and the sum of the resident
 * requests' aroam_solve_footprint stays within `hbm_budget_bytes`; a request whose footprint
 * alone exceeds the budget is finished with status AROAM_ENOMEM.  Each aroam_server_poll
 * call retires completed requests, admits waiting ones, and enqueues `tick_iters` more
 * iterations of every resident request on its own stream, so resident requests run
 * concurrently on the device; it does not block.  A request's kernels and their order do not
 * depend on the other requests, so each result is the same alone and in a mix.
 * Streams are created at the default priority.  All calls on one server must come from one
 * host thread.  aroam_server_destroy waits for resident work and releases everything. */
typedef struct aroam_server aroam_server;
int aroam_server_create(size_t hbm_budget_bytes, int max_slots, int tick_iters,
                        aroam_server** out);
/* Large-request policy (for the latency tail of a mix of small and large requests): a
 * request whose whole solve takes at least `large_macs` multiply-accumulates (A + A^T pairs
 * of the solve times the model's algorithmic MACs per apply: LSQR (iters + 1) per sweep,
 * FISTA power_iters + iters + 1) is large, and at most one large request is resident.  A
 * large request that would be the second waits at its place in the queue.  With
 * large_alone = 0 the requests behind it that are not large are admitted past it; with
 * large_alone = 1 no request is admitted while a large one is resident, so that a large
 * request shares the device only with the requests admitted before it.  large_macs = 0 (the
 * default) turns the policy off.  Set before the first submission.  Errors: AROAM_EINVAL
 * (NULL server, negative threshold, requests already submitted). */
int aroam_server_set_large(aroam_server* server, double large_macs, int large_alone);
/* Admission counters: the polls after which a request waited although a slot was free,
 * because it did not fit the budget (*by_budget) or because of the large-request policy
 * (*by_large).  Either pointer may be NULL.  Errors: AROAM_EINVAL (NULL server). */
int aroam_server_held(const aroam_server* server, long long* by_budget, long long* by_large);
/* Queue a request; *id (may be NULL) receives its identifier (1, 2, ...). */
int aroam_server_submit(aroam_server* server, const aroam_model* model, int kind,
                        const aroam_solve_opts* opts, const void* s, void* x, long long* id);
/* One scheduling round; reports the resident and queued request counts (either may be NULL). */
int aroam_server_poll(aroam_server* server, int* n_resident, int* n_queued);
/* Up to `max` finished requests, oldest first: ids[i], infos[i] (infos may be NULL; status
 * AROAM_OK, AROAM_ENONFINITE or AROAM_ENOMEM).  *n receives the count. */
int aroam_server_collect(aroam_server* server, int max, long long* ids, aroam_solve_info* infos,
                         int* n);
void aroam_server_destroy(aroam_server* server);

/* Release a model and its device memory (NULL is ignored). */
void aroam_model_destroy(aroam_model* model);

/* Message of the calling thread's last error ("" if none). */
const char* aroam_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AROAM_H */
