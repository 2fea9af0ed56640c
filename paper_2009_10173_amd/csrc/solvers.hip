// Solvers of Eq. 5 on the device: LSQR for Tikhonov (Eq. 6) and FISTA for L1 (Eq. 7), with
// the residual-correction refinement schedules for reduced-precision applies.
//
// The host only enqueues: every norm, dot product and scalar recurrence is FP64 on the
// device (deterministic two-stage reductions with a fixed grid), and scalars stay in device
// memory between kernels.  Each solve synchronises its stream once, at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace aroam {

namespace {

constexpr int kRedBlocks = 1024;
constexpr int kRedThreads = 256;

// ------------------------------------------------------------------------------------------
// Deterministic FP64 reductions: each of kRedBlocks blocks sums a fixed strided subset in
// FP64 and writes one partial; a single block then sums the partials in a fixed order.

__device__ inline double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// Maximum that carries a NaN through (fmax drops it), so that a NaN in a vector reaches the
// scalar derived from its maximum and is detected there.
__device__ inline double nan_max(double a, double b) { return (a > b || a != a) ? a : b; }

__device__ inline double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = nan_max(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

// part[b] = sum over this block's elements of a[i] * b[i] (b == nullptr: a[i]^2)
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_dot_partial(const T* __restrict__ a,
                                                             const T* __restrict__ b, long long n,
                                                             double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
    const double x = (double)a[i];
    acc += x * (b ? (double)b[i] : x);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_amax_partial(const T* __restrict__ a, long long n,
                                                              double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride)
    acc = nan_max(acc, fabs((double)a[i]));
  const double s = block_max(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out = sum(part0) (+ sum(part1) if given), or the maximum when is_max.
__global__ __launch_bounds__(kRedThreads) void k_final(const double* __restrict__ part0,
                                                       const double* __restrict__ part1,
                                                       int nparts, bool is_max,
                                                       double* __restrict__ out) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x)
    acc = is_max ? nan_max(acc, part0[i]) : acc + part0[i];
  double r = is_max ? block_max(acc, sh) : block_sum(acc, sh);
  if (part1) {
    double acc1 = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc1 += part1[i];
    r += block_sum(acc1, sh);
  }
  if (threadIdx.x == 0) *out = r;
}

// ------------------------------------------------------------------------------------------
// LSQR state on the device.  Stored vectors carry scales: u = su * u_st, v = sv * v_st, so a
// normalisation costs no extra pass; w and x are stored explicitly.
struct LsqrDev {
  double alpha, beta, su, sv;
  double rhobar, phibar;
  double damp, gamma;  // rotation damping; weight of a stacked identity block
  double xc, wc;       // x += xc w;  w = sv v_st - wc w
  double lambda;
  double nrm_u2, nrm_v2, red;
  int done, bad, bad_iter, iter;
  int failed;      // sticky across the solves of a refinement schedule: an earlier solve failed
  int base;        // iterations of the schedule completed before this solve started
  int fail_iters;  // iterations of the schedule completed before the failure (sticky)
};

__device__ inline bool stop(const LsqrDev* d) { return d->done || d->bad || d->failed; }

// A non-finite value met after `iter` iterations of the current solve.
__device__ inline void lsqr_fail(LsqrDev* d, int iter) {
  d->bad = 1;
  d->bad_iter = iter;
  d->fail_iters = d->base + iter;
}

// Start a new LSQR solve in the state block after `base` iterations of the schedule; `first`
// clears the sticky failure state.
__global__ void k_lsqr_reset(LsqrDev* d, double damp, double gamma, int first, int base) {
  LsqrDev h = {};
  h.damp = damp;
  h.gamma = gamma;
  h.lambda = damp * damp;
  h.su = 1.0;
  h.sv = 1.0;
  h.base = base;
  h.failed = first ? 0 : (d->failed || d->bad);
  h.fail_iters = first ? 0 : d->fail_iters;
  *d = h;
}

// u_st <- a * t + b * u_st with (a, b) read from the state (mode 0: a = sv, b = -alpha su;
// mode 1: a = 1, b = 0, the initial copy).  The stacked block u2 gets a * gamma * v_st.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_lsqr_u(const T* __restrict__ t, T* __restrict__ u,
                                                        long long m, const T* __restrict__ v,
                                                        T* __restrict__ u2, long long n,
                                                        const LsqrDev* __restrict__ d,
                                                        double* __restrict__ part,
                                                        double* __restrict__ part2) {
  __shared__ double sh[kRedThreads];
  if (stop(d)) return;
  const double a = d->sv, b = -d->alpha * d->su;
  const long long stride = (long long)gridDim.x * blockDim.x;
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m; i += stride) {
    const T val = (T)(a * (double)t[i] + b * (double)u[i]);
    u[i] = val;
    acc += (double)val * (double)val;
  }
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
  if (u2) {
    const double ag = a * d->gamma;
    double acc2 = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
      const T val = (T)(ag * (double)v[i] + b * (double)u2[i]);
      u2[i] = val;
      acc2 += (double)val * (double)val;
    }
    s = block_sum(acc2, sh);
    if (threadIdx.x == 0) part2[blockIdx.x] = s;
  }
}

// v_st <- su * (t + gamma * u2_st) - beta * sv * v_st  (init: b = 0)
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_lsqr_v(const T* __restrict__ t,
                                                        const T* __restrict__ u2,
                                                        T* __restrict__ v, long long n, int init,
                                                        const LsqrDev* __restrict__ d,
                                                        double* __restrict__ part) {
  __shared__ double sh[kRedThreads];
  if (stop(d)) return;
  const double a = d->su, b = init ? 0.0 : -d->beta * d->sv, g = d->gamma;
  const long long stride = (long long)gridDim.x * blockDim.x;
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
    double tv = (double)t[i];
    if (u2) tv += g * (double)u2[i];
    const T val = (T)(a * tv + (init ? 0.0 : b * (double)v[i]));
    v[i] = val;
    acc += (double)val * (double)val;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// beta = ||u||, su = 1 / beta (u is left unscaled when beta = 0).
__global__ void k_lsqr_beta(LsqrDev* d) {
  if (stop(d)) return;
  const double b = sqrt(d->red);
  if (!isfinite(b)) {
    lsqr_fail(d, d->iter);
    return;
  }
  d->beta = b;
  d->su = b > 0 ? 1.0 / b : 1.0;
}

// Initial alpha (after v = A^T u) and the LSQR start values.
__global__ void k_lsqr_init_alpha(LsqrDev* d, int lambda_rule) {
  if (stop(d)) return;
  const double a = sqrt(d->red);
  if (!isfinite(a)) {
    lsqr_fail(d, 0);
    return;
  }
  d->alpha = a;
  d->sv = a > 0 ? 1.0 / a : 1.0;
  if (lambda_rule) {  // Tikhonov default: 1e-2 ||A^T s||_2, with ||A^T s|| = alpha beta
    d->lambda = 1e-2 * a * d->beta;
    d->damp = sqrt(d->lambda);
  }
  d->phibar = d->beta;
  d->rhobar = a;
  d->xc = 0.0;
  d->wc = 0.0;
  if (a * d->beta == 0.0) d->done = 1;
}

// alpha = ||v||, then the two plane rotations of LSQR (damping row, then beta).
__global__ void k_lsqr_rotate(LsqrDev* d) {
  if (stop(d)) return;
  const double a = sqrt(d->red);
  if (!isfinite(a)) {
    lsqr_fail(d, d->iter);
    return;
  }
  d->alpha = a;
  d->sv = a > 0 ? 1.0 / a : 1.0;
  const double beta = d->beta;
  const double rhobar1 = sqrt(d->rhobar * d->rhobar + d->damp * d->damp);
  if (rhobar1 == 0.0 || rhobar1 * rhobar1 + beta * beta == 0.0) {
    d->done = 1;  // exact breakdown: x is final
    return;
  }
  const double cs1 = d->rhobar / rhobar1;
  double phibar = cs1 * d->phibar;
  const double rho = sqrt(rhobar1 * rhobar1 + beta * beta);
  const double cs = rhobar1 / rho, sn = beta / rho;
  const double theta = sn * a;
  d->rhobar = -cs * a;
  const double phi = cs * phibar;
  d->phibar = sn * phibar;
  d->xc = phi / rho;
  d->wc = theta / rho;
  d->iter += 1;
}

// x += xc w;  w = sv v_st - wc w   (init: w = sv v_st, x = 0)
template <typename T>
__global__ __launch_bounds__(256) void k_lsqr_xw(T* __restrict__ x, T* __restrict__ w,
                                                 const T* __restrict__ v, long long n, int init,
                                                 const LsqrDev* __restrict__ d) {
  if (stop(d) && !init) return;
  const double xc = d->xc, wc = d->wc, sv = d->sv;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
    if (init) {
      x[i] = T(0);
      w[i] = (T)(sv * (double)v[i]);
    } else {
      const double wi = (double)w[i];
      x[i] = (T)((double)x[i] + xc * wi);
      w[i] = (T)(sv * (double)v[i] - wc * wi);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Small vector kernels shared by the drivers.

template <typename T>
__global__ void k_axpby(T* __restrict__ y, const T* __restrict__ a, const T* __restrict__ b,
                        double ca, double cb, long long n) {  // y = ca a + cb b
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride)
    y[i] = (T)(ca * (double)a[i] + (b ? cb * (double)b[i] : 0.0));
}

template <typename T>
__global__ void k_fill(T* __restrict__ y, double v, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) y[i] = (T)v;
}

template <typename T>
__global__ void k_scale_dev(T* __restrict__ y, const T* __restrict__ a, const double* __restrict__ c,
                            long long n) {  // y = c[0] a
  const double cc = *c;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride)
    y[i] = (T)(cc * (double)a[i]);
}

struct FistaDev {
  double L, lambda, rq, ww, vv, inv, amax, ss;
  int bad;       // a non-finite value was met (sticky: later kernels do nothing)
  int bad_iter;  // FISTA iterations completed before it (0 in the power method / parameters)
};

__global__ void k_fista_reset(FistaDev* f) {
  FistaDev h = {};
  *f = h;
}

// Power method bookkeeping: rq = <v, w>, inv = 1 / ||w||.
__global__ void k_power_scalars(FistaDev* f) {
  f->rq = f->vv;
  const double nw = sqrt(f->ww);
  f->inv = nw > 0 ? 1.0 / nw : 0.0;
  if (!isfinite(nw) || !isfinite(f->vv)) f->bad = 1;
}

// The signals enter FISTA only through A^T (A y - s), which reads the samples the model's
// bands reach; ||s||^2 is tested once so that a non-finite sample anywhere stops the solve.
__global__ void k_signal_check(FistaDev* f) {
  if (!isfinite(f->ss)) f->bad = 1;
}

__global__ void k_power_start(FistaDev* f) {
  const double nv = sqrt(f->ww);
  f->inv = nv > 0 ? 1.0 / nv : 0.0;
  if (!isfinite(nv)) f->bad = 1;
}

__global__ void k_fista_params(FistaDev* f, double lipschitz, double lambda, int lambda_rule) {
  f->L = lipschitz > 0 ? lipschitz : 2.0 * 1.01 * f->rq;
  if (lambda_rule) f->lambda = 5e-3 * f->amax;  // L1 default: 5e-3 max|A^T s|
  else f->lambda = lambda;
  if (!(f->L > 0) || !isfinite(f->L) || !isfinite(f->lambda)) f->bad = 1;
}

// One FISTA update (iteration `it`, counted from 0): g = ga + 2 t2 (either may be absent),
// x+ = S_{lambda/L}(y - g / L), y = x+ + mom (x+ - x), x = x+.  The soft threshold maps a NaN
// to 0, so the step's argument is tested before it: a non-finite gradient step marks the
// solve as failed after `it` iterations (every thread that sees one stores the same values).
template <typename T>
__global__ __launch_bounds__(256) void k_fista_step(T* __restrict__ y, T* __restrict__ x,
                                                    const T* __restrict__ ga,
                                                    const T* __restrict__ t2, double mom,
                                                    long long n, int it, FistaDev* f) {
  if (f->bad) return;
  const double L = f->L, thr = f->lambda / L;
  const long long stride = (long long)gridDim.x * blockDim.x;
  bool finite = true;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
    double g = 0.0;
    if (ga) g += (double)ga[i];
    if (t2) g += 2.0 * (double)t2[i];
    const double v = (double)y[i] - g / L;
    finite = finite && isfinite(v);
    const double av = fabs(v) - thr;
    const double xn = av > 0 ? copysign(av, v) : 0.0;
    const double xo = (double)x[i];
    x[i] = (T)xn;
    y[i] = (T)(xn + mom * (xn - xo));
  }
  if (!finite) {
    f->bad_iter = it;
    f->bad = 1;
  }
}

// ------------------------------------------------------------------------------------------

// Solver objects: creation enqueues the set-up, step(n) enqueues the next n iterations, and
// finish() synchronises once.  The blocking entry points run create + step(all) + finish;
// the request scheduler interleaves the steps of many solvers on separate streams.

int grid_for(long long n) { return (int)std::max<long long>(1, std::min<long long>(ceil_div(n, 256), 4096)); }

int check_dtype(const Model& m, int dt) {
  AROAM_CHECK(dt >= AROAM_FP64 && dt <= AROAM_FP8E4M3, AROAM_EINVAL, "bad dtype %d", dt);
  AROAM_CHECK((m.dtype_mask >> dt) & 1u, AROAM_EUNSUPPORTED, "model was not packed for dtype %d", dt);
  return AROAM_OK;
}

size_t vec_bytes(long long n, size_t esize) { return (size_t)round_up(std::max<long long>(1, n) * esize, 256); }

template <typename T>
class SolverT final : public Solver {
 public:
  SolverT(const Model& m, int kind, const aroam_solve_opts& o, const T* s, T* x, hipStream_t st)
      : m_(m), kind_(kind), o_(o), s_(s), x_(x) {
    stream = st;
    ns_ = (long long)m.grid.ny * m.grid.nx * m.grid.nt;
    nx_ = (long long)m.grid.ny * m.grid.nx * m.grid.nz;
  }
  ~SolverT() override {
    for (void* p : allocs_) (void)hipFreeAsync(p, stream);
  }

  // Device bytes the solver allocates (stage buffers, reductions, state, vectors).
  static size_t footprint(const Model& m, int kind, const aroam_solve_opts& o) {
    const long long ns = (long long)m.grid.ny * m.grid.nx * m.grid.nt;
    const long long nx = (long long)m.grid.ny * m.grid.nx * m.grid.nz;
    size_t b = std::max(stage_bytes(m, false, o.inner), stage_bytes(m, false, o.outer)) +
               std::max(stage_bytes(m, true, o.inner), stage_bytes(m, true, o.outer)) +
               2 * vec_bytes(kRedBlocks, 8) + 2 * vec_bytes(1, 512);
    const size_t e = sizeof(T);
    if (kind == 0) {
      b += 2 * vec_bytes(ns, e) + 3 * vec_bytes(nx, e);  // u, ts; v, w, tx
      if (o.refine_sweeps > 0) b += vec_bytes(ns, e) + 4 * vec_bytes(nx, e);  // rs; u2, gx, rx, dx
    } else {
      b += vec_bytes(ns, e) + 4 * vec_bytes(nx, e);  // ts; y, xp, tx, v
      if (o.inner != o.outer) b += 3 * vec_bytes(nx, e);  // ga, xa, dv
    }
    return b;
  }

  int create() {
    AROAM_TRY(check_dtype(m_, o_.inner));
    AROAM_TRY(check_dtype(m_, o_.outer));
    AROAM_CHECK(s_ && x_, AROAM_EINVAL, "NULL vector");
    AROAM_CHECK(o_.iters >= 0 && o_.refine_sweeps >= 0 && o_.power_iters >= 0, AROAM_EINVAL,
                "negative iteration count");
    AROAM_TRY(alloc_bytes(&stage_f_, std::max(stage_bytes(m_, false, o_.inner),
                                              stage_bytes(m_, false, o_.outer))));
    AROAM_TRY(alloc_bytes(&stage_a_, std::max(stage_bytes(m_, true, o_.inner),
                                              stage_bytes(m_, true, o_.outer))));
    AROAM_TRY(alloc_bytes((void**)&part0_, kRedBlocks * sizeof(double)));
    AROAM_TRY(alloc_bytes((void**)&part1_, kRedBlocks * sizeof(double)));
    return kind_ == 0 ? create_lsqr() : create_l1();
  }

  int step(int n) override { return kind_ == 0 ? step_lsqr(n) : step_l1(n); }
  bool all_enqueued() const override { return enqueued_ >= total_; }
  long long total_iters() const override { return total_; }
  int finish(aroam_solve_info* info) override { return kind_ == 0 ? finish_lsqr(info) : finish_l1(info); }

 private:
  const Model& m_;
  int kind_;
  aroam_solve_opts o_;
  const T* s_;
  T* x_;
  long long ns_ = 0, nx_ = 0;
  std::vector<void*> allocs_;
  void *stage_f_ = nullptr, *stage_a_ = nullptr;
  double *part0_ = nullptr, *part1_ = nullptr;
  long long total_ = 0, enqueued_ = 0;
  // LSQR
  LsqrDev* d_ = nullptr;
  T *u_ = nullptr, *ts_ = nullptr, *v_ = nullptr, *w_ = nullptr, *tx_ = nullptr, *u2_ = nullptr;
  T *rs_ = nullptr, *gx_ = nullptr, *rx_ = nullptr, *dx_ = nullptr;
  int phase_ = 0, it_ = 0;  // LSQR phase: 0 main solve, k = correction solve of sweep k
  double lam_ = 0, gam_ = 0;
  // FISTA
  FistaDev* f_ = nullptr;
  T *y_ = nullptr, *xp_ = nullptr, *ga_ = nullptr, *xa_ = nullptr, *dv_ = nullptr;
  int npow_ = 0, period_ = 5, warmup_ = 0;
  double t_ = 1.0;

  int alloc_bytes(void** p, size_t b) {
    AROAM_TRY(pool_alloc(p, std::max<size_t>(1, b), stream));
    allocs_.push_back(*p);
    return AROAM_OK;
  }
  int alloc(T** p, long long n) { return alloc_bytes((void**)p, vec_bytes(n, sizeof(T))); }
  int fwd(int dt, const T* in, T* out) { return apply(m_, false, dt, in, out, stage_f_, stream); }
  int adj(int dt, const T* in, T* out) { return apply(m_, true, dt, in, out, stage_a_, stream); }

  int reduce_sq(const T* a, long long n, double* out) {
    hipLaunchKernelGGL(k_dot_partial<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, stream, a,
                       (const T*)nullptr, n, part0_);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, stream, part0_,
                       (const double*)nullptr, kRedBlocks, false, out);
    AROAM_HIP(hipGetLastError());
    return AROAM_OK;
  }

  // ---- LSQR ------------------------------------------------------------------------------
  // Start one LSQR solve of min ||[b1; b2] - [A; gamma I] x||^2 + damp^2 ||x||^2 into xout
  // (b2 / gamma only for a correction solve of the refinement).
  int lsqr_init(const T* b1, const T* b2, T* xout, double damp, double gamma, int rule, int first) {
    const int gx = grid_for(nx_);
    hipLaunchKernelGGL(k_lsqr_reset, dim3(1), dim3(1), 0, stream, d_, damp, b2 ? gamma : 0.0, first,
                       phase_ * o_.iters);
    AROAM_HIP(hipMemcpyAsync(u_, b1, ns_ * sizeof(T), hipMemcpyDeviceToDevice, stream));
    if (b2) AROAM_HIP(hipMemcpyAsync(u2_, b2, nx_ * sizeof(T), hipMemcpyDeviceToDevice, stream));
    hipLaunchKernelGGL(k_dot_partial<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, stream,
                       (const T*)u_, (const T*)nullptr, ns_, part0_);
    if (b2)
      hipLaunchKernelGGL(k_dot_partial<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, stream,
                         (const T*)u2_, (const T*)nullptr, nx_, part1_);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, stream, part0_,
                       b2 ? part1_ : (const double*)nullptr, kRedBlocks, false, &d_->red);
    hipLaunchKernelGGL(k_lsqr_beta, dim3(1), dim3(1), 0, stream, d_);
    AROAM_TRY(adj(o_.inner, u_, tx_));
    hipLaunchKernelGGL(k_lsqr_v<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, stream,
                       (const T*)tx_, (const T*)(b2 ? u2_ : nullptr), v_, nx_, 1,
                       (const LsqrDev*)d_, part0_);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, stream, part0_,
                       (const double*)nullptr, kRedBlocks, false, &d_->red);
    hipLaunchKernelGGL(k_lsqr_init_alpha, dim3(1), dim3(1), 0, stream, d_, rule);
    hipLaunchKernelGGL(k_lsqr_xw<T>, dim3(gx), dim3(256), 0, stream, xout, w_, (const T*)v_,
                       nx_, 1, (const LsqrDev*)d_);
    AROAM_HIP(hipGetLastError());
    return AROAM_OK;
  }

  int lsqr_iter(bool stacked, T* xout) {
    const int gx = grid_for(nx_);
    AROAM_TRY(fwd(o_.inner, v_, ts_));
    hipLaunchKernelGGL(k_lsqr_u<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, stream,
                       (const T*)ts_, u_, ns_, (const T*)v_, stacked ? u2_ : (T*)nullptr, nx_,
                       (const LsqrDev*)d_, part0_, part1_);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, stream, part0_,
                       stacked ? part1_ : (const double*)nullptr, kRedBlocks, false, &d_->red);
    hipLaunchKernelGGL(k_lsqr_beta, dim3(1), dim3(1), 0, stream, d_);
    AROAM_TRY(adj(o_.inner, u_, tx_));
    hipLaunchKernelGGL(k_lsqr_v<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, stream,
                       (const T*)tx_, (const T*)(stacked ? u2_ : nullptr), v_, nx_, 0,
                       (const LsqrDev*)d_, part0_);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, stream, part0_,
                       (const double*)nullptr, kRedBlocks, false, &d_->red);
    hipLaunchKernelGGL(k_lsqr_rotate, dim3(1), dim3(1), 0, stream, d_);
    hipLaunchKernelGGL(k_lsqr_xw<T>, dim3(gx), dim3(256), 0, stream, xout, w_, (const T*)v_,
                       nx_, 0, (const LsqrDev*)d_);
    AROAM_HIP(hipGetLastError());
    return AROAM_OK;
  }

  int create_lsqr() {
    AROAM_TRY(alloc_bytes((void**)&d_, sizeof(LsqrDev)));
    AROAM_TRY(alloc(&u_, ns_));
    AROAM_TRY(alloc(&ts_, ns_));
    AROAM_TRY(alloc(&v_, nx_));
    AROAM_TRY(alloc(&w_, nx_));
    AROAM_TRY(alloc(&tx_, nx_));
    int rule = o_.lambda < 0;
    lam_ = rule ? 0.0 : o_.lambda;
    if (o_.refine_sweeps > 0) {
      AROAM_TRY(alloc(&u2_, nx_));
      AROAM_TRY(alloc(&rs_, ns_));
      AROAM_TRY(alloc(&gx_, nx_));
      AROAM_TRY(alloc(&rx_, nx_));
      AROAM_TRY(alloc(&dx_, nx_));
    }
    if (rule && (o_.refine_sweeps > 0 || o_.inner != o_.outer)) {
      // Tikhonov rule 1e-2 ||A^T s||_2 with the high-precision adjoint; the correction
      // solves also need sqrt(lambda) on the host, so the value is read back once
      AROAM_TRY(adj(o_.outer, s_, tx_));
      AROAM_TRY(reduce_sq(tx_, nx_, &d_->red));
      double red = 0.0;
      AROAM_HIP(hipMemcpyAsync(&red, &d_->red, sizeof(red), hipMemcpyDeviceToHost, stream));
      AROAM_HIP(hipStreamSynchronize(stream));
      AROAM_CHECK(std::isfinite(red), AROAM_ENONFINITE,
                  "non-finite value in A^T s (lambda rule of the refined LSQR)");
      lam_ = 1e-2 * std::sqrt(red);
      rule = 0;
    }
    AROAM_TRY(lsqr_init(s_, nullptr, x_, std::sqrt(lam_), 0.0, rule, 1));
    gam_ = std::sqrt(lam_);
    AROAM_CHECK(o_.refine_sweeps == 0 || gam_ > 0, AROAM_EINVAL,
                "refinement sweeps need lambda > 0");
    total_ = (long long)o_.iters * (1 + o_.refine_sweeps);
    phase_ = 0;
    it_ = 0;
    if (o_.iters == 0) enqueued_ = total_;
    return AROAM_OK;
  }

  // End of the current solve: a correction is added to x; then the next sweep starts.
  int lsqr_next_phase() {
    if (phase_ > 0) {
      hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for(nx_)), dim3(256), 0, stream, x_, (const T*)x_,
                         (const T*)dx_, 1.0, 1.0, nx_);
      AROAM_HIP(hipGetLastError());
    }
    if (phase_ >= o_.refine_sweeps) return AROAM_OK;
    // high-precision residual of the normal equations g = A^T (s - A x) - lambda x; the
    // correction solves min || [A; sqrt(lambda) I] d - [0; g / sqrt(lambda)] ||
    AROAM_TRY(fwd(o_.outer, x_, rs_));
    hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for(ns_)), dim3(256), 0, stream, rs_, s_,
                       (const T*)rs_, 1.0, -1.0, ns_);
    AROAM_TRY(adj(o_.outer, rs_, gx_));
    hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for(nx_)), dim3(256), 0, stream, rx_, (const T*)gx_,
                       (const T*)x_, 1.0 / gam_, -gam_, nx_);
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(ns_)), dim3(256), 0, stream, rs_, 0.0, ns_);
    AROAM_HIP(hipGetLastError());
    ++phase_;
    it_ = 0;
    return lsqr_init(rs_, rx_, dx_, 0.0, gam_, 0, 0);
  }

  int step_lsqr(int n) {
    while (n > 0 && enqueued_ < total_) {
      if (it_ == o_.iters) AROAM_TRY(lsqr_next_phase());
      AROAM_TRY(lsqr_iter(phase_ > 0, phase_ > 0 ? dx_ : x_));
      ++it_;
      ++enqueued_;
      --n;
      if (enqueued_ == total_ && phase_ > 0) AROAM_TRY(lsqr_next_phase());
    }
    return AROAM_OK;
  }

  int finish_lsqr(aroam_solve_info* info) {
    LsqrDev h;
    AROAM_HIP(hipMemcpyAsync(&h, d_, sizeof(h), hipMemcpyDeviceToHost, stream));
    AROAM_HIP(hipStreamSynchronize(stream));
    const bool bad = h.bad || h.failed;
    const int done = (int)std::min<long long>(enqueued_, (long long)phase_ * o_.iters + h.iter);
    if (info) {
      info->iters_done = bad ? h.fail_iters : done;
      info->status = bad ? AROAM_ENONFINITE : AROAM_OK;
      info->lambda = phase_ > 0 ? lam_ : h.lambda;
      info->lipschitz = 0.0;
      info->rnorm = std::fabs(h.phibar);
      info->alpha = h.alpha;
      info->beta = h.beta;
    }
    if (bad) {
      set_error("non-finite value in LSQR");
      return AROAM_ENONFINITE;
    }
    return AROAM_OK;
  }

  // ---- FISTA -----------------------------------------------------------------------------
  int create_l1() {
    npow_ = o_.lipschitz > 0 ? 0 : (o_.power_iters > 0 ? o_.power_iters : 50);
    period_ = o_.anchor_period > 0 ? o_.anchor_period : 5;
    warmup_ = o_.anchor_warmup >= 0 ? o_.anchor_warmup : o_.iters / 4;
    AROAM_TRY(alloc_bytes((void**)&f_, sizeof(FistaDev)));
    AROAM_TRY(alloc(&y_, nx_));
    AROAM_TRY(alloc(&xp_, nx_));
    AROAM_TRY(alloc(&ts_, ns_));
    AROAM_TRY(alloc(&tx_, nx_));
    AROAM_TRY(alloc(&v_, nx_));
    if (o_.inner != o_.outer) {
      AROAM_TRY(alloc(&ga_, nx_));
      AROAM_TRY(alloc(&xa_, nx_));
      AROAM_TRY(alloc(&dv_, nx_));
    }
    const int gx = grid_for(nx_);
    hipLaunchKernelGGL(k_fista_reset, dim3(1), dim3(1), 0, stream, f_);
    AROAM_TRY(reduce_sq(s_, ns_, &f_->ss));
    hipLaunchKernelGGL(k_signal_check, dim3(1), dim3(1), 0, stream, f_);
    if (npow_ > 0) {
      if (o_.power_start)
        AROAM_HIP(hipMemcpyAsync(v_, o_.power_start, nx_ * sizeof(T), hipMemcpyDeviceToDevice, stream));
      else
        hipLaunchKernelGGL(k_fill<T>, dim3(gx), dim3(256), 0, stream, v_, 1.0, nx_);
      AROAM_TRY(reduce_sq(v_, nx_, &f_->ww));
      hipLaunchKernelGGL(k_power_start, dim3(1), dim3(1), 0, stream, f_);
      hipLaunchKernelGGL(k_scale_dev<T>, dim3(gx), dim3(256), 0, stream, v_, (const T*)v_,
                         (const double*)&f_->inv, nx_);
    }
    hipLaunchKernelGGL(k_fill<T>, dim3(gx), dim3(256), 0, stream, xp_, 0.0, nx_);
    hipLaunchKernelGGL(k_fill<T>, dim3(gx), dim3(256), 0, stream, y_, 0.0, nx_);
    AROAM_HIP(hipGetLastError());
    total_ = npow_ + (long long)o_.iters;
    if (npow_ == 0) AROAM_TRY(l1_params());
    return AROAM_OK;
  }

  // L and lambda once the power method is done (lambda rule: 5e-3 max |A^T s|).
  int l1_params() {
    const int rule = o_.lambda < 0;
    if (rule) {
      AROAM_TRY(adj(o_.outer, s_, tx_));
      hipLaunchKernelGGL(k_amax_partial<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, stream,
                         (const T*)tx_, nx_, part0_);
      hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, stream, part0_,
                         (const double*)nullptr, kRedBlocks, true, &f_->amax);
    }
    hipLaunchKernelGGL(k_fista_params, dim3(1), dim3(1), 0, stream, f_, o_.lipschitz, o_.lambda, rule);
    AROAM_HIP(hipGetLastError());
    return AROAM_OK;
  }

  int power_iter() {
    const int gx = grid_for(nx_);
    AROAM_TRY(fwd(o_.outer, v_, ts_));
    AROAM_TRY(adj(o_.outer, ts_, tx_));
    hipLaunchKernelGGL(k_dot_partial<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, stream,
                       (const T*)v_, (const T*)tx_, nx_, part0_);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, stream, part0_,
                       (const double*)nullptr, kRedBlocks, false, &f_->vv);
    AROAM_TRY(reduce_sq(tx_, nx_, &f_->ww));
    hipLaunchKernelGGL(k_power_scalars, dim3(1), dim3(1), 0, stream, f_);
    hipLaunchKernelGGL(k_scale_dev<T>, dim3(gx), dim3(256), 0, stream, v_, (const T*)tx_,
                       (const double*)&f_->inv, nx_);
    AROAM_HIP(hipGetLastError());
    return AROAM_OK;
  }

  int fista_iter(int it) {
    const int gx = grid_for(nx_), gs = grid_for(ns_);
    const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t_ * t_));
    const double mom = (t_ - 1.0) / tn;
    const bool anchored = o_.inner != o_.outer;
    if (!anchored) {
      AROAM_TRY(fwd(o_.inner, y_, ts_));
      hipLaunchKernelGGL(k_axpby<T>, dim3(gs), dim3(256), 0, stream, ts_, (const T*)ts_, s_, 1.0, -1.0, ns_);
      AROAM_TRY(adj(o_.inner, ts_, tx_));
      hipLaunchKernelGGL(k_fista_step<T>, dim3(gx), dim3(256), 0, stream, y_, xp_,
                         (const T*)nullptr, (const T*)tx_, mom, nx_, it, f_);
    } else if (it < warmup_ || (it - warmup_) % period_ == 0) {
      // anchor: the exact gradient at y in the outer precision
      AROAM_HIP(hipMemcpyAsync(xa_, y_, nx_ * sizeof(T), hipMemcpyDeviceToDevice, stream));
      AROAM_TRY(fwd(o_.outer, y_, ts_));
      hipLaunchKernelGGL(k_axpby<T>, dim3(gs), dim3(256), 0, stream, ts_, (const T*)ts_, s_, 1.0, -1.0, ns_);
      AROAM_TRY(adj(o_.outer, ts_, tx_));
      hipLaunchKernelGGL(k_axpby<T>, dim3(gx), dim3(256), 0, stream, ga_, (const T*)tx_,
                         (const T*)nullptr, 2.0, 0.0, nx_);
      hipLaunchKernelGGL(k_fista_step<T>, dim3(gx), dim3(256), 0, stream, y_, xp_, (const T*)ga_,
                         (const T*)nullptr, mom, nx_, it, f_);
    } else {
      // correction: g = g_a + 2 A^T A (y - x_a) with the inner-precision applies
      hipLaunchKernelGGL(k_axpby<T>, dim3(gx), dim3(256), 0, stream, dv_, (const T*)y_,
                         (const T*)xa_, 1.0, -1.0, nx_);
      AROAM_TRY(fwd(o_.inner, dv_, ts_));
      AROAM_TRY(adj(o_.inner, ts_, tx_));
      hipLaunchKernelGGL(k_fista_step<T>, dim3(gx), dim3(256), 0, stream, y_, xp_, (const T*)ga_,
                         (const T*)tx_, mom, nx_, it, f_);
    }
    AROAM_HIP(hipGetLastError());
    t_ = tn;
    return AROAM_OK;
  }

  int step_l1(int n) {
    while (n > 0 && enqueued_ < total_) {
      if (enqueued_ < npow_) {
        AROAM_TRY(power_iter());
        if (enqueued_ + 1 == npow_) AROAM_TRY(l1_params());
      } else {
        AROAM_TRY(fista_iter((int)(enqueued_ - npow_)));
      }
      ++enqueued_;
      --n;
    }
    return AROAM_OK;
  }

  int finish_l1(aroam_solve_info* info) {
    AROAM_HIP(hipMemcpyAsync(x_, xp_, nx_ * sizeof(T), hipMemcpyDeviceToDevice, stream));
    FistaDev h;
    AROAM_HIP(hipMemcpyAsync(&h, f_, sizeof(h), hipMemcpyDeviceToHost, stream));
    AROAM_HIP(hipStreamSynchronize(stream));
    if (info) {
      info->iters_done = h.bad ? h.bad_iter : (int)std::max<long long>(0, enqueued_ - npow_);
      info->status = h.bad ? AROAM_ENONFINITE : AROAM_OK;
      info->lambda = h.lambda;
      info->lipschitz = h.L;
      info->rnorm = 0.0;
      info->alpha = h.rq;
      info->beta = 0.0;
    }
    if (h.bad) {
      set_error("non-finite value in FISTA after %d iterations", h.bad_iter);
      return AROAM_ENONFINITE;
    }
    return AROAM_OK;
  }
};

template <typename T>
int make_solver(const Model& m, int kind, const aroam_solve_opts& o, const void* s, void* x,
                hipStream_t st, Solver** out) {
  auto* sv = new (std::nothrow) SolverT<T>(m, kind, o, (const T*)s, (T*)x, st);
  AROAM_CHECK(sv, AROAM_ENOMEM, "host allocation failed");
  const int rc = sv->create();
  if (rc != AROAM_OK) {
    delete sv;
    return rc;
  }
  *out = sv;
  return AROAM_OK;
}

int run_blocking(const Model& m, int kind, const aroam_solve_opts& o, const void* s, void* x,
                 aroam_solve_info* info, hipStream_t st) {
  Solver* sv = nullptr;
  const int rc0 = solver_create(m, kind, o, s, x, st, &sv);
  if (rc0 != AROAM_OK) {
    if (info) {  // failed in the set-up: no iteration was done
      *info = aroam_solve_info{};
      info->status = rc0;
    }
    return rc0;
  }
  int rc = sv->step(0x7fffffff);
  if (rc == AROAM_OK) rc = sv->finish(info);
  else (void)hipStreamSynchronize(st);
  delete sv;
  return rc;
}

}  // namespace

int solver_create(const Model& m, int kind, const aroam_solve_opts& o, const void* s, void* x,
                  hipStream_t st, Solver** out) {
  AROAM_CHECK(out && (kind == 0 || kind == 1), AROAM_EINVAL, "bad solver kind");
  AROAM_CHECK(s && x, AROAM_EINVAL, "NULL vector");
  AROAM_CHECK((o.inner == AROAM_FP64) == (o.outer == AROAM_FP64), AROAM_EINVAL,
              "FP64 cannot be mixed with single-precision vectors");
  *out = nullptr;
  if (o.inner == AROAM_FP64) return make_solver<double>(m, kind, o, s, x, st, out);
  return make_solver<float>(m, kind, o, s, x, st, out);
}

size_t solver_footprint(const Model& m, int kind, const aroam_solve_opts& o) {
  if (o.inner == AROAM_FP64) return SolverT<double>::footprint(m, kind, o);
  return SolverT<float>::footprint(m, kind, o);
}

// Multiply-accumulates of a whole solve, for the request scheduler's size policy: A + A^T
// pairs (LSQR: one per iteration and one for the start, per sweep; FISTA: one per power and
// per FISTA iteration, one for the start) times the model's algorithmic MACs per apply.
double solver_work(const Model& m, int kind, const aroam_solve_opts& o) {
  const double pairs = kind == 0 ? (o.iters + 1.0) * (1.0 + o.refine_sweeps)
                                 : (double)o.power_iters + o.iters + 1.0;
  return 2.0 * pairs * (double)m.mac_alg;
}

int solve_lsqr(const Model& m, const aroam_solve_opts& o, const void* s, void* x,
               aroam_solve_info* info, hipStream_t st) {
  return run_blocking(m, 0, o, s, x, info, st);
}

int solve_l1(const Model& m, const aroam_solve_opts& o, const void* s, void* x,
             aroam_solve_info* info, hipStream_t st) {
  return run_blocking(m, 1, o, s, x, info, st);
}

}  // namespace aroam
