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

__device__ inline double block_max(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
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
    acc = fmax(acc, fabs((double)a[i]));
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
    acc = is_max ? fmax(acc, part0[i]) : acc + part0[i];
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
};

__device__ inline bool stop(const LsqrDev* d) { return d->done || d->bad; }

__global__ void k_lsqr_reset(LsqrDev* d, double damp, double gamma) {
  LsqrDev h = {};
  h.damp = damp;
  h.gamma = gamma;
  h.lambda = damp * damp;
  h.su = 1.0;
  h.sv = 1.0;
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
    d->bad = 1;
    d->bad_iter = d->iter;
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
    d->bad = 1;
    d->bad_iter = 0;
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
    d->bad = 1;
    d->bad_iter = d->iter;
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
  double L, lambda, rq, ww, vv, inv, amax;
  int bad;
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
  if (!isfinite(nw)) f->bad = 1;
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

// One FISTA update: g = ga + 2 t2 (either may be absent), x+ = S_{lambda/L}(y - g / L),
// y = x+ + mom (x+ - x), x = x+.
template <typename T>
__global__ __launch_bounds__(256) void k_fista_step(T* __restrict__ y, T* __restrict__ x,
                                                    const T* __restrict__ ga,
                                                    const T* __restrict__ t2, double mom,
                                                    long long n, const FistaDev* __restrict__ f) {
  if (f->bad) return;
  const double L = f->L, thr = f->lambda / L;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += stride) {
    double g = 0.0;
    if (ga) g += (double)ga[i];
    if (t2) g += 2.0 * (double)t2[i];
    const double v = (double)y[i] - g / L;
    const double av = fabs(v) - thr;
    const double xn = av > 0 ? copysign(av, v) : 0.0;
    const double xo = (double)x[i];
    x[i] = (T)xn;
    y[i] = (T)(xn + mom * (xn - xo));
  }
}

// ------------------------------------------------------------------------------------------

int grid_for(long long n) { return (int)std::max<long long>(1, std::min<long long>(ceil_div(n, 256), 4096)); }

template <typename T>
struct Work {
  std::vector<void*> ptrs;
  hipStream_t st;
  int alloc(T** p, long long n) {
    void* q = nullptr;
    AROAM_HIP(hipMallocAsync(&q, (size_t)std::max<long long>(1, n) * sizeof(T), st));
    ptrs.push_back(q);
    *p = (T*)q;
    return AROAM_OK;
  }
  int alloc_bytes(void** p, size_t b) {
    AROAM_HIP(hipMallocAsync(p, std::max<size_t>(1, b), st));
    ptrs.push_back(*p);
    return AROAM_OK;
  }
  ~Work() {
    for (void* p : ptrs) (void)hipFreeAsync(p, st);
  }
};

template <typename T>
struct Ctx {
  const Model& m;
  hipStream_t st;
  long long ns, nx;  // signal and image lengths
  void* stage_f;     // stage buffers for forward / adjoint (large enough for any dtype used)
  void* stage_a;
  double* part0;
  double* part1;
};

template <typename T>
int reduce_sq(Ctx<T>& c, const T* a, long long n, double* out) {
  hipLaunchKernelGGL(k_dot_partial<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, c.st, a,
                     (const T*)nullptr, n, c.part0);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, c.st, c.part0, (const double*)nullptr,
                     kRedBlocks, false, out);
  AROAM_HIP(hipGetLastError());
  return AROAM_OK;
}

// One LSQR solve: min ||[b1; b2] - [A; gamma I] x||^2 + damp^2 ||x||^2 (b2 / gamma only for
// the stacked correction system).  x receives the result.
template <typename T>
int lsqr_run(Ctx<T>& c, int dtype, int iters, double damp, double gamma, int lambda_rule,
             const T* b1, const T* b2, T* x, LsqrDev* d, Work<T>& w) {
  T *u, *v, *wv, *ts, *tx, *u2 = nullptr;
  AROAM_TRY(w.alloc(&u, c.ns));
  AROAM_TRY(w.alloc(&ts, c.ns));
  AROAM_TRY(w.alloc(&v, c.nx));
  AROAM_TRY(w.alloc(&wv, c.nx));
  AROAM_TRY(w.alloc(&tx, c.nx));
  if (b2) AROAM_TRY(w.alloc(&u2, c.nx));
  hipLaunchKernelGGL(k_lsqr_reset, dim3(1), dim3(1), 0, c.st, d, damp, b2 ? gamma : 0.0);
  const int gx = grid_for(c.nx);
  // u = b, beta = ||b||
  AROAM_HIP(hipMemcpyAsync(u, b1, c.ns * sizeof(T), hipMemcpyDeviceToDevice, c.st));
  if (b2) AROAM_HIP(hipMemcpyAsync(u2, b2, c.nx * sizeof(T), hipMemcpyDeviceToDevice, c.st));
  hipLaunchKernelGGL(k_dot_partial<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, c.st, (const T*)u,
                     (const T*)nullptr, c.ns, c.part0);
  if (b2)
    hipLaunchKernelGGL(k_dot_partial<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, c.st,
                       (const T*)u2, (const T*)nullptr, c.nx, c.part1);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, c.st, c.part0,
                     b2 ? c.part1 : (const double*)nullptr, kRedBlocks, false, &d->red);
  hipLaunchKernelGGL(k_lsqr_beta, dim3(1), dim3(1), 0, c.st, d);
  // v = A^T u / beta, alpha = ||v||
  AROAM_TRY(apply(c.m, true, dtype, u, tx, c.stage_a, c.st));
  hipLaunchKernelGGL(k_lsqr_v<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, c.st, (const T*)tx,
                     (const T*)u2, v, c.nx, 1, d, c.part0);
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, c.st, c.part0, (const double*)nullptr,
                     kRedBlocks, false, &d->red);
  hipLaunchKernelGGL(k_lsqr_init_alpha, dim3(1), dim3(1), 0, c.st, d, lambda_rule);
  hipLaunchKernelGGL(k_lsqr_xw<T>, dim3(gx), dim3(256), 0, c.st, x, wv, (const T*)v, c.nx, 1,
                     (const LsqrDev*)d);
  AROAM_HIP(hipGetLastError());
  for (int it = 0; it < iters; ++it) {
    AROAM_TRY(apply(c.m, false, dtype, v, ts, c.stage_f, c.st));
    hipLaunchKernelGGL(k_lsqr_u<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, c.st, (const T*)ts, u,
                       c.ns, (const T*)v, u2, c.nx, (const LsqrDev*)d, c.part0, c.part1);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, c.st, c.part0,
                       b2 ? c.part1 : (const double*)nullptr, kRedBlocks, false, &d->red);
    hipLaunchKernelGGL(k_lsqr_beta, dim3(1), dim3(1), 0, c.st, d);
    AROAM_TRY(apply(c.m, true, dtype, u, tx, c.stage_a, c.st));
    hipLaunchKernelGGL(k_lsqr_v<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, c.st, (const T*)tx,
                       (const T*)u2, v, c.nx, 0, (const LsqrDev*)d, c.part0);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, c.st, c.part0,
                       (const double*)nullptr, kRedBlocks, false, &d->red);
    hipLaunchKernelGGL(k_lsqr_rotate, dim3(1), dim3(1), 0, c.st, d);
    hipLaunchKernelGGL(k_lsqr_xw<T>, dim3(gx), dim3(256), 0, c.st, x, wv, (const T*)v, c.nx, 0,
                       (const LsqrDev*)d);
    AROAM_HIP(hipGetLastError());
  }
  return AROAM_OK;
}

int check_dtype(const Model& m, int dt) {
  AROAM_CHECK(dt >= AROAM_FP64 && dt <= AROAM_FP8E4M3, AROAM_EINVAL, "bad dtype %d", dt);
  AROAM_CHECK((m.dtype_mask >> dt) & 1u, AROAM_EUNSUPPORTED, "model was not packed for dtype %d", dt);
  return AROAM_OK;
}

template <typename T>
int setup_ctx(Ctx<T>& c, Work<T>& w, int inner, int outer) {
  size_t sf = std::max(stage_bytes(c.m, false, inner), stage_bytes(c.m, false, outer));
  size_t sa = std::max(stage_bytes(c.m, true, inner), stage_bytes(c.m, true, outer));
  AROAM_TRY(w.alloc_bytes(&c.stage_f, sf));
  AROAM_TRY(w.alloc_bytes(&c.stage_a, sa));
  AROAM_TRY(w.alloc_bytes((void**)&c.part0, kRedBlocks * sizeof(double)));
  AROAM_TRY(w.alloc_bytes((void**)&c.part1, kRedBlocks * sizeof(double)));
  return AROAM_OK;
}

template <typename T>
int lsqr_solve(const Model& m, const aroam_solve_opts& o, const T* s, T* x,
               aroam_solve_info* info, hipStream_t st) {
  const int inner = o.inner, outer = o.outer;
  AROAM_TRY(check_dtype(m, inner));
  AROAM_TRY(check_dtype(m, outer));
  AROAM_CHECK(o.iters >= 0 && o.refine_sweeps >= 0, AROAM_EINVAL, "negative iteration count");
  Work<T> w;
  w.st = st;
  Ctx<T> c{m, st, (long long)m.grid.ny * m.grid.nx * m.grid.nt,
           (long long)m.grid.ny * m.grid.nx * m.grid.nz, nullptr, nullptr, nullptr, nullptr};
  AROAM_TRY(setup_ctx(c, w, inner, outer));
  LsqrDev* d = nullptr;
  AROAM_TRY(w.alloc_bytes((void**)&d, sizeof(LsqrDev)));
  const int rule = o.lambda < 0;
  const double damp0 = rule ? 0.0 : std::sqrt(o.lambda);
  AROAM_TRY(lsqr_run<T>(c, inner, o.iters, damp0, 0.0, rule, s, nullptr, x, d, w));
  LsqrDev first;
  AROAM_HIP(hipMemcpyAsync(&first, d, sizeof(first), hipMemcpyDeviceToHost, st));
  AROAM_HIP(hipStreamSynchronize(st));
  int status = first.bad ? AROAM_ENONFINITE : AROAM_OK;
  LsqrDev last = first;
  int done_total = first.bad ? first.bad_iter : first.iter;
  if (status == AROAM_OK && o.refine_sweeps > 0) {
    const double lam = first.lambda;
    const double g = std::sqrt(lam);
    AROAM_CHECK(g > 0, AROAM_EINVAL, "refinement sweeps need lambda > 0");
    T *rs, *gx, *rx, *dx;
    AROAM_TRY(w.alloc(&rs, c.ns));
    AROAM_TRY(w.alloc(&gx, c.nx));
    AROAM_TRY(w.alloc(&rx, c.nx));
    AROAM_TRY(w.alloc(&dx, c.nx));
    for (int sw = 0; sw < o.refine_sweeps; ++sw) {
      // high-precision residual of the normal equations: g = A^T (s - A x) - lam x.  The
      // correction solves min || [A; sqrt(lam) I] d - [0; g / sqrt(lam)] || at low precision.
      AROAM_TRY(apply(m, false, outer, x, rs, c.stage_f, st));
      hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for(c.ns)), dim3(256), 0, st, rs, s, (const T*)rs,
                         1.0, -1.0, c.ns);
      AROAM_TRY(apply(m, true, outer, rs, gx, c.stage_a, st));
      hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for(c.nx)), dim3(256), 0, st, rx, (const T*)gx,
                         (const T*)x, 1.0 / g, -g, c.nx);
      hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(c.ns)), dim3(256), 0, st, rs, 0.0, c.ns);
      AROAM_HIP(hipGetLastError());
      AROAM_TRY(lsqr_run<T>(c, inner, o.iters, 0.0, g, 0, rs, rx, dx, d, w));
      hipLaunchKernelGGL(k_axpby<T>, dim3(grid_for(c.nx)), dim3(256), 0, st, x, (const T*)x,
                         (const T*)dx, 1.0, 1.0, c.nx);
      AROAM_HIP(hipGetLastError());
      AROAM_HIP(hipMemcpyAsync(&last, d, sizeof(last), hipMemcpyDeviceToHost, st));
      AROAM_HIP(hipStreamSynchronize(st));
      if (last.bad) {
        status = AROAM_ENONFINITE;
        done_total += last.bad_iter;
        break;
      }
      done_total += last.iter;
    }
  }
  AROAM_HIP(hipStreamSynchronize(st));
  if (info) {
    info->iters_done = done_total;
    info->status = status;
    info->lambda = first.lambda;
    info->lipschitz = 0.0;
    info->rnorm = std::fabs(last.phibar);
    info->alpha = last.alpha;
    info->beta = last.beta;
  }
  if (status != AROAM_OK) set_error("non-finite value in LSQR after %d iterations", done_total);
  return status;
}

template <typename T>
int l1_solve(const Model& m, const aroam_solve_opts& o, const T* s, T* x, aroam_solve_info* info,
             hipStream_t st) {
  const int inner = o.inner, outer = o.outer;
  AROAM_TRY(check_dtype(m, inner));
  AROAM_TRY(check_dtype(m, outer));
  AROAM_CHECK(o.iters >= 0, AROAM_EINVAL, "negative iteration count");
  const int npow = o.power_iters > 0 ? o.power_iters : 50;
  const int period = o.anchor_period > 0 ? o.anchor_period : 5;
  const int warmup = o.anchor_warmup >= 0 ? o.anchor_warmup : o.iters / 4;
  const bool anchored = inner != outer;
  Work<T> w;
  w.st = st;
  Ctx<T> c{m, st, (long long)m.grid.ny * m.grid.nx * m.grid.nt,
           (long long)m.grid.ny * m.grid.nx * m.grid.nz, nullptr, nullptr, nullptr, nullptr};
  AROAM_TRY(setup_ctx(c, w, inner, outer));
  FistaDev* f = nullptr;
  AROAM_TRY(w.alloc_bytes((void**)&f, sizeof(FistaDev)));
  hipLaunchKernelGGL(k_fista_reset, dim3(1), dim3(1), 0, st, f);
  T *y, *xp, *ts, *tx, *v, *ga = nullptr, *xa = nullptr, *dv = nullptr;
  AROAM_TRY(w.alloc(&y, c.nx));
  AROAM_TRY(w.alloc(&xp, c.nx));
  AROAM_TRY(w.alloc(&ts, c.ns));
  AROAM_TRY(w.alloc(&tx, c.nx));
  AROAM_TRY(w.alloc(&v, c.nx));
  const int gx = grid_for(c.nx), gs = grid_for(c.ns);
  // Lipschitz constant: power method on A^T A in the outer precision
  if (o.lipschitz <= 0) {
    if (o.power_start)
      AROAM_HIP(hipMemcpyAsync(v, o.power_start, c.nx * sizeof(T), hipMemcpyDeviceToDevice, st));
    else
      hipLaunchKernelGGL(k_fill<T>, dim3(gx), dim3(256), 0, st, v, 1.0, c.nx);
    AROAM_TRY(reduce_sq<T>(c, v, c.nx, &f->ww));
    hipLaunchKernelGGL(k_power_start, dim3(1), dim3(1), 0, st, f);
    hipLaunchKernelGGL(k_scale_dev<T>, dim3(gx), dim3(256), 0, st, v, (const T*)v,
                       (const double*)&f->inv, c.nx);
    for (int it = 0; it < npow; ++it) {
      AROAM_TRY(apply(m, false, outer, v, ts, c.stage_f, st));
      AROAM_TRY(apply(m, true, outer, ts, tx, c.stage_a, st));
      hipLaunchKernelGGL(k_dot_partial<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, (const T*)v,
                         (const T*)tx, c.nx, c.part0);
      hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, st, c.part0,
                         (const double*)nullptr, kRedBlocks, false, &f->vv);
      AROAM_TRY(reduce_sq<T>(c, tx, c.nx, &f->ww));
      hipLaunchKernelGGL(k_power_scalars, dim3(1), dim3(1), 0, st, f);
      hipLaunchKernelGGL(k_scale_dev<T>, dim3(gx), dim3(256), 0, st, v, (const T*)tx,
                         (const double*)&f->inv, c.nx);
      AROAM_HIP(hipGetLastError());
    }
  }
  // lambda rule needs max |A^T s|
  const int rule = o.lambda < 0;
  if (rule) {
    AROAM_TRY(apply(m, true, outer, s, tx, c.stage_a, st));
    hipLaunchKernelGGL(k_amax_partial<T>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, (const T*)tx,
                       c.nx, c.part0);
    hipLaunchKernelGGL(k_final, dim3(1), dim3(kRedThreads), 0, st, c.part0, (const double*)nullptr,
                       kRedBlocks, true, &f->amax);
  }
  hipLaunchKernelGGL(k_fista_params, dim3(1), dim3(1), 0, st, f, o.lipschitz, o.lambda, rule);
  AROAM_HIP(hipGetLastError());
  // FISTA from x0 = 0
  hipLaunchKernelGGL(k_fill<T>, dim3(gx), dim3(256), 0, st, xp, 0.0, c.nx);
  hipLaunchKernelGGL(k_fill<T>, dim3(gx), dim3(256), 0, st, y, 0.0, c.nx);
  if (anchored) {
    AROAM_TRY(w.alloc(&ga, c.nx));
    AROAM_TRY(w.alloc(&xa, c.nx));
    AROAM_TRY(w.alloc(&dv, c.nx));
  }
  double t = 1.0;
  for (int it = 0; it < o.iters; ++it) {
    const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
    const double mom = (t - 1.0) / tn;
    if (!anchored) {
      AROAM_TRY(apply(m, false, inner, y, ts, c.stage_f, st));
      hipLaunchKernelGGL(k_axpby<T>, dim3(gs), dim3(256), 0, st, ts, (const T*)ts, s, 1.0, -1.0, c.ns);
      AROAM_TRY(apply(m, true, inner, ts, tx, c.stage_a, st));
      hipLaunchKernelGGL(k_fista_step<T>, dim3(gx), dim3(256), 0, st, y, xp, (const T*)nullptr,
                         (const T*)tx, mom, c.nx, (const FistaDev*)f);
    } else if (it < warmup || (it - warmup) % period == 0) {
      // anchor: exact gradient at y in the outer precision
      AROAM_HIP(hipMemcpyAsync(xa, y, c.nx * sizeof(T), hipMemcpyDeviceToDevice, st));
      AROAM_TRY(apply(m, false, outer, y, ts, c.stage_f, st));
      hipLaunchKernelGGL(k_axpby<T>, dim3(gs), dim3(256), 0, st, ts, (const T*)ts, s, 1.0, -1.0, c.ns);
      AROAM_TRY(apply(m, true, outer, ts, tx, c.stage_a, st));
      hipLaunchKernelGGL(k_axpby<T>, dim3(gx), dim3(256), 0, st, ga, (const T*)tx,
                         (const T*)nullptr, 2.0, 0.0, c.nx);
      hipLaunchKernelGGL(k_fista_step<T>, dim3(gx), dim3(256), 0, st, y, xp, (const T*)ga,
                         (const T*)nullptr, mom, c.nx, (const FistaDev*)f);
    } else {
      // correction: g = g_a + 2 A^T A (y - x_a) with the inner-precision applies
      hipLaunchKernelGGL(k_axpby<T>, dim3(gx), dim3(256), 0, st, dv, (const T*)y, (const T*)xa,
                         1.0, -1.0, c.nx);
      AROAM_TRY(apply(m, false, inner, dv, ts, c.stage_f, st));
      AROAM_TRY(apply(m, true, inner, ts, tx, c.stage_a, st));
      hipLaunchKernelGGL(k_fista_step<T>, dim3(gx), dim3(256), 0, st, y, xp, (const T*)ga,
                         (const T*)tx, mom, c.nx, (const FistaDev*)f);
    }
    AROAM_HIP(hipGetLastError());
    t = tn;
  }
  AROAM_HIP(hipMemcpyAsync(x, xp, c.nx * sizeof(T), hipMemcpyDeviceToDevice, st));
  FistaDev fh;
  AROAM_HIP(hipMemcpyAsync(&fh, f, sizeof(fh), hipMemcpyDeviceToHost, st));
  AROAM_HIP(hipStreamSynchronize(st));
  const int status = fh.bad ? AROAM_ENONFINITE : AROAM_OK;
  if (info) {
    info->iters_done = fh.bad ? 0 : o.iters;
    info->status = status;
    info->lambda = fh.lambda;
    info->lipschitz = fh.L;
    info->rnorm = 0.0;
    info->alpha = fh.rq;
    info->beta = 0.0;
  }
  if (status != AROAM_OK) set_error("non-finite value in FISTA (Lipschitz constant or lambda)");
  return status;
}

}  // namespace

int solve_lsqr(const Model& m, const aroam_solve_opts& o, const void* s, void* x,
               aroam_solve_info* info, hipStream_t st) {
  AROAM_CHECK(s && x, AROAM_EINVAL, "NULL vector");
  AROAM_CHECK((o.inner == AROAM_FP64) == (o.outer == AROAM_FP64), AROAM_EINVAL,
              "FP64 cannot be mixed with single-precision vectors");
  if (o.inner == AROAM_FP64) return lsqr_solve<double>(m, o, (const double*)s, (double*)x, info, st);
  return lsqr_solve<float>(m, o, (const float*)s, (float*)x, info, st);
}

int solve_l1(const Model& m, const aroam_solve_opts& o, const void* s, void* x,
             aroam_solve_info* info, hipStream_t st) {
  AROAM_CHECK(s && x, AROAM_EINVAL, "NULL vector");
  AROAM_CHECK((o.inner == AROAM_FP64) == (o.outer == AROAM_FP64), AROAM_EINVAL,
              "FP64 cannot be mixed with single-precision vectors");
  if (o.inner == AROAM_FP64) return l1_solve<double>(m, o, (const double*)s, (double*)x, info, st);
  return l1_solve<float>(m, o, (const float*)s, (float*)x, info, st);
}

}  // namespace aroam
