// Band-pass filtering along time of the signals and of every model column (Results: the
// raw signals and the model matrix are band-pass filtered before inversion, 0.5-80 MHz for
// the simulated pairs; Methods, in vivo imaging: 1-120 MHz).  The filter is a zero-phase FIR
// designed by the window method,
//     h[d] = w[d] ((2 f_hi / fs) sinc(2 f_hi d / fs) - (2 f_lo / fs) sinc(2 f_lo d / fs)),
//     w[d] = 0.42 + 0.5 cos(pi d / L) + 0.08 cos(2 pi d / L)   (Blackman),  |d| <= L,
// applied as the linear convolution y[n] = sum_d h[d] x[n - d] cut to the record [0, nt), so
// the filtered model is F A and a column window [lo, hi] becomes [lo - L, hi + L] in [0, nt).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.h"

namespace aroam {

namespace {

constexpr double kPi = 3.14159265358979323846;

double sinc(double u) { return u == 0.0 ? 1.0 : std::sin(kPi * u) / (kPi * u); }

// One wave per stored column: the filtered window [flo, flo + flen) from the raw window
// [rlo, rlo + rlen) of the same column, summed in FP64 over the taps that meet the window.
__global__ __launch_bounds__(64) void k_fir_cols(const int* __restrict__ rlo,
                                                 const long long* __restrict__ roff,
                                                 const double* __restrict__ raw,
                                                 const int* __restrict__ flo,
                                                 const long long* __restrict__ foff,
                                                 const double* __restrict__ taps, int L,
                                                 double* __restrict__ band) {
  const int c = blockIdx.x;
  const int r0 = rlo[c], f0 = flo[c];
  const long long ro = roff[c], fo = foff[c];
  const int rlen = (int)(roff[c + 1] - ro), flen = (int)(foff[c + 1] - fo);
  for (int i = threadIdx.x; i < flen; i += 64) {
    const int n = f0 + i;
    // y[n] = sum_{m in raw window, |n - m| <= L} h[n - m] x[m]
    const int m0 = max(r0, n - L), m1 = min(r0 + rlen - 1, n + L);
    double acc = 0.0;
    for (int m = m0; m <= m1; ++m) acc += taps[n - m + L] * raw[ro + (m - r0)];
    band[fo + i] = acc;
  }
}

constexpr int kFirPad = 8;  // zero coefficients kept on each side of the padded tap table

// Signals [rows][nt]: a workgroup filters 256 * VEC consecutive samples of one row.  The
// input span (with an L halo, zero outside [0, nt)) is staged in LDS; thread t owns the VEC
// consecutive outputs n = n0 + VEC t + r, reads the span in aligned 16-byte chunks, and value
// v of its chunks (x[n0 + VEC t + v - L]) meets output r through h[L + r - v].  The padded
// table P[j + kFirPad] = h[j - L] for j in [0, 2L] (0 for j in [-kFirPad, -1] and
// [2L + 1, 2L + kFirPad]) turns that into P[2L - v + r + kFirPad] without branches.
template <typename T>
__global__ __launch_bounds__(256) void k_fir_signals(const T* __restrict__ in,
                                                     T* __restrict__ out,
                                                     const T* __restrict__ P, int L, int nt,
                                                     int span, int ntiles) {
  constexpr int VEC = 16 / sizeof(T);
  constexpr int OUT = 256 * VEC;
  extern __shared__ __attribute__((aligned(16))) unsigned char sh_raw[];
  T* xs = reinterpret_cast<T*>(sh_raw);
  const long long row = blockIdx.x / ntiles;
  const int n0 = (int)(blockIdx.x % ntiles) * OUT;
  const T* x = in + row * nt;
  for (int i = threadIdx.x; i < span; i += 256) {
    const int m = n0 - L + i;
    xs[i] = (m >= 0 && m < nt) ? x[m] : T(0);
  }
  __syncthreads();
  T acc[VEC];
#pragma unroll
  for (int r = 0; r < VEC; ++r) acc[r] = T(0);
  const int nq = (2 * L + VEC - 1) / VEC + 1;  // chunks covering v in [0, 2L + VEC - 1]
  const T* base = xs + VEC * threadIdx.x;
  for (int q = 0; q < nq; ++q) {
    T v[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) v[e] = base[VEC * q + e];
#pragma unroll
    for (int e = 0; e < VEC; ++e)
#pragma unroll
      for (int r = 0; r < VEC; ++r) {
        const int j = 2 * L - (VEC * q + e) + r;  // in [2 - 2 VEC, 2L + VEC - 1]
        acc[r] += P[j + kFirPad] * v[e];
      }
  }
#pragma unroll
  for (int r = 0; r < VEC; ++r) {
    const int n = n0 + VEC * threadIdx.x + r;
    if (n < nt) out[row * nt + n] = acc[r];
  }
}

template <typename T>
int launch_fir_signals(const Model& m, const void* in, void* out, hipStream_t st) {
  constexpr int VEC = 16 / sizeof(T);
  constexpr int OUT = 256 * VEC;
  const int L = m.fir_L, nt = m.grid.nt;
  const long long rows = (long long)m.grid.nx * m.grid.ny;
  const int nq = (2 * L + VEC - 1) / VEC + 1;
  // every thread reads up to index VEC * 255 + VEC * nq - 1
  const int span = VEC * 255 + VEC * nq;
  const size_t lds = (size_t)span * sizeof(T);
  AROAM_CHECK(lds <= 64 * 1024, AROAM_EINVAL, "filter too long for the LDS stage (%zu bytes)",
              lds);
  const int ntiles = ceil_div(nt, OUT);
  AROAM_CHECK(rows * ntiles < (1LL << 31), AROAM_EUNSUPPORTED, "too many signals per call");
  const T* P = reinterpret_cast<const T*>(sizeof(T) == 8 ? (const void*)m.d_fir_pad64
                                                         : (const void*)m.d_fir_pad32);
  hipLaunchKernelGGL(k_fir_signals<T>, dim3((unsigned)(rows * ntiles)), dim3(256), lds, st,
                     (const T*)in, (T*)out, P, L, nt, span, ntiles);
  AROAM_HIP(hipGetLastError());
  return AROAM_OK;
}

}  // namespace

std::vector<double> fir_taps(const aroam_filter& f, double fs) {
  const int L = f.half_taps;
  std::vector<double> h(2 * L + 1);
  const double lo = 2.0 * f.f_lo_hz / fs, hi = 2.0 * f.f_hi_hz / fs;
  for (int d = -L; d <= L; ++d) {
    const double ideal = hi * sinc(hi * d) - lo * sinc(lo * d);
    const double w = L == 0 ? 1.0
                            : 0.42 + 0.5 * std::cos(kPi * d / L) + 0.08 * std::cos(2.0 * kPi * d / L);
    h[d + L] = w * ideal;
  }
  return h;
}

int check_filter(const aroam_filter& f, double fs, int nt) {
  AROAM_CHECK(std::isfinite(f.f_lo_hz) && std::isfinite(f.f_hi_hz) && f.f_lo_hz >= 0 &&
                  f.f_lo_hz < f.f_hi_hz && f.f_hi_hz <= 0.5 * fs,
              AROAM_EINVAL, "band edges must satisfy 0 <= f_lo < f_hi <= fs / 2");
  AROAM_CHECK(f.half_taps >= 0 && f.half_taps <= 1024 && f.half_taps < nt, AROAM_EINVAL,
              "half_taps must be in [0, min(1024, nt - 1)]");
  return AROAM_OK;
}

int setup_filter(Model& m, const aroam_filter& f) {
  m.filtered = true;
  m.filter = f;
  m.fir_L = f.half_taps;
  m.fir_taps = fir_taps(f, m.grid.fs_hz);
  const int L = m.fir_L;
  // padded table P[j + kFirPad] = h[j - L] for j in [0, 2L], zero on kFirPad entries each side
  std::vector<double> p64(2 * L + 1 + 2 * kFirPad, 0.0);
  std::vector<float> p32(p64.size(), 0.0f);
  for (int j = 0; j <= 2 * L; ++j) {
    p64[j + kFirPad] = m.fir_taps[j];
    p32[j + kFirPad] = (float)m.fir_taps[j];
  }
  AROAM_HIP(hipMalloc((void**)&m.d_fir_taps, m.fir_taps.size() * sizeof(double)));
  AROAM_HIP(hipMalloc((void**)&m.d_fir_pad64, p64.size() * sizeof(double)));
  AROAM_HIP(hipMalloc((void**)&m.d_fir_pad32, p32.size() * sizeof(float)));
  AROAM_HIP(hipMemcpy(m.d_fir_taps, m.fir_taps.data(), m.fir_taps.size() * sizeof(double),
                      hipMemcpyHostToDevice));
  AROAM_HIP(hipMemcpy(m.d_fir_pad64, p64.data(), p64.size() * sizeof(double), hipMemcpyHostToDevice));
  AROAM_HIP(hipMemcpy(m.d_fir_pad32, p32.data(), p32.size() * sizeof(float), hipMemcpyHostToDevice));
  return AROAM_OK;
}

int filter_columns(const Model& m, const int* d_rlo, const long long* d_roff,
                   const double* d_raw, hipStream_t st) {
  if (m.n_stored == 0) return AROAM_OK;
  hipLaunchKernelGGL(k_fir_cols, dim3((unsigned)m.n_stored), dim3(64), 0, st, d_rlo, d_roff,
                     d_raw, m.d_lo, m.d_off, m.d_fir_taps, m.fir_L, m.d_band);
  AROAM_HIP(hipGetLastError());
  return AROAM_OK;
}

int filter_signals(const Model& m, int dtype, const void* in, void* out, hipStream_t st) {
  AROAM_CHECK(m.filtered, AROAM_EINVAL, "the model was built without a band-pass filter");
  AROAM_CHECK(in && out, AROAM_EINVAL, "NULL signal pointer");
  AROAM_CHECK(in != out, AROAM_EINVAL, "in-place filtering is not supported");
  if (dtype == AROAM_FP64) return launch_fir_signals<double>(m, in, out, st);
  if (dtype == AROAM_FP32) return launch_fir_signals<float>(m, in, out, st);
  set_error("signals are filtered in FP64 or FP32 (dtype %d)", dtype);
  return AROAM_EINVAL;
}

}  // namespace aroam
