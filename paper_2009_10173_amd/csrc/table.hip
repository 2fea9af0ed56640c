// Model construction: sensor sub-elements, footprint, FP64 table on the device, band tiles.
//
// The compressed model holds one scan position's columns (Methods, "Efficient
// reconstruction based on scanning symmetries"): for every lateral offset o = (dx, dy) and
// depth k inside the footprint, the time signal
//     H[o][n, k] = sum_j dS_j / (2 pi r_j) e'((n - nt/2) - fs (r_j - R) / c)
// of a point voxel (Eq. 1) seen by the sub-element sum of the spherical sensor (Eq. 3-4),
// convolved with the electrical impulse response e (Results: IR = EIR * SIR).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.h"
#include "plan.h"

namespace aroam {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kMM = 1e3;
constexpr double kCutoffSigmas = 5.0;

// Sub-elements of the spherical cap (Eq. 3): equal-angle rings between the hole and the
// rim; ring l is cut into a multiple of 8 equal patches (square-symmetric set) centred at
// azimuth 2 pi (m + 1/2) / n_l; each patch has the exact zone area / n_l.  Positions are
// relative to the focus in mm, with the sensor above the focal plane (negative z).
void make_elements(const aroam_sensor& s, std::vector<double>& ex, std::vector<double>& ey,
                   std::vector<double>& ez, std::vector<double>& area) {
  const double R = s.radius_m * kMM;
  const double th_m = std::asin(s.aperture_m / (2.0 * s.radius_m));
  const double th_h = s.hole_m > 0 ? std::asin(s.hole_m / (2.0 * s.radius_m)) : 0.0;
  const int nr = s.n_rings > 0 ? s.n_rings : 20;
  const double dth = (th_m - th_h) / nr;
  for (int l = 0; l < nr; ++l) {
    const double t0 = th_h + (th_m - th_h) * l / nr;
    const double t1 = th_h + (th_m - th_h) * (l + 1) / nr;
    const double tb = 0.5 * (t0 + t1);
    const int nl = 8 * std::max(1, (int)std::floor(2.0 * kPi * std::sin(tb) / (8.0 * dth) + 0.5));
    const double a = R * R * (std::cos(t0) - std::cos(t1)) * 2.0 * kPi / nl;
    for (int m = 0; m < nl; ++m) {
      const double phi = 2.0 * kPi * (m + 0.5) / nl;
      ex.push_back(R * std::sin(tb) * std::cos(phi));
      ey.push_back(R * std::sin(tb) * std::sin(phi));
      ez.push_back(-R * std::cos(tb));
      area.push_back(a);
    }
  }
}

double depth_mm(const aroam_grid& g, int k) { return ((k - g.nz / 2) * g.dz_m) * kMM; }

// Lateral footprint (Results, first paragraph; Methods, scanning symmetries): the model is
// cut to |dx|, |dy| <= K, and in mode 1 to the cone (dx^2 + dy^2) step^2 <= rho(z)^2 with
// rho(z) = 2 * 0.71 lambda / NA + |z| tan(theta_max).
bool in_footprint(const aroam_sensor& s, const aroam_grid& g, int dx, int dy, int k) {
  if (g.footprint_mode == 0) return true;
  const double th_m = std::asin(s.aperture_m / (2.0 * s.radius_m));
  const double na = std::sin(th_m);
  const double rho0 = 2.0 * (0.71 * (g.c_mps / s.f0_hz) * kMM / na);
  const double step = g.step_m * kMM;
  const double rho = rho0 + std::fabs(depth_mm(g, k)) * std::tan(th_m);
  return (double)(dx * dx + dy * dy) * step * step <= rho * rho;
}

struct Geo {
  double step, R, cfs, sigma5, inv2s2, invs2, omega;
  int nz, nt, M;
  double dz_m;
  double reach;      // samples around an arrival that the derivative kernel can touch
  int fd;            // 0: analytic derivative of the EIR, 1: central difference
  int nq;            // basis quadrature points (1 for the point voxel)
};

// Time derivative of the EIR truncated at 5 sigma (samples): the analytic e'(tau), or the
// central difference (e(tau + 1) - e(tau - 1)) / 2 (Methods, Forward modeling: finite
// differences in time).
__device__ inline double eir_trunc(double tau, const Geo& geo) {
  if (fabs(tau) > geo.sigma5) return 0.0;
  double sn, cs;
  sincos(geo.omega * tau, &sn, &cs);
  return exp(-tau * tau * geo.inv2s2) * cs;
}

__device__ inline double deriv_kernel(double tau, const Geo& geo) {
  if (geo.fd) return 0.5 * (eir_trunc(tau + 1.0, geo) - eir_trunc(tau - 1.0, geo));
  if (fabs(tau) > geo.sigma5) return 0.0;
  const double g = exp(-tau * tau * geo.inv2s2);
  double sn, cs;
  sincos(geo.omega * tau, &sn, &cs);
  return -g * ((tau * geo.invs2) * cs + geo.omega * sn);
}

// Distance-derived quantities of sub-element j for the voxel p (mm): the path difference
// r - R is formed as (r^2 - R^2) / (r + R) with r^2 - R^2 = |p|^2 - 2 p.e + (|e|^2 - R^2), so
// no digits cancel when r is close to R.
__device__ inline void path(double px, double py, double pz, double p2, double ex, double ey,
                            double ez, double eoff, double R, double& r, double& dr) {
  const double q = p2 - 2.0 * (px * ex + py * ey + pz * ez) + eoff;
  r = sqrt(R * R + q);
  dr = q / (r + R);
}

// Window of every column: the samples within the kernel's reach of some arrival, over all
// sub-elements and basis quadrature points (qp: offsets in mm, x y z per point).
__global__ void k_support(int n, const int* __restrict__ cdx, const int* __restrict__ cdy,
                          const int* __restrict__ ck, const double* __restrict__ ex,
                          const double* __restrict__ ey, const double* __restrict__ ez,
                          const double* __restrict__ eoff, const double* __restrict__ qp,
                          Geo geo, int* __restrict__ lo, int* __restrict__ hi) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double dmin = 1e300, dmax = -1e300;
  for (int q = 0; q < geo.nq; ++q) {
    const double px = cdx[c] * geo.step + qp[3 * q], py = cdy[c] * geo.step + qp[3 * q + 1];
    const double pz = ((ck[c] - geo.nz / 2) * geo.dz_m) * 1e3 + qp[3 * q + 2];
    const double p2 = px * px + py * py + pz * pz;
    for (int j = 0; j < geo.M; ++j) {
      double r, dr;
      path(px, py, pz, p2, ex[j], ey[j], ez[j], eoff[j], geo.R, r, dr);
      const double d = dr / geo.cfs;
      dmin = fmin(dmin, d);
      dmax = fmax(dmax, d);
    }
  }
  const int h = geo.nt / 2;
  int a = (int)ceil(h + dmin - geo.reach);
  int b = (int)floor(h + dmax + geo.reach);
  a = max(a, 0);
  b = min(b, geo.nt - 1);
  lo[c] = a <= b ? a : -1;
  hi[c] = a <= b ? b : -1;
}

// One wave per stored column: for every basis quadrature point (qw: weights) the wave
// tabulates each sub-element's delay and weight in LDS, then each lane adds the
// sub-elements' terms for its time samples in FP64.
__global__ __launch_bounds__(64) void k_table(const int* __restrict__ cdx,
                                             const int* __restrict__ cdy,
                                             const int* __restrict__ ck,
                                             const int* __restrict__ lo,
                                             const long long* __restrict__ off,
                                             const double* __restrict__ ex,
                                             const double* __restrict__ ey,
                                             const double* __restrict__ ez,
                                             const double* __restrict__ eoff,
                                             const double* __restrict__ area,
                                             const double* __restrict__ qp,
                                             const double* __restrict__ qw, Geo geo,
                                             double* __restrict__ band) {
  extern __shared__ double sh[];  // [M] delay (samples), [M] weight dS / (2 pi r)
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  const int l = lo[c];
  const long long o = off[c];
  const int len = (int)(off[c + 1] - o);
  for (int i = lane; i < len; i += 64) band[o + i] = 0.0;
  for (int q = 0; q < geo.nq; ++q) {
    const double px = cdx[c] * geo.step + qp[3 * q], py = cdy[c] * geo.step + qp[3 * q + 1];
    const double pz = ((ck[c] - geo.nz / 2) * geo.dz_m) * 1e3 + qp[3 * q + 2];
    const double p2 = px * px + py * py + pz * pz;
    __syncthreads();  // the previous point's table is no longer read
    for (int j = lane; j < geo.M; j += 64) {
      double r, dr;
      path(px, py, pz, p2, ex[j], ey[j], ez[j], eoff[j], geo.R, r, dr);
      sh[j] = dr / geo.cfs;
      sh[geo.M + j] = area[j] / (2.0 * kPi * r);
    }
    __syncthreads();
    for (int i = lane; i < len; i += 64) {
      const double nrel = (double)(l + i - geo.nt / 2);
      double acc = 0.0;
      for (int j = 0; j < geo.M; ++j) {
        const double tau = nrel - sh[j];
        if (fabs(tau) <= geo.reach) acc += sh[geo.M + j] * deriv_kernel(tau, geo);
      }
      band[o + i] += qw[q] * acc;
    }
  }
}

// Fill band tiles: element (group, row m, entry j) of the pack is the table value at
//   forward: time n = TM tile + m, depth k = start + j
//   adjoint: depth k = TM tile + m, time n = start + j
// of the group's offset, or 0 outside the footprint, the band or the grid.
template <typename T>
__device__ inline T cvt(double v);
template <>
__device__ inline double cvt<double>(double v) { return v; }
template <>
__device__ inline float cvt<float>(double v) { return (float)v; }
template <>
__device__ inline uint16_t cvt<uint16_t>(double v) {  // bf16, round to nearest even
  float f = (float)v;
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline double table_value(int oi, int n, int k, int nz, int nt,
                                     const int* __restrict__ colidx, const int* __restrict__ lo,
                                     const long long* __restrict__ off,
                                     const double* __restrict__ band) {
  if (oi < 0 || n < 0 || n >= nt || k < 0 || k >= nz) return 0.0;
  const int c = colidx[(long long)oi * nz + k];
  if (c < 0) return 0.0;
  const int l = lo[c];
  const long long o = off[c];
  const long long len = off[c + 1] - o;
  if (n < l || n >= l + len) return 0.0;
  return band[o + (n - l)];
}

template <typename T>
__global__ void k_pack(long long total, int G, int TM, bool adjoint,
                       const int4* __restrict__ groups, int nz, int nt,
                       const int* __restrict__ colidx, const int* __restrict__ lo,
                       const long long* __restrict__ off, const double* __restrict__ band,
                       T* __restrict__ pack) {
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long grp = idx / ((long long)TM * G);
    const int m = (int)((idx / G) % TM);
    const int j = (int)(idx % G);
    const int4 gd = groups[grp];  // (offset index, start, tile, active)
    int n, k;
    if (!adjoint) {
      n = TM * gd.z + m;
      k = gd.y + j;
    } else {
      k = TM * gd.z + m;
      n = gd.y + j;
    }
    pack[idx] = cvt<T>(table_value(gd.x, n, k, nz, nt, colidx, lo, off, band));
  }
}

// Per (offset, 16-depth block) FP32 scale: the smallest power of two >= amax / 448 of the
// block's table values (powers of two let the kernel apply the scale inside the FP8 -> BF16
// conversion).
__global__ void k_block_scale(int n_off, int nz, const int* __restrict__ colidx,
                              const long long* __restrict__ off, const double* __restrict__ band,
                              float* __restrict__ scale) {
  const int nblk = (nz + 15) / 16;
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n_off * nblk) return;
  const int oi = id / nblk, blk = id % nblk;
  double amax = 0.0;
  for (int k = 16 * blk; k < min(nz, 16 * blk + 16); ++k) {
    const int c = colidx[(long long)oi * nz + k];
    if (c < 0) continue;
    for (long long i = off[c]; i < off[c + 1]; ++i) amax = fmax(amax, fabs(band[i]));
  }
  float sc = 1.0f;
  if (amax > 0.0) {
    int e;
    frexp(amax / 448.0, &e);            // amax / 448 in [2^(e-1), 2^e)
    sc = ldexpf(1.0f, e);
    if ((double)ldexpf(1.0f, e - 1) >= amax / 448.0) sc = ldexpf(1.0f, e - 1);
  }
  scale[id] = sc;
}

// FP8 pack of the block-scaled MFMA layout: entries are e4m3(value / scale) with the scale of
// the entry's (offset, 16-depth block); K-group q of the layout (operand position order:
// [bundle][lane group][8-byte slot]) fills, for each 16-row half h and row n, bytes
// [8 slot, + 8) of lane (n, lane group) in the half's 64 x 32-byte operand.
__global__ void k_pack_fp8(long long total, bool adjoint, const int4* __restrict__ groups, int nz,
                           int nt, const int* __restrict__ colidx, const int* __restrict__ lo,
                           const long long* __restrict__ off, const double* __restrict__ band,
                           const float* __restrict__ bscale, uint8_t* __restrict__ pack) {
  const int nblk = (nz + 15) / 16;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < total;
       idx += (long long)gridDim.x * blockDim.x) {
    const long long q = idx / (32 * 8);
    const int m = (int)((idx / 8) % 32);
    const int j = (int)(idx % 8);
    const long long bi = q / 16;
    const int ln = (int)((q % 16) / 4), slot = (int)(q % 4);
    const int h = m / 16, n = m % 16;
    const int4 gd = groups[q];  // (offset index, run start, tile, active)
    uint8_t code = 0;
    if (gd.x >= 0) {
      const int kblk = min(nblk - 1, adjoint ? 2 * gd.z + h : gd.y / 16);
      const float sc = bscale[(long long)gd.x * nblk + kblk];
      const int nn = adjoint ? gd.y + j : 32 * gd.z + m;
      const int k = adjoint ? 32 * gd.z + m : gd.y + j;
      const double v = table_value(gd.x, nn, k, nz, nt, colidx, lo, off, band);
      code = f32_to_e4m3((float)(v / sc));
    }
    pack[((bi * 2 + h) * 64 + ln * 16 + n) * 32 + slot * 8 + j] = code;
  }
}

template <typename T>
int alloc_copy(T** dst, const std::vector<T>& src, size_t& bytes) {
  const size_t b = std::max<size_t>(1, src.size()) * sizeof(T);
  AROAM_HIP(hipMalloc((void**)dst, b));
  bytes += b;
  if (!src.empty()) AROAM_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return AROAM_OK;
}

PadGeom pad_geom(const aroam_grid& g, int L, int BR = 1, int BC = 16, int CH = 0) {
  PadGeom p;
  p.K = g.k_half;
  p.nx = g.nx;
  p.ny = g.ny;
  p.ntx = (int)ceil_div(g.nx, 16);
  p.nxp = (int)round_up(g.nx, BC) + 2 * p.K;
  p.nyp = (int)round_up(g.ny, BR) + 2 * p.K;
  p.L = L;
  p.Lp = CH > 0 ? (int)round_up(L, CH) : (int)round_up(L, 8) + 8;
  return p;
}

// Mark the G-aligned runs of the inner axis that meet some column's band inside output
// tile t for offset oi (hit[q] = 1 for run q).  Returns whether any run was hit.
bool tile_hits(const Model& m, bool adjoint, int G, int TM, int t, int oi, std::vector<char>& hit) {
  const int nz = m.grid.nz;
  const int out_len = adjoint ? nz : m.grid.nt;
  const int r0 = TM * t, r1 = std::min(out_len, r0 + TM) - 1;
  std::fill(hit.begin(), hit.end(), 0);
  bool any = false;
  if (!adjoint) {
    for (int k = 0; k < nz; ++k) {
      const int lo = m.h_lo[(size_t)oi * nz + k];
      if (lo < 0) continue;
      const int hi = m.h_hi[(size_t)oi * nz + k];
      if (lo <= r1 && hi >= r0) {
        hit[k / G] = (char)(hit[k / G] | (1 << (k % G)));
        any = true;
      }
    }
  } else {
    for (int k = r0; k <= r1; ++k) {
      const int lo = m.h_lo[(size_t)oi * nz + k];
      if (lo < 0) continue;
      const int hi = m.h_hi[(size_t)oi * nz + k];
      for (int n = lo; n <= hi; ++n) hit[n / G] = (char)(hit[n / G] | (1 << (n % G)));
      any = true;
    }
  }
  return any;
}

// Build the K-group lists of one operator (direct form).  For output tile t (rows 16t ..
// 16t+15) and each offset, the K-groups are the G-aligned runs of the inner axis that meet
// some column's band inside the tile; runs with no band entry are skipped; each tile's list
// is padded with empty groups to a multiple of four (one bundle = four groups).
int build_layout(const Model& m, bool adjoint, int G, Layout& lay, size_t& bytes) {
  const aroam_grid& g = m.grid;
  const int K = m.K, W = 2 * K + 1, nz = g.nz, nt = g.nt;
  lay.G = G;
  lay.out_len = adjoint ? nz : nt;
  lay.n_tiles = (int)ceil_div(lay.out_len, kTile);
  lay.in = pad_geom(g, adjoint ? nt : nz);
  const int inner = adjoint ? nt : nz;
  std::vector<int4> groups;
  std::vector<int> meta;
  lay.h_tile_start.assign(lay.n_tiles + 1, 0);
  std::vector<char> hit((size_t)ceil_div(inner, G) + 1);
  for (int t = 0; t < lay.n_tiles; ++t) {
    lay.h_tile_start[t] = (int)(groups.size() / kLaneGroups);
    for (int oi = 0; oi < m.n_off; ++oi) {
      const int dy = oi / W - K, dx = oi % W - K;
      if (!tile_hits(m, adjoint, G, kTile, t, oi, hit)) continue;
      for (size_t q = 0; q < hit.size(); ++q) {
        if (!hit[q]) continue;
        const int start = (int)q * G;
        groups.push_back(make_int4(oi, start, t, 1));
        const long long delta =
            adjoint ? ((long long)(-dy) * lay.in.nxp - dx) * lay.in.Lp + start
                    : ((long long)dy * lay.in.nxp + dx) * lay.in.Lp + start;
        meta.push_back((int)delta);
      }
    }
    while (groups.size() % kLaneGroups) {
      groups.push_back(make_int4(-1, 0, t, 0));
      meta.push_back(0);
    }
  }
  lay.h_tile_start[lay.n_tiles] = (int)(groups.size() / kLaneGroups);
  lay.n_bundles = (long long)groups.size() / kLaneGroups;
  lay.mac_exec = lay.n_bundles * kLaneGroups * kTile * G * (long long)g.ny * 16 * lay.in.ntx;
  AROAM_CHECK(lay.in.elems() < (1ll << 31), AROAM_EINVAL,
              "grid too large for 32-bit operand offsets (%lld padded elements)", lay.in.elems());
  AROAM_TRY(alloc_copy(&lay.d_tile_start, lay.h_tile_start, bytes));
  AROAM_TRY(alloc_copy(&lay.d_meta, meta, bytes));
  AROAM_TRY(alloc_copy(&lay.d_groups, groups, bytes));
  return AROAM_OK;
}

// LDS-staged form (see Layout).  For tile t, the hit runs of every lateral offset are
// grouped by chunk (CH inner entries = CH / G runs) and by input row offset; each non-empty
// (chunk, row offset) is one stage unit whose K-groups (dx, run) are packed four to a
// bundle.  Units are ordered by chunk, then by ascending row offset, so that the LDS rows
// form a ring: a unit only loads the input rows that the previous unit of the same chunk did
// not hold (one row when the offset steps by one).  The row range to load is stored per unit
// as [lo, hi) in patch-relative padded rows G = row offset + K + r.  A null K-group reads
// staged column 0 and multiplies zero table entries.
// LDS bank model of a bundle's position-fragment reads, measured on gfx950 with a probe of
// single-lane-pair collisions and the SQ_LDS_BANK_CONFLICT counter: a 64-lane 16-byte LDS read
// is served in four passes of 16 lanes x 16 bytes over the 64 banks.  Lane l belongs to half
// l / 32 and to the pass given by the parity of the bits of (l / 4) mod 8, so within a half
// the passes take lanes n in {0-3, 12-15} of lane group g (even) with n in {4-11} of g + 1,
// and the converse.  A pass is conflict-free when its 16 lanes hit 16 distinct 16-byte bank
// groups.  Lane (n, g) of a bundle reads vector run_g of staged column c + n + col_g; with a
// column stride of 80 bytes (5 groups of 16 bytes) its bank group is 5 (c + n + col_g) + run_g
// (mod 16).  The patch offset c and the row start shift all lanes of a read alike.
constexpr int kColumnGroups = kColumnBytes / 16;  // LDS column stride in 16-byte groups

bool pair_conflict_free(int col_a, int run_a, int col_b, int run_b) {
  static const int lo_hi[8] = {0, 1, 2, 3, 12, 13, 14, 15};
  static const int mid[8] = {4, 5, 6, 7, 8, 9, 10, 11};
  for (int pass = 0; pass < 2; ++pass) {
    const int* na = pass ? mid : lo_hi;  // lanes of the even group in this pass
    const int* nb = pass ? lo_hi : mid;  // lanes of the odd group
    unsigned used = 0;
    for (int i = 0; i < 8; ++i) {
      const int ba = (kColumnGroups * (na[i] + col_a) + run_a) & 15;
      const int bb = (kColumnGroups * (nb[i] + col_b) + run_b) & 15;
      used |= (1u << ba) | (1u << bb);
    }
    if (used != 0xffffu) return false;
  }
  return true;
}

// One K-group of a stage unit: its group record, staged column offset, vector run, and the
// 16-row halves of the tile its band reaches (bit h for half h).
struct UnitEntry {
  int4 group;
  int col, run;
  int mask;
};

// Pair the K-groups of one stage unit so that bundle slots (0, 1) and (2, 3) read the LDS
// without bank conflicts wherever possible: a greedy matching over the 64 classes
// (column mod 16, run) that pairs the most constrained class first.  K-groups left without a
// partner are paired with each other; an odd one out gets a zero padding K-group of a
// matching class.  The result has an even number of entries; with pad4 it is padded to a
// multiple of four (whole bundles).
struct CompatTable {
  std::vector<int> partners[64];  // classes whose K-groups pair with this one without conflicts
  CompatTable() {
    for (int a = 0; a < 64; ++a)
      for (int b = 0; b < 64; ++b)
        if (pair_conflict_free(a >> 2, a & 3, b >> 2, b & 3)) partners[a].push_back(b);
  }
};

std::vector<UnitEntry> pair_unit(const std::vector<UnitEntry>& in, int maxcol, int t,
                                 bool pad4 = true) {
  static const CompatTable table;  // classes (column mod 16, run)
  std::vector<int> cls_items[64];
  for (int i = (int)in.size() - 1; i >= 0; --i)
    cls_items[((in[i].col & 15) << 2) | in[i].run].push_back(i);
  auto avail = [&](int a) {
    int n = 0;
    for (int b : table.partners[a]) n += (int)cls_items[b].size() - (a == b ? 1 : 0);
    return n;
  };
  std::vector<UnitEntry> out;
  out.reserve(in.size() + 4);
  std::vector<int> left;
  for (;;) {
    int a = -1, best = 1 << 30;
    for (int c = 0; c < 64; ++c)
      if (!cls_items[c].empty()) {
        const int v = avail(c);
        if (v < best) best = v, a = c;
      }
    if (a < 0) break;
    const int ia = cls_items[a].back();
    cls_items[a].pop_back();
    int b = -1, bbest = 1 << 30;
    for (int c : table.partners[a])
      if (!cls_items[c].empty()) {
        const int v = avail(c);
        if (v < bbest) bbest = v, b = c;
      }
    if (b < 0) {
      left.push_back(ia);
      continue;
    }
    const int ib = cls_items[b].back();
    cls_items[b].pop_back();
    out.push_back(in[ia]);
    out.push_back(in[ib]);
  }
  const UnitEntry pad0{make_int4(-1, 0, t, 0), 0, 0, 0};
  for (size_t i = 0; i + 1 < left.size(); i += 2) {
    out.push_back(in[left[i]]);
    out.push_back(in[left[i + 1]]);
  }
  if (left.size() % 2) {
    const UnitEntry& e = in[left.back()];
    UnitEntry p = pad0;
    bool found = false;
    for (int c = 0; c <= maxcol && !found; ++c)
      for (int r = 0; r < 4 && !found; ++r)
        if (pair_conflict_free(e.col, e.run, c, r)) {
          p.col = c;
          p.run = r;
          found = true;
        }
    out.push_back(e);
    out.push_back(p);
  }
  if (pad4 && out.size() % 4) {
    UnitEntry p = pad0;
    for (int r = 1; r < 4; ++r)
      if (pair_conflict_free(0, 0, 0, r)) {
        p.run = r;
        break;
      }
    out.push_back(pad0);
    out.push_back(p);
  }
  return out;
}

// Order a stage unit's K-groups into bundles.  With two 16-row halves per tile, K-groups
// are first grouped by the halves their bands reach, so that most bundles reach only one
// half and the kernel skips the other half's MFMAs; with one half (FP32, runs of 4), by the
// entries of their run that the band reaches in the tile, so that the kernel skips the
// MFMAs of entries no K-group of the bundle reaches.  Each group is paired for the LDS as
// above.
std::vector<UnitEntry> order_unit(const std::vector<UnitEntry>& in, int maxcol, int t, int NH) {
  std::vector<UnitEntry> out;
  const int nmask = NH > 1 ? 1 << NH : 16;  // half masks, or masks of a run's four entries
  for (int mask = 1; mask < nmask; ++mask) {
    std::vector<UnitEntry> cls;
    for (const UnitEntry& e : in)
      if (e.mask == mask) cls.push_back(e);
    if (cls.empty()) continue;
    for (const UnitEntry& e : pair_unit(cls, maxcol, t, false)) out.push_back(e);
  }
  if (out.size() % 4) {
    UnitEntry p{make_int4(-1, 0, t, 0), 0, 0, 0};
    for (int r = 1; r < 4; ++r)
      if (pair_conflict_free(0, 0, 0, r)) {
        p.run = r;
        break;
      }
    out.push_back(UnitEntry{make_int4(-1, 0, t, 0), 0, 0, 0});
    out.push_back(p);
  }
  return out;
}

// Plan the staged launch of a layout (plan.h) and upload the pieces.  The partial slots are
// capped at 1 GiB.
int plan_pieces(Layout& lay, const std::vector<int>& tile_units,
                const std::vector<std::vector<int>>& chunk_starts,
                const std::vector<double>& unit_work, int slots, size_t& bytes) {
  const double slot_bytes = (double)lay.TM * kPatchRows * kPatchCols * sizeof(float);
  const LaunchPlan plan = plan_launch(tile_units, chunk_starts, unit_work, lay.n_patches, slots,
                                      /*allow_cut=*/true, slot_bytes, (double)(1ll << 30));
  std::vector<int4> pieces;
  for (const PlanPiece& p : plan.pieces) pieces.push_back(make_int4(p.tile, p.u0, p.u1, p.slot));
  std::vector<int2> split(lay.n_tiles);
  for (int t = 0; t < lay.n_tiles; ++t)
    split[t] = make_int2(plan.tile_pieces[t], plan.tile_first_slot[t]);
  lay.n_pieces = (int)pieces.size();
  lay.n_slots = plan.n_slots;
  AROAM_TRY(alloc_copy(&lay.d_pieces, pieces, bytes));
  AROAM_TRY(alloc_copy(&lay.d_tile_split, split, bytes));
  return AROAM_OK;
}

int build_staged_layout(const Model& m, bool adjoint, int G, int TM, int CH, int BR, int BC,
                        int esize, Layout& lay, size_t& bytes) {
  const aroam_grid& g = m.grid;
  const int K = m.K, W = 2 * K + 1, nz = g.nz, nt = g.nt;
  lay.G = G;
  lay.TM = TM;
  lay.staged = true;
  lay.CH = CH;
  lay.BR = BR;
  lay.BC = BC;
  lay.NCOL = BC + 2 * K;
  AROAM_CHECK(CH * esize == kChunkBytes && G * esize == 16, AROAM_EINVAL,
              "staged layout needs 64-byte chunks of four 16-byte runs");
  lay.CS = kColumnBytes / esize;  // 64 bytes of chunk + 16 bytes of padding
  lay.out_len = adjoint ? nz : nt;
  lay.n_tiles = (int)ceil_div(lay.out_len, TM);
  lay.in = pad_geom(g, adjoint ? nt : nz, BR, BC, CH);
  lay.lds_bytes = (size_t)(BR + 1) * lay.NCOL * lay.CS * esize;  // BR rows + one free slot
  AROAM_CHECK(BR == kPatchRows && BC == kPatchCols && (long long)lay.lds_bytes == staged_lds_bytes(K),
              AROAM_EINVAL, "staged layout shape differs from the LDS stage's");
  const int inner = adjoint ? nt : nz;
  const int nq = (int)ceil_div(inner, G);
  const int qpc = CH / G;  // runs per chunk
  const int nch = (int)ceil_div(inner, CH);
  std::vector<int4> groups, units;
  std::vector<int2> urows;
  std::vector<int> meta, tile_units(lay.n_tiles + 1, 0);
  std::vector<std::vector<char>> hits(W, std::vector<char>((size_t)nq + 1));
  const int NH = TM / kTile;  // 16-row halves per tile
  std::vector<std::vector<char>> hhits(NH > 1 ? (size_t)W * NH : 0,
                                       std::vector<char>((size_t)nq + 1));
  std::vector<int> bmask;
  std::vector<char> dx_any(W);
  std::vector<std::vector<int>> chunk_starts(lay.n_tiles);  // first unit of each chunk
  std::vector<double> unit_work;                           // MFMA halves a unit issues
  // per (chunk, row-offset slot) list of the current tile's K-groups
  std::vector<std::vector<UnitEntry>> per((size_t)nch * W);
  for (int t = 0; t < lay.n_tiles; ++t) {
    tile_units[t] = (int)units.size();
    for (auto& v : per) v.clear();
    for (int a = 0; a < W; ++a) {
      // input row offset: +dy for the forward, -dy for the adjoint; slot = offset + K
      const int slot = adjoint ? (W - 1 - a) : a;
      for (int b = 0; b < W; ++b) {
        dx_any[b] = tile_hits(m, adjoint, G, TM, t, a * W + b, hits[b]);
        if (NH > 1 && dx_any[b])
          for (int h = 0; h < NH; ++h)
            tile_hits(m, adjoint, G, kTile, t * NH + h, a * W + b, hhits[(size_t)b * NH + h]);
      }
      for (int b = 0; b < W; ++b) {
        if (!dx_any[b]) continue;
        const int col = adjoint ? (W - 1 - b) : b;  // input column offset + K
        for (int q = 0; q < nq; ++q) {
          if (!hits[b][q]) continue;
          const int c = q / qpc;
          // two row halves: the halves the K-group's band reaches; one half (G = 4): the
          // entries of the run the band reaches in this tile (one MFMA each)
          int mask = (unsigned char)hits[b][q] & 15;
          if (NH > 1) {
            mask = 0;
            for (int h = 0; h < NH; ++h) mask |= hhits[(size_t)b * NH + h][q] ? 1 << h : 0;
          }
          per[(size_t)c * W + slot].push_back(
              UnitEntry{make_int4(a * W + b, q * G, t, 1), col, (q * G - c * CH) / G, mask});
        }
      }
    }
    for (int c = 0; c < nch; ++c) {
      int prevR = -1;
      for (int R = 0; R < W; ++R) {
        auto& lst = per[(size_t)c * W + R];
        if (lst.empty()) continue;
        if (prevR < 0) chunk_starts[t].push_back((int)units.size());
        const size_t first = groups.size();
        const std::vector<UnitEntry> ord = order_unit(lst, 2 * K, t, NH);
        for (size_t i = 0; i < ord.size(); ++i) {
          const UnitEntry& e = ord[i];
          groups.push_back(e.group);
          meta.push_back(e.col * lay.CS + e.run * G);
          if (i % kLaneGroups == 0) bmask.push_back(0);
          bmask.back() |= e.mask;
        }
        // the bundle's mask rides in the top bits of its K-groups' offsets
        for (size_t q = first; q < groups.size(); ++q)
          meta[q] = (int)((unsigned)meta[q] | ((unsigned)bmask[q / kLaneGroups] << kMetaMaskShift));
        const int lo = (prevR < 0 || R >= prevR + BR) ? R : prevR + BR;
        units.push_back(make_int4(R - K, c * CH, (int)(first / kLaneGroups),
                                  (int)(groups.size() / kLaneGroups)));
        urows.push_back(make_int2(lo, R + BR));
        double w = 0;  // MFMA halves (one-half tiles: quarters of a bundle's four MFMAs)
        for (size_t b = first / kLaneGroups; b < groups.size() / kLaneGroups; ++b)
          w += __builtin_popcount((unsigned)bmask[b]) * (NH > 1 ? 1.0 : 0.25);
        unit_work.push_back(w);
        prevR = R;
      }
    }
  }
  tile_units[lay.n_tiles] = (int)units.size();
  lay.n_units = (long long)units.size();
  lay.n_bundles = (long long)groups.size() / kLaneGroups;
  // MACs the kernel issues: per bundle, its 16-row halves times the positions of every patch.
  // The FP32 kernel (esize 4) leaves out two things: a wave's MFMAs for a unit whose row
  // offset makes its BR / 4 rows read only the zero rows around the grid, and the second
  // 16-position tile column of a patch that holds at most 16 scan columns.
  long long mac_exec = 0;
  {
    const int RW = BR / 4;
    const long long cols =
        esize == 4 && BC == 32 && g.nx % BC > 0 && g.nx % BC <= 16
            ? (long long)(g.nx / BC) * BC + 16
            : round_up(g.nx, BC);
    std::vector<long long> rows_live(W, 0);  // computed rows per row offset dy (index dy + K)
    for (int d = 0; d < W; ++d)
      for (int py0 = 0; py0 < g.ny; py0 += BR)
        for (int w = 0; w < 4; ++w) {
          const int src = py0 + w * RW + d - K;
          if (esize != 4 || (src + RW > 0 && src < g.ny)) rows_live[d] += RW;
        }
    // per position, a bundle issues 16 rows x 4 K-groups x G entries per reached half, or,
    // with one half (G = 4), 16 rows x 4 K-groups for each of its four MFMAs it issues
    const long long per_bit = (long long)kLaneGroups * kTile * (NH > 1 ? G : 1);
    for (size_t u = 0; u < units.size(); ++u) {
      long long bits = 0;
      for (int b = units[u].z; b < units[u].w; ++b) bits += __builtin_popcount((unsigned)bmask[b]);
      mac_exec += bits * rows_live[units[u].x + K];
    }
    mac_exec *= per_bit * cols;
  }
  lay.mac_exec = mac_exec;
  AROAM_CHECK(lay.in.elems() < (1ll << 31), AROAM_EINVAL,
              "grid too large for 32-bit operand offsets (%lld padded elements)", lay.in.elems());
  AROAM_TRY(alloc_copy(&lay.d_units, units, bytes));
  AROAM_TRY(alloc_copy(&lay.d_ucols, urows, bytes));
  AROAM_TRY(alloc_copy(&lay.d_meta, meta, bytes));
  AROAM_TRY(alloc_copy(&lay.d_groups, groups, bytes));
  lay.h_tile_start = tile_units;
  lay.n_patches = (int)(ceil_div(g.ny, BR) * ceil_div(g.nx, BC));
  int cus = 0;
  AROAM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m.device));
  return plan_pieces(lay, tile_units, chunk_starts, unit_work, 3 * std::max(cus, 1), bytes);
}

// ---- FP8 layouts: bundles of the block-scaled FP8 MFMA ---------------------------------
// v_mfma_scale_f32_16x16x128_f8f6f4 multiplies 16 rows by 128 K per 16 positions; lane
// (n, g) holds 32 bytes of row n (A) or position n (B), and each of the four scale blocks of
// 32 K takes the scale byte (E8M0, 2^(byte - 127)) of one lane group.  A bundle holds 16
// K-groups of 8 entries: K-group i of scale block b sits in lane group kFp8Lane[b][i], bytes
// [8 kFp8Slot[b][i], + 8) of its 32, and lane group kFp8ScaleLane[b] carries block b's scale.
// The four K-groups of a block share one table scale (and the unit's operand scale).
bool fp8_key_less(const int4& a, const int4& b) {
  return a.x != b.x ? a.x < b.x : a.y != b.y ? a.y < b.y : a.z < b.z;
}

int build_fp8_layout(const Model& m, bool adjoint, const std::vector<float>& bscale, Layout& lay,
                     size_t& bytes) {
  const aroam_grid& g = m.grid;
  const int K = m.K, W = 2 * K + 1, nz = g.nz, nt = g.nt;
  const int G = 8, TM = kTileRows8, CH = kChunkBytes, BR = kPatchRows, BC = kPatchCols;
  const int nblk = (int)ceil_div(nz, 16);
  lay.G = G;
  lay.TM = TM;
  lay.staged = true;
  lay.CH = CH;
  lay.BR = BR;
  lay.BC = BC;
  lay.NCOL = BC + 2 * K;
  lay.CS = kColumnBytes;  // one byte per entry
  lay.out_len = adjoint ? nz : nt;
  lay.n_tiles = (int)ceil_div(lay.out_len, TM);
  lay.in = pad_geom(g, adjoint ? nt : nz, BR, BC, CH);
  lay.lds_bytes = (size_t)(BR + 1) * lay.NCOL * lay.CS;
  AROAM_CHECK((long long)lay.lds_bytes == staged_lds_bytes(K), AROAM_EINVAL,
              "FP8 layout shape differs from the LDS stage's");
  const int inner = adjoint ? nt : nz;
  const int nq = (int)ceil_div(inner, G);
  const int qpc = CH / G;
  const int nch = (int)ceil_div(inner, CH);
  // E8M0 byte of a table block scale (a power of two; 1 for an empty block)
  auto e8 = [&](int oi, int blk) {
    int e = 0;
    std::frexp((double)bscale[(size_t)oi * nblk + std::min(blk, nblk - 1)], &e);
    return std::max(0, std::min(254, e - 1 + 127));
  };
  std::vector<int4> groups, units;  // groups in operand position order: [bundle][lane][slot]
  std::vector<int2> urows;
  std::vector<int> rec, bmask, tile_units(lay.n_tiles + 1, 0);
  std::vector<std::vector<char>> hits(W, std::vector<char>((size_t)nq + 1));
  std::vector<std::vector<char>> hhits((size_t)W * 2, std::vector<char>((size_t)nq + 1));
  std::vector<char> dx_any(W);
  std::vector<std::vector<int>> chunk_starts(lay.n_tiles);
  std::vector<double> unit_work;
  struct Entry {
    int4 group;
    int off;   // LDS offset of the K-group's run
    int4 key;  // (half mask, scale byte of half 0, of half 1)
  };
  std::vector<std::vector<Entry>> per((size_t)nch * W);
  const int4 null_group = make_int4(-1, 0, 0, 0);
  for (int t = 0; t < lay.n_tiles; ++t) {
    tile_units[t] = (int)units.size();
    for (auto& v : per) v.clear();
    for (int a = 0; a < W; ++a) {
      const int slot_r = adjoint ? (W - 1 - a) : a;
      for (int b = 0; b < W; ++b) {
        dx_any[b] = tile_hits(m, adjoint, G, TM, t, a * W + b, hits[b]);
        if (dx_any[b])
          for (int h = 0; h < 2; ++h)
            tile_hits(m, adjoint, G, kTile, 2 * t + h, a * W + b, hhits[(size_t)b * 2 + h]);
      }
      for (int b = 0; b < W; ++b) {
        if (!dx_any[b]) continue;
        const int col = adjoint ? (W - 1 - b) : b;
        const int oi = a * W + b;
        for (int q = 0; q < nq; ++q) {
          if (!hits[b][q]) continue;
          const int c = q / qpc;
          const int mask = (hhits[(size_t)b * 2][q] ? 1 : 0) | (hhits[(size_t)b * 2 + 1][q] ? 2 : 0);
          const int s0 = adjoint ? e8(oi, 2 * t) : e8(oi, (q * G) / 16);
          const int s1 = adjoint ? e8(oi, 2 * t + 1) : s0;
          per[(size_t)c * W + slot_r].push_back(
              Entry{make_int4(oi, q * G, t, 1), col * lay.CS + (q % qpc) * G,
                    make_int4(mask, s0, s1, 0)});
        }
      }
    }
    for (int c = 0; c < nch; ++c) {
      int prevR = -1;
      for (int R = 0; R < W; ++R) {
        auto& lst = per[(size_t)c * W + R];
        if (lst.empty()) continue;
        if (prevR < 0) chunk_starts[t].push_back((int)units.size());
        const int first_bundle = (int)(groups.size() / 16);
        // scale blocks: K-groups of equal key, four at a time (a short block is padded with
        // null K-groups, whose table entries are zero).  A block's K-groups 0, 1 and 2, 3 sit
        // in two lane groups at the same two 8-byte slots, and the 32 lanes of a pass of an
        // 8-byte LDS read hit distinct banks only when those two lane groups' runs (8-byte
        // steps within a column of 80 bytes) differ in parity: a block takes two K-groups of
        // even and two of odd run where the class has them, evens first.
        std::stable_sort(lst.begin(), lst.end(),
                         [](const Entry& x, const Entry& y) { return fp8_key_less(x.key, y.key); });
        std::vector<std::vector<Entry>> blocks;
        for (size_t i = 0; i < lst.size();) {
          size_t j = i;
          std::vector<Entry> ev, od;
          while (j < lst.size() && !fp8_key_less(lst[i].key, lst[j].key) &&
                 !fp8_key_less(lst[j].key, lst[i].key)) {
            ((lst[j].off / G) % 2 ? od : ev).push_back(lst[j]);
            ++j;
          }
          const Entry null_even{null_group, 0, lst[i].key}, null_odd{null_group, G, lst[i].key};
          size_t a = 0, b = 0;
          while (a < ev.size() || b < od.size()) {
            std::vector<Entry> blk;
            // two evens then two odds when both are left, else four of what is left
            const bool both = ev.size() - a >= 2 && od.size() - b >= 2;
            for (int k = 0; k < 4; ++k) {
              const bool want_even = both ? k < 2 : (a < ev.size());
              if (want_even && a < ev.size()) blk.push_back(ev[a++]);
              else if (!want_even && b < od.size()) blk.push_back(od[b++]);
              else if (a < ev.size()) blk.push_back(ev[a++]);
              else if (b < od.size()) blk.push_back(od[b++]);
              else blk.push_back(k < 2 ? null_even : null_odd);
            }
            blocks.push_back(blk);
          }
          i = j;
        }
        // bundles: four blocks of one half mask (blocks are sorted by mask first)
        for (size_t i = 0; i < blocks.size();) {
          const int mask = blocks[i][0].key.x;
          std::vector<std::vector<Entry>> bun;
          while (i < blocks.size() && bun.size() < 4 && blocks[i][0].key.x == mask)
            bun.push_back(blocks[i++]);
          while (bun.size() < 4)
            bun.push_back(std::vector<Entry>(4, Entry{null_group, 0, make_int4(mask, 127, 127, 0)}));
          const size_t base = groups.size();
          groups.resize(base + 16, null_group);
          std::vector<int> off(16, 0), sc(4, 0);
          for (int bb = 0; bb < 4; ++bb) {
            for (int k = 0; k < 4; ++k) {
              const int pos = kFp8Lane[bb][k] * 4 + kFp8Slot[bb][k];
              groups[base + pos] = bun[bb][k].group;
              if (groups[base + pos].x >= 0) groups[base + pos].z = t;
              off[pos] = bun[bb][k].off;
            }
            sc[kFp8ScaleLane[bb]] = bun[bb][0].key.y | (bun[bb][0].key.z << 8);
          }
          for (int ln = 0; ln < 4; ++ln) {
            rec.push_back(off[4 * ln] | (off[4 * ln + 1] << 16));
            rec.push_back(off[4 * ln + 2] | (off[4 * ln + 3] << 16));
            rec.push_back(sc[ln]);
            rec.push_back(ln == 0 ? mask : 0);
          }
          bmask.push_back(mask);
        }
        const int lo = (prevR < 0 || R >= prevR + BR) ? R : prevR + BR;
        const int nb = (int)(groups.size() / 16);
        units.push_back(make_int4(R - K, c * CH, first_bundle, nb));
        urows.push_back(make_int2(lo, R + BR));
        double w = 0;
        for (int bi = first_bundle; bi < nb; ++bi) w += __builtin_popcount((unsigned)bmask[bi]);
        unit_work.push_back(w);
        prevR = R;
      }
    }
  }
  tile_units[lay.n_tiles] = (int)units.size();
  lay.n_units = (long long)units.size();
  lay.n_bundles = (long long)groups.size() / 16;
  long long halves = 0;
  for (int bm : bmask) halves += __builtin_popcount((unsigned)bm);
  lay.mac_exec = halves * 16LL * kTile * G * (round_up(g.ny, BR) * round_up(g.nx, BC));
  AROAM_CHECK(lay.in.elems() < (1ll << 31), AROAM_EINVAL,
              "grid too large for 32-bit operand offsets (%lld padded elements)", lay.in.elems());
  AROAM_CHECK(lay.NCOL * lay.CS < 65536, AROAM_EINVAL, "LDS offsets exceed 16 bits");
  AROAM_TRY(alloc_copy(&lay.d_units, units, bytes));
  AROAM_TRY(alloc_copy(&lay.d_ucols, urows, bytes));
  AROAM_TRY(alloc_copy(&lay.d_meta, rec, bytes));
  AROAM_TRY(alloc_copy(&lay.d_groups, groups, bytes));
  lay.h_tile_start = tile_units;
  lay.n_patches = (int)(ceil_div(g.ny, BR) * ceil_div(g.nx, BC));
  int cus = 0;
  AROAM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, m.device));
  return plan_pieces(lay, tile_units, chunk_starts, unit_work, 3 * std::max(cus, 1), bytes);
}

template <typename T>
int pack_dtype(const Model& m, const Layout& lay, bool adjoint, Pack& p, hipStream_t st,
               size_t& bytes) {
  const long long total = lay.n_bundles * kLaneGroups * lay.TM * lay.G;
  p.bytes = std::max<long long>(1, total) * sizeof(T);
  AROAM_HIP(hipMalloc(&p.d, p.bytes));
  bytes += p.bytes;
  if (total > 0) {
    const int blocks = (int)std::min<long long>(ceil_div(total, 256), 1 << 16);
    hipLaunchKernelGGL(k_pack<T>, dim3(blocks), dim3(256), 0, st, total, lay.G, lay.TM, adjoint,
                       lay.d_groups, m.grid.nz, m.grid.nt, m.d_colidx, m.d_lo, m.d_off,
                       m.d_band, (T*)p.d);
    AROAM_HIP(hipGetLastError());
  }
  return AROAM_OK;
}

int pack_fp8(const Model& m, const Layout& lay, bool adjoint, const float* bscale, Pack& p,
             hipStream_t st, size_t& bytes) {
  const long long total = lay.n_bundles * 16 * 32 * 8;
  p.bytes = std::max<long long>(1, total);
  AROAM_HIP(hipMalloc(&p.d, p.bytes));
  bytes += p.bytes;
  if (total > 0) {
    const int blocks = (int)std::min<long long>(ceil_div(total, 256), 1 << 16);
    hipLaunchKernelGGL(k_pack_fp8, dim3(blocks), dim3(256), 0, st, total, adjoint, lay.d_groups,
                       m.grid.nz, m.grid.nt, m.d_colidx, m.d_lo, m.d_off, m.d_band, bscale,
                       (uint8_t*)p.d);
    AROAM_HIP(hipGetLastError());
  }
  return AROAM_OK;
}

// Block scales on the device, their copy on the host (the layout groups K-groups by scale),
// the FP8 layouts of both directions, and their packs.
int pack_all_fp8(Model& m, hipStream_t st, size_t& bytes) {
  const int nblk = (int)ceil_div(m.grid.nz, 16);
  float* bscale = nullptr;
  const long long nb = (long long)m.n_off * nblk;
  AROAM_HIP(hipMalloc((void**)&bscale, std::max<long long>(1, nb) * sizeof(float)));
  hipLaunchKernelGGL(k_block_scale, dim3((unsigned)ceil_div(nb, 256)), dim3(256), 0, st, m.n_off,
                     m.grid.nz, m.d_colidx, m.d_off, m.d_band, bscale);
  int rc = hipGetLastError() == hipSuccess ? AROAM_OK : AROAM_EDEVICE;
  std::vector<float> h_scale((size_t)std::max<long long>(1, nb));
  if (!rc && (hipMemcpyAsync(h_scale.data(), bscale, nb * sizeof(float), hipMemcpyDeviceToHost,
                             st) != hipSuccess ||
              hipStreamSynchronize(st) != hipSuccess))
    rc = AROAM_EDEVICE;
  if (!rc) rc = build_fp8_layout(m, false, h_scale, m.f8f, bytes);
  if (!rc) rc = build_fp8_layout(m, true, h_scale, m.f8a, bytes);
  if (!rc) rc = pack_fp8(m, m.f8f, false, bscale, m.fwd_pack[AROAM_FP8E4M3], st, bytes);
  if (!rc) rc = pack_fp8(m, m.f8a, true, bscale, m.adj_pack[AROAM_FP8E4M3], st, bytes);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = AROAM_EDEVICE;
  (void)hipFree(bscale);
  if (rc) set_error("FP8 packing failed");
  return rc;
}

int set_columns(Model& m, const std::vector<int>& foi, const std::vector<int>& fk,
                const std::vector<int>& fsrc, const std::vector<int>& stored,
                const std::vector<int>& src_lo, const std::vector<int>& src_hi,
                const std::vector<int>& slo, const std::vector<long long>& soff,
                const std::vector<double>& values, size_t& bytes);
int pack_fp(Model& m, hipStream_t st, size_t& bytes);

// q-point Gauss-Legendre nodes and weights on [-1, 1]: roots of the Legendre polynomial P_q
// by Newton's method from the usual cosine guesses, weights 2 / ((1 - x^2) P_q'(x)^2).
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  for (int i = 0; i < q; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (q + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q == 1 ? 1.0 : q * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= q; ++k) {
      const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = q == 1 ? 1.0 : q * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Quadrature of the voxel basis (Methods, Forward modeling: trilinear interpolation of
// neighbouring voxel values): offsets (mm, x y z per point) and weights.  The point voxel is
// one point at the centre.  The trilinear basis is the product of tents 1 - |t| along x, y
// and z (t in voxel spacings); each axis takes q Gauss-Legendre points on each half with the
// tent folded into the weights, which sum to one.
void basis_points(const aroam_grid& g, std::vector<double>& qp, std::vector<double>& qw) {
  qp.clear();
  qw.clear();
  if (g.voxel_basis == 0) {
    qp = {0.0, 0.0, 0.0};
    qw = {1.0};
    return;
  }
  const int q = g.basis_quad > 0 ? g.basis_quad : 3;
  std::vector<double> x, w, t, wt;
  gauss_legendre(q, x, w);
  // nodes t on [0, 1] in ascending order with weights w/2 (1 - t)
  std::vector<std::pair<double, double>> half(q);
  for (int i = 0; i < q; ++i) {
    const double th = 0.5 * (x[i] + 1.0);
    half[i] = {th, 0.5 * w[i] * (1.0 - th)};
  }
  std::sort(half.begin(), half.end());
  std::vector<double> th(q), wh(q);
  for (int i = 0; i < q; ++i) th[i] = half[i].first, wh[i] = half[i].second;
  for (int i = q - 1; i >= 0; --i) t.push_back(-th[i]), wt.push_back(wh[i]);
  for (int i = 0; i < q; ++i) t.push_back(th[i]), wt.push_back(wh[i]);
  const double step = g.step_m * kMM, dz = g.dz_m * kMM;
  for (size_t a = 0; a < t.size(); ++a)
    for (size_t b = 0; b < t.size(); ++b)
      for (size_t c = 0; c < t.size(); ++c) {
        qp.push_back(t[a] * step);
        qp.push_back(t[b] * step);
        qp.push_back(t[c] * dz);
        qw.push_back(wt[a] * wt[b] * wt[c]);
      }
}

int build_impl(Model& m, hipStream_t st) {
  const aroam_sensor& s = m.sensor;
  const aroam_grid& g = m.grid;
  const int K = m.K, W = 2 * K + 1, nz = g.nz;
  size_t bytes = 0;

  std::vector<double> ex, ey, ez, area;
  make_elements(s, ex, ey, ez, area);
  m.M = (int)area.size();
  AROAM_CHECK(m.M <= kMaxElements, AROAM_EINVAL, "%d sub-elements exceed the limit of %d", m.M,
              kMaxElements);
  m.R_mm = s.radius_m * kMM;
  std::vector<double> eoff(m.M);
  for (int j = 0; j < m.M; ++j)
    eoff[j] = ex[j] * ex[j] + ey[j] * ey[j] + ez[j] * ez[j] - m.R_mm * m.R_mm;
  const double sigma_f = s.f0_hz * s.frac_bw / (2.0 * std::sqrt(2.0 * std::log(2.0)));
  m.sigma = g.fs_hz / (2.0 * kPi * sigma_f);
  m.omega = 2.0 * kPi * s.f0_hz / g.fs_hz;
  m.cfs = g.c_mps * kMM / g.fs_hz;
  m.step_mm = g.step_m * kMM;
  m.dz_mm = g.dz_m * kMM;

  // Footprint columns, in (dy, dx, k) order.  The sub-element set and the footprint are
  // invariant under the square's symmetry group (the sensor's axial symmetry, Methods,
  // scanning symmetries), so H[dx, dy] = H[+-dx, +-dy] = H[dy, dx]: only the canonical
  // columns (cx, cy, k) with 0 <= cy <= cx are evaluated and stored, and every footprint
  // column points at its canonical one.
  const int Kc = K + 1;
  std::vector<int> can_of((size_t)Kc * Kc * nz, -1);  // (cy, cx, k) -> canonical column
  std::vector<int> cdx, cdy, ck;                      // canonical columns
  std::vector<int> foi, fk, fcan;                     // footprint columns
  for (int a = 0; a < W; ++a)
    for (int b = 0; b < W; ++b)
      for (int k = 0; k < nz; ++k) {
        if (!in_footprint(s, g, b - K, a - K, k)) continue;
        const int ax = std::abs(b - K), ay = std::abs(a - K);
        const int cx = std::max(ax, ay), cy = std::min(ax, ay);
        int& ci = can_of[((size_t)cy * Kc + cx) * nz + k];
        if (ci < 0) {
          ci = (int)cdx.size();
          cdx.push_back(cx);
          cdy.push_back(cy);
          ck.push_back(k);
        }
        foi.push_back(a * W + b);
        fk.push_back(k);
        fcan.push_back(ci);
      }
  const int nc = (int)cdx.size();

  Geo geo;
  geo.step = m.step_mm;
  geo.R = m.R_mm;
  geo.cfs = m.cfs;
  geo.sigma5 = kCutoffSigmas * m.sigma;
  geo.inv2s2 = 1.0 / (2.0 * m.sigma * m.sigma);
  geo.invs2 = 1.0 / (m.sigma * m.sigma);
  geo.omega = m.omega;
  geo.nz = nz;
  geo.nt = g.nt;
  geo.M = m.M;
  geo.dz_m = g.dz_m;
  geo.fd = g.time_derivative;
  geo.reach = geo.sigma5 + (g.time_derivative ? 1.0 : 0.0);
  std::vector<double> qp, qw;
  basis_points(g, qp, qw);
  geo.nq = (int)qw.size();

  double *d_ex = nullptr, *d_ey = nullptr, *d_ez = nullptr, *d_eoff = nullptr, *d_area = nullptr;
  int *d_cdx = nullptr, *d_cdy = nullptr, *d_ck = nullptr, *d_clo = nullptr, *d_chi = nullptr;
  double *d_qp = nullptr, *d_qw = nullptr;
  size_t tmp = 0;
  int rc = AROAM_OK;
  auto cleanup = [&]() {
    (void)hipFree(d_ex); (void)hipFree(d_ey); (void)hipFree(d_ez); (void)hipFree(d_eoff); (void)hipFree(d_area);
    (void)hipFree(d_cdx); (void)hipFree(d_cdy); (void)hipFree(d_ck); (void)hipFree(d_clo); (void)hipFree(d_chi);
    (void)hipFree(d_qp); (void)hipFree(d_qw);
  };
  do {
    if ((rc = alloc_copy(&d_qp, qp, tmp))) break;
    if ((rc = alloc_copy(&d_qw, qw, tmp))) break;
    if ((rc = alloc_copy(&d_ex, ex, tmp))) break;
    if ((rc = alloc_copy(&d_ey, ey, tmp))) break;
    if ((rc = alloc_copy(&d_ez, ez, tmp))) break;
    if ((rc = alloc_copy(&d_eoff, eoff, tmp))) break;
    if ((rc = alloc_copy(&d_area, area, tmp))) break;
    if ((rc = alloc_copy(&d_cdx, cdx, tmp))) break;
    if ((rc = alloc_copy(&d_cdy, cdy, tmp))) break;
    if ((rc = alloc_copy(&d_ck, ck, tmp))) break;
    std::vector<int> zeros(nc, 0);
    if ((rc = alloc_copy(&d_clo, zeros, tmp))) break;
    if ((rc = alloc_copy(&d_chi, zeros, tmp))) break;
    if (nc > 0) {
      hipLaunchKernelGGL(k_support, dim3((unsigned)ceil_div(nc, 128)), dim3(128), 0, st, nc,
                         d_cdx, d_cdy, d_ck, d_ex, d_ey, d_ez, d_eoff, d_qp, geo, d_clo, d_chi);
      if (hipGetLastError() != hipSuccess) { set_error("support kernel launch failed"); rc = AROAM_EDEVICE; break; }
    }
    std::vector<int> clo(nc), chi(nc);
    if (nc > 0) {
      if (hipMemcpyAsync(clo.data(), d_clo, nc * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipMemcpyAsync(chi.data(), d_chi, nc * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        set_error("support download failed");
        rc = AROAM_EDEVICE;
        break;
      }
    }
    // stored columns: canonical columns with a non-empty window.  With a band-pass filter the
    // stored window is the filtered one, [lo - L, hi + L] in [0, nt); the sub-element sum is
    // first evaluated on the raw window [lo, hi].
    const int L = m.filtered ? m.fir_L : 0;
    std::vector<int> elo(nc, -1), ehi(nc, -1);
    for (int c = 0; c < nc; ++c)
      if (clo[c] >= 0) {
        elo[c] = std::max(0, clo[c] - L);
        ehi[c] = std::min(g.nt - 1, chi[c] + L);
      }
    std::vector<int> stored(nc, -1), sdx, sdy, sk, slo, rlo;
    std::vector<long long> soff(1, 0), roff(1, 0);
    for (int c = 0; c < nc; ++c) {
      if (clo[c] < 0) continue;
      stored[c] = (int)slo.size();
      sdx.push_back(cdx[c]);
      sdy.push_back(cdy[c]);
      sk.push_back(ck[c]);
      slo.push_back(elo[c]);
      soff.push_back(soff.back() + (ehi[c] - elo[c] + 1));
      rlo.push_back(clo[c]);
      roff.push_back(roff.back() + (chi[c] - clo[c] + 1));
    }
    std::vector<double> no_values;
    if ((rc = set_columns(m, foi, fk, fcan, stored, elo, ehi, slo, soff, no_values, bytes))) break;
    int *d_sdx = nullptr, *d_sdy = nullptr, *d_sk = nullptr, *d_rlo = nullptr;
    long long* d_roff = nullptr;
    double* d_raw = nullptr;
    auto free_cols = [&]() {
      (void)hipFree(d_sdx); (void)hipFree(d_sdy); (void)hipFree(d_sk);
      (void)hipFree(d_rlo); (void)hipFree(d_roff); (void)hipFree(d_raw);
    };
    if ((rc = alloc_copy(&d_sdx, sdx, tmp)) || (rc = alloc_copy(&d_sdy, sdy, tmp)) ||
        (rc = alloc_copy(&d_sk, sk, tmp))) {
      free_cols();
      break;
    }
    if (m.filtered) {
      if ((rc = alloc_copy(&d_rlo, rlo, tmp)) || (rc = alloc_copy(&d_roff, roff, tmp))) {
        free_cols();
        break;
      }
      if (hipMalloc((void**)&d_raw, std::max<long long>(1, roff.back()) * sizeof(double)) !=
          hipSuccess) {
        set_error("out of device memory for the unfiltered table");
        rc = AROAM_ENOMEM;
        free_cols();
        break;
      }
    }
    if (m.n_stored > 0) {
      hipLaunchKernelGGL(k_table, dim3((unsigned)m.n_stored), dim3(64), 2 * m.M * sizeof(double),
                         st, d_sdx, d_sdy, d_sk, m.filtered ? d_rlo : m.d_lo,
                         m.filtered ? d_roff : m.d_off, d_ex, d_ey, d_ez, d_eoff, d_area, d_qp,
                         d_qw, geo, m.filtered ? d_raw : m.d_band);
      if (hipGetLastError() != hipSuccess) { set_error("table kernel launch failed"); rc = AROAM_EDEVICE; }
      if (rc == AROAM_OK && m.filtered) rc = filter_columns(m, d_rlo, d_roff, d_raw, st);
    }
    if (rc == AROAM_OK && hipStreamSynchronize(st) != hipSuccess) { set_error("table build failed"); rc = AROAM_EDEVICE; }
    free_cols();
  } while (false);
  cleanup();
  if (rc) return rc;
  return pack_fp(m, st, bytes);
}

// Host side of the column set: the footprint columns (offset index, depth, source column)
// point at stored columns; windows come from the source columns.  Uploads the column maps
// and allocates the FP64 band (filled from `values` when it is not empty).
int set_columns(Model& m, const std::vector<int>& foi, const std::vector<int>& fk,
                const std::vector<int>& fsrc, const std::vector<int>& stored,
                const std::vector<int>& src_lo, const std::vector<int>& src_hi,
                const std::vector<int>& slo, const std::vector<long long>& soff,
                const std::vector<double>& values, size_t& bytes) {
  const aroam_grid& g = m.grid;
  const int nz = g.nz, K = m.K;
  m.h_lo.assign((size_t)m.n_off * nz, -1);
  m.h_hi.assign((size_t)m.n_off * nz, -1);
  m.h_colidx.assign((size_t)m.n_off * nz, -1);
  m.h_off = soff;
  m.n_columns = 0;
  m.nnz = 0;
  m.mac_alg = 0;
  const int W = 2 * K + 1;
  for (size_t i = 0; i < foi.size(); ++i) {
    const int c = fsrc[i];
    if (c < 0 || stored[c] < 0) continue;
    const size_t key = (size_t)foi[i] * nz + fk[i];
    m.h_lo[key] = src_lo[c];
    m.h_hi[key] = src_hi[c];
    m.h_colidx[key] = stored[c];
    const long long len = src_hi[c] - src_lo[c] + 1;
    const int dy = foi[i] / W - K, dx = foi[i] % W - K;
    const long long pairs = (long long)std::max(0, g.ny - std::abs(dy)) *
                            std::max(0, g.nx - std::abs(dx));
    m.n_columns += 1;
    m.nnz += len;
    m.mac_alg += pairs * len;
  }
  m.n_stored = (long long)slo.size();
  m.nnz_stored = soff.back();
  size_t tmp = 0;
  AROAM_TRY(alloc_copy(&m.d_colidx, m.h_colidx, bytes));
  AROAM_TRY(alloc_copy(&m.d_lo, slo, tmp));
  AROAM_TRY(alloc_copy(&m.d_off, soff, tmp));
  const size_t band_bytes = std::max<long long>(1, m.nnz_stored) * sizeof(double);
  if (hipMalloc((void**)&m.d_band, band_bytes) != hipSuccess) {
    set_error("out of device memory for the table");
    return AROAM_ENOMEM;
  }
  if (!values.empty() &&
      hipMemcpy(m.d_band, values.data(), m.nnz_stored * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess) {
    set_error("table upload failed");
    return AROAM_EDEVICE;
  }
  return AROAM_OK;
}

// Band tiles of the always-packed dtypes (FP64 direct form, FP32 staged form).
int pack_fp(Model& m, hipStream_t st, size_t& bytes) {
  // band tiles
  AROAM_TRY(build_layout(m, false, 4, m.g4f, bytes));
  AROAM_TRY(build_layout(m, true, 4, m.g4a, bytes));
  AROAM_TRY(pack_dtype<double>(m, m.g4f, false, m.fwd_pack[AROAM_FP64], st, bytes));
  AROAM_TRY(pack_dtype<double>(m, m.g4a, true, m.adj_pack[AROAM_FP64], st, bytes));
  AROAM_TRY(build_staged_layout(m, false, 4, kTile, 16, kPatchRows, kPatchCols, 4, m.s4f, bytes));
  AROAM_TRY(build_staged_layout(m, true, 4, kTile, 16, kPatchRows, kPatchCols, 4, m.s4a, bytes));
  AROAM_TRY(pack_dtype<float>(m, m.s4f, false, m.fwd_pack[AROAM_FP32], st, bytes));
  AROAM_TRY(pack_dtype<float>(m, m.s4a, true, m.adj_pack[AROAM_FP32], st, bytes));
  m.dtype_mask = (1u << AROAM_FP64) | (1u << AROAM_FP32);
  return AROAM_OK;
}

}  // namespace

int build_model(const aroam_sensor* s, const aroam_grid* g, const aroam_filter* f,
                unsigned mask, hipStream_t st, Model** out) {
  AROAM_CHECK(s && g && out, AROAM_EINVAL, "NULL argument to aroam_build_model");
  *out = nullptr;
  AROAM_CHECK(s->radius_m > 0 && s->aperture_m > 0 && s->aperture_m <= 2 * s->radius_m &&
                  s->hole_m >= 0 && s->hole_m < s->aperture_m && s->f0_hz > 0 &&
                  s->frac_bw > 0 && s->n_rings >= 0 && s->n_rings <= 1000,
              AROAM_EINVAL, "invalid sensor geometry");
  AROAM_TRY(check_grid(g));
  AROAM_CHECK(g->footprint_mode == 0 || g->footprint_mode == 1, AROAM_EINVAL,
              "footprint_mode must be 0 or 1");
  if (f) AROAM_TRY(check_filter(*f, g->fs_hz, g->nt));
  AROAM_CHECK((g->voxel_basis == 0 || g->voxel_basis == 1) &&
                  (g->time_derivative == 0 || g->time_derivative == 1) && g->basis_quad >= 0 &&
                  g->basis_quad <= 8,
              AROAM_EINVAL, "voxel_basis, time_derivative must be 0 or 1, basis_quad 0..8");
  Model* m = new (std::nothrow) Model();
  AROAM_CHECK(m, AROAM_ENOMEM, "host allocation failed");
  m->sensor = *s;
  m->grid = *g;
  m->K = g->k_half;
  m->n_off = (2 * g->k_half + 1) * (2 * g->k_half + 1);
  (void)hipGetDevice(&m->device);
  int rc = AROAM_OK;
  if (f) rc = setup_filter(*m, *f);
  if (rc == AROAM_OK) rc = build_impl(*m, st);
  return finish_model(m, rc, mask, st, out);
}

namespace {

// Value of an OCP e4m3 code (sign, 4 exponent bits of bias 7, 3 mantissa bits; exponent 0 is
// subnormal; 0x7f / 0xff are NaN).
double e4m3_value(uint8_t c) {
  const int e = (c >> 3) & 15, mant = c & 7;
  if (e == 15 && mant == 7) return std::nan("");
  const double mag = e == 0 ? std::ldexp(mant / 8.0, -6) : std::ldexp(1.0 + mant / 8.0, e - 7);
  return (c & 0x80) ? -mag : mag;
}

template <typename T>
int download(std::vector<T>& h, const void* d, size_t n) {
  h.resize(std::max<size_t>(1, n));
  if (n > 0 && hipMemcpy(h.data(), d, n * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("download of a packed table failed");
    return AROAM_EDEVICE;
  }
  return AROAM_OK;
}

}  // namespace

int export_quantized(const Model& m, int dtype, bool adjoint, double* dense, float* scales) {
  AROAM_CHECK(dense, AROAM_EINVAL, "NULL output");
  AROAM_CHECK(dtype == AROAM_FP32 || dtype == AROAM_BF16 || dtype == AROAM_FP8E4M3, AROAM_EINVAL,
              "export of the FP32, BF16 or FP8 packs (dtype %d)", dtype);
  AROAM_CHECK((m.dtype_mask >> dtype) & 1u, AROAM_EUNSUPPORTED, "model was not packed for dtype %d",
              dtype);
  const Layout& lay = layout_for(m, adjoint, dtype);
  const Pack& pk = adjoint ? m.adj_pack[dtype] : m.fwd_pack[dtype];
  const int nz = m.grid.nz, nt = m.grid.nt, TM = lay.TM, G = lay.G;
  const int nblk = (int)ceil_div(nz, 16);
  const bool fp8 = dtype == AROAM_FP8E4M3;
  const size_t n_groups = (size_t)lay.n_bundles * (fp8 ? 16 : kLaneGroups);
  std::vector<int4> groups;
  AROAM_TRY(download(groups, lay.d_groups, n_groups));
  const size_t esize = dtype == AROAM_FP32 ? 4 : dtype == AROAM_BF16 ? 2 : 1;
  std::vector<uint8_t> raw;
  AROAM_TRY(download(raw, pk.d, n_groups * TM * G * esize));
  std::vector<int> rec;
  if (fp8) AROAM_TRY(download(rec, lay.d_meta, (size_t)lay.n_bundles * 16));
  int block_of[4][4];  // scale block of (lane group, slot) in an FP8 bundle
  for (int b = 0; b < 4; ++b)
    for (int i = 0; i < 4; ++i) block_of[kFp8Lane[b][i]][kFp8Slot[b][i]] = b;
  std::fill(dense, dense + (size_t)m.n_off * nz * nt, 0.0);
  if (scales) std::fill(scales, scales + (size_t)m.n_off * nblk, 0.0f);
  for (size_t q = 0; q < n_groups; ++q) {
    const int4 gd = groups[q];  // (offset index, run start, tile, active)
    if (gd.x < 0) continue;
    for (int r = 0; r < TM; ++r)
      for (int j = 0; j < G; ++j) {
        const int n = adjoint ? gd.y + j : TM * gd.z + r;
        const int k = adjoint ? TM * gd.z + r : gd.y + j;
        if (n >= nt || k >= nz) continue;
        double v;
        if (dtype == AROAM_FP32) {
          float f;
          std::memcpy(&f, &raw[4 * (q * TM * G + (size_t)r * G + j)], 4);
          v = f;
        } else if (dtype == AROAM_BF16) {
          const size_t e = q * TM * G + (size_t)r * G + j;
          const uint32_t bits = (uint32_t)(raw[2 * e] | (raw[2 * e + 1] << 8)) << 16;
          float f;
          std::memcpy(&f, &bits, 4);
          v = f;
        } else {
          // K-group q = [bundle][lane group][slot]; its scale is the E8M0 byte of the half in
          // the record word of the lane group that carries its block's scale
          const size_t bi = q / 16;
          const int ln = (int)((q % 16) / 4), slot = (int)(q % 4), h = r / kTile;
          const size_t pos = ((bi * 2 + h) * 64 + ln * 16 + r % kTile) * 32 + slot * 8 + j;
          const int sl = kFp8ScaleLane[block_of[ln][slot]];
          const int e8 = (rec[bi * 16 + sl * 4 + 2] >> (8 * h)) & 0xff;
          const double sc = std::ldexp(1.0, e8 - 127);
          v = e4m3_value(raw[pos]) * sc;
          // a block with entries has a nonzero code (its largest lands in the top binade);
          // the scale a pack carries for an empty block is not reported
          if (scales && v != 0.0) scales[(size_t)gd.x * nblk + k / 16] = (float)sc;
        }
        dense[((size_t)gd.x * nz + k) * nt + n] = v;
      }
  }
  return AROAM_OK;
}

int check_grid(const aroam_grid* g) {
  AROAM_CHECK(g->c_mps > 0 && g->fs_hz > 0 && g->step_m > 0 && g->dz_m > 0, AROAM_EINVAL,
              "invalid grid spacing");
  AROAM_CHECK(g->nx >= 1 && g->ny >= 1 && g->nz >= 1 && g->nt >= 1 && g->nx <= 65536 &&
                  g->ny <= 65536 && g->nz <= 65536 && g->nt <= 65536,
              AROAM_EINVAL, "grid sizes out of range");
  AROAM_CHECK(g->k_half >= 0 && g->k_half <= AROAM_MAX_K_HALF, AROAM_EINVAL,
              "k_half %d out of range 0..%d (the staged applies' LDS row ring holds %d + 2 k_half "
              "columns)", g->k_half, AROAM_MAX_K_HALF, kPatchCols);
  return AROAM_OK;
}

int import_model(const aroam_grid* g, const double* dense, const int* col_lo,
                 const int* col_hi, unsigned mask, hipStream_t st, Model** out) {
  AROAM_CHECK(g && dense && out, AROAM_EINVAL, "NULL argument to aroam_import_model");
  *out = nullptr;
  AROAM_CHECK((col_lo == nullptr) == (col_hi == nullptr), AROAM_EINVAL,
              "col_lo and col_hi must both be given or both be NULL");
  AROAM_TRY(check_grid(g));
  const int K = g->k_half, W = 2 * K + 1, nz = g->nz, nt = g->nt;
  const size_t ncol = (size_t)W * W * nz;
  // columns and their windows: as given, or first..last nonzero sample
  std::vector<int> foi, fk, fsrc, stored, clo, chi, slo;
  std::vector<long long> soff(1, 0);
  std::vector<double> values;
  for (size_t key = 0; key < ncol; ++key) {
    const double* col = dense + key * nt;
    int lo = -1, hi = -1;
    if (col_lo) {
      lo = col_lo[key];
      hi = col_hi[key];
      AROAM_CHECK((lo < 0 && hi < 0) || (0 <= lo && lo <= hi && hi < nt), AROAM_EINVAL,
                  "column %zu: window [%d, %d] outside [0, %d)", key, lo, hi, nt);
    } else {
      for (int n = 0; n < nt; ++n)
        if (col[n] != 0.0) {
          if (lo < 0) lo = n;
          hi = n;
        }
    }
    if (lo < 0) continue;
    for (int n = lo; n <= hi; ++n)
      AROAM_CHECK(std::isfinite(col[n]), AROAM_ENONFINITE, "column %zu: non-finite value", key);
    const int c = (int)clo.size();
    foi.push_back((int)(key / nz));
    fk.push_back((int)(key % nz));
    fsrc.push_back(c);
    stored.push_back(c);
    clo.push_back(lo);
    chi.push_back(hi);
    slo.push_back(lo);
    values.insert(values.end(), col + lo, col + hi + 1);
    soff.push_back((long long)values.size());
  }
  Model* m = new (std::nothrow) Model();
  AROAM_CHECK(m, AROAM_ENOMEM, "host allocation failed");
  m->grid = *g;
  m->grid.footprint_mode = 0;
  m->K = K;
  m->n_off = W * W;
  (void)hipGetDevice(&m->device);
  size_t bytes = 0;
  int rc = set_columns(*m, foi, fk, fsrc, stored, clo, chi, slo, soff, values, bytes);
  if (!rc) rc = pack_fp(*m, st, bytes);
  return finish_model(m, rc, mask, st, out);
}

// Reduced-precision packs, device-memory accounting, and ownership of a model whose FP64
// table and FP64 / FP32 packs are built (rc: status of that stage).
int finish_model(Model* m, int rc, unsigned mask, hipStream_t st, Model** out) {
  if (rc == AROAM_OK) {
    const bool want8 = (mask & (1u << AROAM_BF16)) != 0;
    size_t bytes = 0;
    if (want8) {
      rc = build_staged_layout(*m, false, 8, kTileRows8, 32, kPatchRows, kPatchCols, 2, m->s8f,
                               bytes);
      if (!rc)
        rc = build_staged_layout(*m, true, 8, kTileRows8, 32, kPatchRows, kPatchCols, 2, m->s8a,
                                 bytes);
    }
    if (!rc && (mask & (1u << AROAM_BF16))) {
      rc = pack_dtype<uint16_t>(*m, m->s8f, false, m->fwd_pack[AROAM_BF16], st, bytes);
      if (!rc) rc = pack_dtype<uint16_t>(*m, m->s8a, true, m->adj_pack[AROAM_BF16], st, bytes);
      if (!rc) m->dtype_mask |= 1u << AROAM_BF16;
    }
    if (!rc && (mask & (1u << AROAM_FP8E4M3))) {
      rc = pack_all_fp8(*m, st, bytes);
      if (!rc) m->dtype_mask |= 1u << AROAM_FP8E4M3;
    }
    if (!rc && hipStreamSynchronize(st) != hipSuccess) {
      set_error("model packing failed");
      rc = AROAM_EDEVICE;
    }
  }
  if (rc != AROAM_OK) {
    destroy_model(m);
    return rc;
  }
  // account device memory
  size_t b = (size_t)std::max<long long>(1, m->nnz_stored) * sizeof(double);
  b += m->h_colidx.size() * sizeof(int) + m->n_stored * sizeof(int) + m->h_off.size() * 8;
  for (const Layout* l : {&m->g4f, &m->g4a, &m->s4f, &m->s4a, &m->s8f, &m->s8a, &m->f8f, &m->f8a})
    b += l->n_bundles * kLaneGroups * (sizeof(int) + sizeof(int4)) * (l == &m->f8f || l == &m->f8a ? 4 : 1) +
         (l->staged ? l->n_bundles * sizeof(int) + l->n_pieces * sizeof(int4) +
                          l->n_tiles * sizeof(int2)
                    : l->h_tile_start.size() * sizeof(int)) +
         l->n_units * (sizeof(int4) + sizeof(int2));
  for (int d = 0; d < 4; ++d) b += m->fwd_pack[d].bytes + m->adj_pack[d].bytes;
  m->device_bytes = b;
  *out = m;
  return AROAM_OK;
}

void destroy_model(Model* m) {
  if (!m) return;
  (void)hipFree(m->d_fir_taps);
  (void)hipFree(m->d_fir_pad64);
  (void)hipFree(m->d_fir_pad32);
  (void)hipFree(m->d_band);
  (void)hipFree(m->d_colidx);
  (void)hipFree(m->d_lo);
  (void)hipFree(m->d_off);
  for (Layout* l : {&m->g4f, &m->g4a, &m->s4f, &m->s4a, &m->s8f, &m->s8a, &m->f8f, &m->f8a}) {
    (void)hipFree(l->d_tile_start);
    (void)hipFree(l->d_meta);
    (void)hipFree(l->d_groups);
    (void)hipFree(l->d_pieces);
    (void)hipFree(l->d_tile_split);
    (void)hipFree(l->d_units);
    (void)hipFree(l->d_ucols);
  }
  for (int d = 0; d < 4; ++d) {
    (void)hipFree(m->fwd_pack[d].d);
    (void)hipFree(m->adj_pack[d].d);
  }
  delete m;
}

}  // namespace aroam
