// Applies of the scan-symmetric model: s = A x and x = A^T s.
//
// Both operators have the same shape once the table is cut into band tiles (Methods,
// "Efficient reconstruction based on scanning symmetries": an absolute index over the voxel
// grid and a relative one from each scan position select the model vector):
//     out[p][16 t + m] = sum_{K-groups q of tile t} sum_{j < G} pack[q][m][j] * in[p + d_q + j]
// where p runs over scan positions, the K-group q names one lateral offset o and a run of G
// consecutive depths (forward) or time samples (adjoint), and d_q is the offset of
// (p + o, run start) in the zero-padded input (p - o for the adjoint).  The lateral halo
// of the padded input supplies the zeros outside the region of interest.
//
// GEMM view per tile: M = 16 output rows, N = scan positions (16 per MFMA), K = the tile's
// K-groups.  Kernels: a plain FP64/FP32 FMA kernel, FP32 MFMA (v_mfma_f32_16x16x4f32), BF16
// MFMA (v_mfma_f32_16x16x32_bf16) and the block-scaled FP8 MFMA
// (v_mfma_scale_f32_16x16x128_f8f6f4, e4m3 table and operand) on gfx950.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <mutex>

#include "internal.h"

namespace aroam {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
// Register operands are clang vector types and are reinterpreted with __builtin_bit_cast, so
// no local variable has its address taken (which would place it in scratch memory).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));


template <typename Tin, typename Tout>
__device__ inline Tout conv(Tin v);
template <>
__device__ inline double conv<double, double>(double v) { return v; }
template <>
__device__ inline float conv<float, float>(float v) { return v; }
template <>
__device__ inline uint16_t conv<float, uint16_t>(float f) {  // bf16, round to nearest even
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Stage an input vector [ny][nx][L] into the padded layout [nyp][nxp][Lp]; the halo and the
// tail of every column are written as zeros.  One workgroup per padded column.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(256) void k_stage(const Tin* __restrict__ in, Tout* __restrict__ out,
                                               int K, int nx, int ny, int nxp, int L, int Lp) {
  const int col = blockIdx.x;
  const int px = col % nxp - K, py = col / nxp - K;
  Tout* o = out + (long long)col * Lp;
  const bool inside = px >= 0 && px < nx && py >= 0 && py < ny;
  const Tin* src = in + ((long long)py * nx + px) * L;
  for (int l = threadIdx.x; l < Lp; l += blockDim.x) {
    Tout v = Tout(0);
    if (inside && l < L) v = conv<Tin, Tout>(src[l]);
    o[l] = v;
  }
}

struct ApplyArgs {
  const int* tile_start;
  const int* meta;
  int out_len;
  int n_ntiles;  // 16-position tiles over the whole scan grid
  int ntx, nx, K, nxp, Lp;
};

// Plain kernel: one thread per (output row, position); G-entry FMA loops in the vector type.
template <typename T>
__global__ __launch_bounds__(256) void k_apply_fma(const T* __restrict__ pack, const T* __restrict__ in,
                                                   T* __restrict__ out, ApplyArgs a, int G) {
  const int tile = blockIdx.y;
  const int ntile = blockIdx.x;
  const int m = threadIdx.x / 16, n = threadIdx.x % 16;
  const int py = ntile / a.ntx, tx = ntile % a.ntx;
  const long long base = ((long long)(py + a.K) * a.nxp + 16 * tx + n + a.K) * a.Lp;
  T acc = T(0);
  const int b0 = a.tile_start[tile], b1 = a.tile_start[tile + 1];
  for (int b = b0; b < b1; ++b) {
    for (int g = 0; g < kLaneGroups; ++g) {
      const int q = b * kLaneGroups + g;
      const T* ap = pack + ((long long)q * 16 + m) * G;
      const T* xp = in + base + a.meta[q];
      for (int j = 0; j < G; ++j) acc += ap[j] * xp[j];
    }
  }
  const int row = kTile * tile + m, px = 16 * tx + n;
  if (row < a.out_len && px < a.nx) out[((long long)py * a.nx + px) * a.out_len + row] = acc;
}

struct StagedArgs {
  const int4* pieces;      // (tile, unit begin, unit end, partial slot or -1)
  const int2* tile_split;  // per tile: (pieces, first slot)
  float* partial;          // [slot][patch][position][TM rows] partial sums of cut tiles
  int n_patches;
  const int4* units;  // (row offset, chunk start, bundle begin, bundle end)
  const int2* urows;  // padded patch rows [lo, hi) each unit loads into the LDS ring
  const int* meta;
  int out_len, nx, ny, K, nxp, Lp;
  int ncc;            // patch column chunks
  int NCOL, CS;
};

// Table operand of one bundle for one lane: 16 bytes per 16-row half (MH = TM / 16 halves).
template <typename T, int MH>
struct AFrag {
  u32x4 v[MH];
  int mo;  // the K-group's meta word: LDS offset (and for MH > 1 the bundle's half mask)
};

template <typename T, int MH>
__device__ __forceinline__ void load_a(const void* __restrict__ pack_raw,
                                       const int* __restrict__ meta,
                                       int b, int g, int n,
                                       AFrag<T, MH>& f) {
  const int q = b * kLaneGroups + g;
#pragma unroll
  for (int h = 0; h < MH; ++h) {
    const long long row = (long long)q * (16 * MH) + 16 * h + n;
    constexpr int VEC = 16 / sizeof(T);
    f.v[h] = *reinterpret_cast<const u32x4*>(reinterpret_cast<const T*>(pack_raw) + row * VEC);
  }
  f.mo = meta[q];  // raw word: for MH > 1 the bundle's half mask sits in its top bits
}

// Global source and LDS destination of flat stage vector idx of a unit that loads padded
// patch rows from `lo`, for the chunk starting at inner entry e0.
struct StageAddr {
  long long src;
  int lds;
};

// RS: slots of the LDS row ring (padded row G lives in slot G mod RS).
template <int RS>
__device__ __forceinline__ StageAddr stage_addr(const StagedArgs& a, int lo, int e0, int idx,
                                                int py0, int px0, int rowvec, int nvec, int vec) {
  const int G = lo + idx / rowvec;
  const int rem = idx % rowvec;
  const int c = rem / nvec, v = rem % nvec;
  StageAddr r;
  r.lds = ((G % RS) * a.NCOL + c) * a.CS + v * vec;
  r.src = ((long long)(py0 + G) * a.nxp + (px0 + c)) * a.Lp + e0 + v * vec;
  return r;
}

// Fetch up to 256 * PF stage vectors of unit u into registers (the rest is loaded when the
// unit's rows are written); pf_off = -1 marks an unused slot.
template <typename T, int RS, int PF>
__device__ __forceinline__ void stage_prefetch(const StagedArgs& a, const T* __restrict__ in,
                                               int u, int py0, int px0, int rowvec, int nvec,
                                               u32x4 (&pf)[PF], int (&pf_off)[PF]) {
  constexpr int VEC = 16 / sizeof(T);
  const int4 U = a.units[u];
  const int2 Rr = a.urows[u];
  const int nv = (Rr.y - Rr.x) * rowvec;
#pragma unroll
  for (int i = 0; i < PF; ++i) {
    const int idx = threadIdx.x + 256 * i;
    pf_off[i] = -1;
    if (idx < nv) {
      const StageAddr sa = stage_addr<RS>(a, Rr.x, U.y, idx, py0, px0, rowvec, nvec, VEC);
      pf_off[i] = sa.lds;
      pf[i] = *reinterpret_cast<const u32x4*>(in + sa.src);
    }
  }
}

// Write the rows unit u adds to the LDS ring: the prefetched vectors, then the rest (a full
// ring reload) with four loads in flight per thread.
template <typename T, int RS, int PF>
__device__ __forceinline__ void stage_rows(const StagedArgs& a, const T* __restrict__ in, T* lds,
                                           int u, int py0, int px0, int rowvec, int nvec,
                                           const u32x4 (&pf)[PF], const int (&pf_off)[PF]) {
  constexpr int VEC = 16 / sizeof(T);
#pragma unroll
  for (int i = 0; i < PF; ++i)
    if (pf_off[i] >= 0) *reinterpret_cast<u32x4*>(lds + pf_off[i]) = pf[i];
  const int4 U = a.units[u];
  const int2 Rr = a.urows[u];
  const int nv = (Rr.y - Rr.x) * rowvec;
  for (int base = 256 * PF; base < nv; base += 256 * 4) {
    u32x4 tmp[4];
    int off[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = base + threadIdx.x + 256 * i;
      off[i] = -1;
      if (idx < nv) {
        const StageAddr sa = stage_addr<RS>(a, Rr.x, U.y, idx, py0, px0, rowvec, nvec, VEC);
        off[i] = sa.lds;
        tmp[i] = *reinterpret_cast<const u32x4*>(in + sa.src);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (off[i] >= 0) *reinterpret_cast<u32x4*>(lds + off[i]) = tmp[i];
  }
}

// Position fragments of one bundle for the NT tiles of this lane: 16 bytes each from LDS.
// Tiles t with t % TPR >= NTC (16-position tiles beyond the last scan column, in a patch at
// the grid's edge) are left out.
template <typename T, int NT, int TPR = 1, int NTC = TPR>
__device__ __forceinline__ void read_x(const T* lds, const int (&lbase)[NT], int mo,
                                       u32x4 (&x)[NT]) {
  mo &= (1 << kMetaMaskShift) - 1;  // the top bits hold the bundle's mask
#pragma unroll
  for (int t = 0; t < NT; ++t)
    if (t % TPR < NTC) x[t] = *reinterpret_cast<const u32x4*>(lds + lbase[t] + mo);
}

// read_x for a lane whose tile t sits at row base rb[t / TPR] plus column offset
// (t % TPR) * 16 * CSC (compile-time column stride CSC, so the offsets are immediates).
template <typename T, int NT, int TPR, int CSC, int NR>
__device__ __forceinline__ void read_x_rows(const T* lds, const int (&rb)[NR], int mo,
                                            u32x4 (&x)[NT]) {
  mo &= (1 << kMetaMaskShift) - 1;  // the top bits hold the bundle's mask
#pragma unroll
  for (int t = 0; t < NT; ++t)
    x[t] = *reinterpret_cast<const u32x4*>(lds + rb[t / TPR] + mo + (t % TPR) * 16 * CSC);
}

// MFMAs of one bundle whose position fragments are already in registers (tiles as read_x).
template <typename T, int MH, int NT, int TPR = 1, int NTC = TPR>
__device__ __forceinline__ void bundle_mma(const AFrag<T, MH>& f, const u32x4 (&xraw)[NT],
                                           floatx4 (&acc)[MH][NT]) {
  // the bundle's mask: for FP32 the entries of its runs (one MFMA each) that a K-group's band
  // reaches, for BF16 the 16-row halves; uniform over the wave
  const unsigned bm = (unsigned)__builtin_amdgcn_readfirstlane(f.mo) >> kMetaMaskShift;
  if constexpr (sizeof(T) == 4) {
    static_assert(MH == 1, "FP32 tiles have one 16-row half");
    const floatx4 av = __builtin_bit_cast(floatx4, f.v[0]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (!((bm >> j) & 1)) continue;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t % TPR >= NTC) continue;
        const floatx4 xv = __builtin_bit_cast(floatx4, xraw[t]);
        acc[0][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[j], xv[j], acc[0][t], 0, 0, 0);
      }
    }
  } else {
#pragma unroll
    for (int h = 0; h < MH; ++h) {
      if (MH > 1 && !((bm >> h) & 1)) continue;  // the bundle's bands miss this half
      const bf16x8 av = __builtin_bit_cast(bf16x8, f.v[h]);
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t % TPR >= NTC) continue;
        const bf16x8 xv = __builtin_bit_cast(bf16x8, xraw[t]);
        acc[h][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, xv, acc[h][t], 0, 0, 0);
      }
    }
  }
}

// FP32 bundles [U.z, U.w) of one stage unit for the tiles of the NTC live tile columns: the
// next bundle's position fragments are read while this bundle's 16 MFMAs run (two register
// sets), and ring slot (j + 1) mod PD holds the next bundle (or a clamped copy of the last).
template <int MH, int NT, int TPR, int NTC, int PD>
__device__ __forceinline__ void fp32_unit_bundles(const float* lds, const int (&lbase)[NT],
                                                  AFrag<float, MH> (&ring)[PD],
                                                  floatx4 (&acc)[MH][NT],
                                                  const void* __restrict__ pack_raw,
                                                  const StagedArgs& a, int4 U, int g, int n) {
  u32x4 xa[NT], xb[NT];
  read_x<float, NT, TPR, NTC>(lds, lbase, ring[0].mo, xa);
  for (int b0 = U.z; b0 < U.w; b0 += PD) {
#pragma unroll
    for (int j = 0; j < PD; ++j) {
      read_x<float, NT, TPR, NTC>(lds, lbase, ring[(j + 1) % PD].mo, (j % 2) ? xa : xb);
      if (b0 + j < U.w) bundle_mma<float, MH, NT, TPR, NTC>(ring[j], (j % 2) ? xb : xa, acc);
      // refill unconditionally (clamped to the unit's last bundle) so that the number of
      // loads in flight is fixed and the waits can count them
      load_a<float, MH>(pack_raw, a.meta, min(b0 + j + PD, U.w - 1), g, n, ring[j]);
    }
  }
}

// LDS-staged FP32 MFMA kernel.  A workgroup (4 waves) owns one output tile (16 MH rows) and
// one patch of BR scan rows x BC scan columns; each wave owns BR/4 rows x BC columns = NT
// 16-position tiles.  The tile's bundles are grouped into stage units (chunk, input row
// offset).  The LDS holds the BR input rows a unit reads (all BC + 2K columns, the chunk's CH
// inner entries) plus one free row, as a ring of BR + 1 slots indexed by padded row: a unit
// loads only the rows it adds to the ring, and those rows are fetched into registers while
// the previous unit computes.  Table fragments stream through a PD-deep register ring, whose
// refill for the next unit is issued before that unit's rows are staged.  Lane (n = lane % 16,
// g = lane / 16) holds row n of K-group g of the table and the entries of K-group g for
// position n.
// Two waves per SIMD (the LDS holds two workgroups of the 81 x 81 footprint): with that
// target the compiler keeps the accumulators in VGPRs and the next bundle's reads ahead of the
// MFMAs.
template <typename T, int BR, int BC, int MH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_apply_staged(const void* __restrict__ pack_raw,
                                                      const T* __restrict__ in,
                                                      float* __restrict__ out, StagedArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  static_assert(sizeof(T) == 4, "the staged kernel is the FP32 path");
  constexpr int VEC = 16 / sizeof(T);  // entries per 16-byte vector == K-group width G
  constexpr int TPR = BC / 16;
  constexpr int RW = BR / 4;
  constexpr int NT = RW * TPR;
  constexpr int PF = 4;                // prefetched stage vectors per thread (>= one row)
  constexpr int PD = 4;                // table-fragment ring depth (even)
  constexpr int CH = 4 * VEC;          // chunk = one bundle's four K-groups... per lane group
  const int4 piece = a.pieces[blockIdx.y];
  const int tile = piece.x;
  const int py0 = (blockIdx.x / a.ncc) * BR, px0 = (blockIdx.x % a.ncc) * BC;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int n = lane % 16, g = lane / 16;
  constexpr int nvec = CH / VEC;       // 16-byte vectors per staged column
  const int rowvec = a.NCOL * nvec;    // 16-byte vectors per staged row
  floatx4 acc[MH][NT];
#pragma unroll
  for (int h = 0; h < MH; ++h)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[h][t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int u0 = piece.y, u1 = piece.z;
  if (u0 < u1) {
    // the ring has one slot more than the BR rows a unit reads: when the next unit adds the
    // single row after the current unit's rows (consecutive row offsets in one chunk), that
    // row goes to the free slot while other waves still read the current unit, and one
    // barrier per unit suffices
    constexpr int RS = BR + 1;
    u32x4 pf[PF];
    int pf_off[PF];
    // table fragments stream through a ring of PD slots per stage unit, unrolled so that
    // every slot stays in fixed registers (shifting a ring would move registers that loads
    // in flight still target, which forces full waits)
    AFrag<T, MH> ring[PD];
    {
      const int4 U = a.units[u0];
#pragma unroll
      for (int j = 0; j < PD; ++j)
        load_a<T, MH>(pack_raw, a.meta, min(U.z + j, U.w - 1), g, n, ring[j]);
      stage_prefetch<T, RS, PF>(a, in, u0, py0, px0, rowvec, nvec, pf, pf_off);
      stage_rows<T, RS, PF>(a, in, lds, u0, py0, px0, rowvec, nvec, pf, pf_off);
      __syncthreads();
      if (u0 + 1 < u1) stage_prefetch<T, RS, PF>(a, in, u0 + 1, py0, px0, rowvec, nvec, pf, pf_off);
    }
    for (int u = u0; u < u1; ++u) {
      const int4 U = a.units[u];
      // LDS base of this lane's positions for the unit's row offset
      const int R = U.x + a.K;
      int lbase[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int r = wave * RW + t / TPR, c = (t % TPR) * 16 + n;
        lbase[t] = (((r + R) % RS) * a.NCOL + c) * a.CS;
      }
      // a wave whose rows read only the zero rows around the scan grid at this unit's row
      // offset skips the unit's MFMAs (it still stages its share of the unit's rows)
      const int src_row = py0 + wave * RW + U.x;
      const bool live = src_row + RW > 0 && src_row < a.ny;
      if (!live) {
      } else if constexpr (TPR == 2) {
        // a patch at the grid's last columns computes only its tiles that hold scan columns
        if (px0 + 16 >= a.nx)
          fp32_unit_bundles<MH, NT, TPR, 1, PD>(lds, lbase, ring, acc, pack_raw, a, U, g, n);
        else
          fp32_unit_bundles<MH, NT, TPR, TPR, PD>(lds, lbase, ring, acc, pack_raw, a, U, g, n);
      } else {
        fp32_unit_bundles<MH, NT, TPR, TPR, PD>(lds, lbase, ring, acc, pack_raw, a, U, g, n);
      }
      if (u + 1 < u1) {
        const int4 Un = a.units[u + 1];
        const int2 Rn = a.urows[u + 1];
        // the next unit's first table fragments; their loads overlap the staging below
#pragma unroll
        for (int j = 0; j < PD; ++j)
          load_a<T, MH>(pack_raw, a.meta, min(Un.z + j, Un.w - 1), g, n, ring[j]);
        // one new row right after this unit's rows: its slot is the free one
        const bool free_slot = Rn.y - Rn.x == 1 && Rn.x == R + BR;
        if (!free_slot) __syncthreads();  // every wave is done reading the rows replaced
        stage_rows<T, RS, PF>(a, in, lds, u + 1, py0, px0, rowvec, nvec, pf, pf_off);
        __syncthreads();  // the next unit's rows are in LDS; every wave is done with this unit
        if (u + 2 < u1) stage_prefetch<T, RS, PF>(a, in, u + 2, py0, px0, rowvec, nvec, pf, pf_off);
      }
    }
  }
  // the output, or for a piece of a cut tile its partial slot (the patch's positions in order,
  // TM rows each), which k_add_slots adds up
  constexpr int PS = BR * BC * 16 * MH;  // floats per slot and patch
  float* slot =
      piece.w >= 0 ? a.partial + ((long long)piece.w * a.n_patches + blockIdx.x) * PS : nullptr;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int py = py0 + wave * RW + t / TPR, px = px0 + (t % TPR) * 16 + n;
    if (py >= a.ny || px >= a.nx) continue;
    const int local = (wave * RW + t / TPR) * BC + (t % TPR) * 16 + n;
    // element offset of output row `row` of this position: in the slot the rows of the tile
    // start at 0, in the output at 0 of the position's column
    float* dst = slot ? slot : out;
    const long long off = slot ? (long long)local * (16 * MH) - 16 * MH * tile
                               : ((long long)py * a.nx + px) * a.out_len;
#pragma unroll
    for (int h = 0; h < MH; ++h)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * MH * tile + 16 * h + 4 * g + i;
        if (row < a.out_len) dst[off + row] = acc[h][t][i];
      }
  }
}

// Waves that share a BF16 stage unit's bundle stream (the split kernel's S).
constexpr int kSplit = 4;

// BF16 staged kernel with each stage unit's bundle stream split over waves.  The four waves
// of a workgroup form 4 / S row groups of the BR x BC patch, and the S waves of a row group
// take every S-th bundle of each unit, so each wave holds NT = BR * BC / (16 * 4 / S)
// position tiles and every table fragment is loaded once per row group (S times fewer table
// loads through the texture-address path per MFMA than with S = 1).  Staging and the LDS row
// ring are those of k_apply_staged.  At the end the S partial sums of a position are added in
// wave order through the LDS, in phases of S tiles (red_bytes() of LDS).
template <int BR, int BC, int MH, int S>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_apply_split(
    const void* __restrict__ pack_raw, const uint16_t* __restrict__ in, float* __restrict__ out,
    StagedArgs a) {
  using T = uint16_t;
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  constexpr int VEC = 8;
  constexpr int TPR = BC / 16;
  constexpr int P = 4 / S;      // row groups
  constexpr int RW = BR / P;    // patch rows per wave
  constexpr int NT = RW * TPR;  // 16-position tiles per wave
  static_assert(4 % S == 0 && BR % P == 0 && NT % S == 0, "split shape");
  constexpr int PF = 2;         // prefetched stage vectors per thread
  constexpr int PD = 2;         // table-fragment ring depth
  constexpr int CSC = kColumnBytes / 2;  // LDS column stride (elements; checked at launch)
  constexpr int CH = 4 * VEC;
  const int4 piece = a.pieces[blockIdx.y];
  const int tile = piece.x;
  const int py0 = (blockIdx.x / a.ncc) * BR, px0 = (blockIdx.x % a.ncc) * BC;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int grp = wave / S, sw = wave % S;
  const int n = lane % 16, g = lane / 16;
  constexpr int nvec = CH / VEC;
  const int rowvec = a.NCOL * nvec;
  floatx4 acc[MH][NT];
#pragma unroll
  for (int h = 0; h < MH; ++h)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[h][t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int u0 = piece.y, u1 = piece.z;
  if (u0 < u1) {
    constexpr int RS = BR + 1;
    u32x4 pf[PF];
    int pf_off[PF];
    AFrag<T, MH> ring[PD];
    {
      const int4 U = a.units[u0];
#pragma unroll
      for (int j = 0; j < PD; ++j)
        load_a<T, MH>(pack_raw, a.meta, min(U.z + sw + S * j, U.w - 1), g, n, ring[j]);
      stage_prefetch<T, RS, PF>(a, in, u0, py0, px0, rowvec, nvec, pf, pf_off);
      stage_rows<T, RS, PF>(a, in, lds, u0, py0, px0, rowvec, nvec, pf, pf_off);
      __syncthreads();
      if (u0 + 1 < u1)
        stage_prefetch<T, RS, PF>(a, in, u0 + 1, py0, px0, rowvec, nvec, pf, pf_off);
    }
    for (int u = u0; u < u1; ++u) {
      const int4 U = a.units[u];
      const int R = U.x + a.K;
      // LDS base of this lane's position in each of the wave's rows for the unit's row offset
      // (eight row bases instead of sixteen tile bases: fewer VGPRs, 3-4 % faster)
      int rb[RW];
#pragma unroll
      for (int r = 0; r < RW; ++r) rb[r] = (((grp * RW + r + R) % RS) * a.NCOL + n) * CSC;
      for (int b0 = U.z + sw; b0 < U.w; b0 += S * PD) {
#pragma unroll
        for (int j = 0; j < PD; ++j) {
          const int b = b0 + S * j;
          if (b < U.w) {
            u32x4 x[NT];
            read_x_rows<T, NT, TPR, CSC>(lds, rb, ring[j].mo, x);
            bundle_mma<T, MH, NT>(ring[j], x, acc);
          }
          load_a<T, MH>(pack_raw, a.meta, min(b + S * PD, U.w - 1), g, n, ring[j]);
        }
      }
      if (u + 1 < u1) {
        const int4 Un = a.units[u + 1];
        const int2 Rn = a.urows[u + 1];
#pragma unroll
        for (int j = 0; j < PD; ++j)
          load_a<T, MH>(pack_raw, a.meta, min(Un.z + sw + S * j, Un.w - 1), g, n, ring[j]);
        const bool free_slot = Rn.y - Rn.x == 1 && Rn.x == R + BR;
        if (!free_slot) __syncthreads();
        stage_rows<T, RS, PF>(a, in, lds, u + 1, py0, px0, rowvec, nvec, pf, pf_off);
        __syncthreads();
        if (u + 2 < u1)
          stage_prefetch<T, RS, PF>(a, in, u + 2, py0, px0, rowvec, nvec, pf, pf_off);
      }
    }
  }
  constexpr int PS = BR * BC * 16 * MH;  // floats per slot and patch
  float* slot =
      piece.w >= 0 ? a.partial + ((long long)piece.w * a.n_patches + blockIdx.x) * PS : nullptr;
  // partial sums of the S waves of a row group, S tiles per phase: wave sw of the group adds
  // tile p + sw over the group's waves (in wave order) and writes it
  floatx4* red = reinterpret_cast<floatx4*>(lds_raw);
  __syncthreads();  // every wave is done with the row ring
#pragma unroll
  for (int p = 0; p < NT; p += S) {
#pragma unroll
    for (int k = 0; k < S; ++k)
#pragma unroll
      for (int h = 0; h < MH; ++h) red[((wave * S + k) * MH + h) * 64 + lane] = acc[h][p + k];
    __syncthreads();
    floatx4 v[MH];
#pragma unroll
    for (int h = 0; h < MH; ++h) {
      v[h] = red[(((grp * S) * S + sw) * MH + h) * 64 + lane];
#pragma unroll
      for (int s = 1; s < S; ++s) v[h] += red[(((grp * S + s) * S + sw) * MH + h) * 64 + lane];
    }
    const int t = p + sw;
    const int py = py0 + grp * RW + t / TPR, px = px0 + (t % TPR) * 16 + n;
    if (py < a.ny && px < a.nx) {
      const int local = (grp * RW + t / TPR) * BC + (t % TPR) * 16 + n;
      float* dst = slot ? slot : out;
      const long long off = slot ? (long long)local * (16 * MH) - 16 * MH * tile
                                 : ((long long)py * a.nx + px) * a.out_len;
#pragma unroll
      for (int h = 0; h < MH; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * MH * tile + 16 * h + 4 * g + i;
          if (row < a.out_len) dst[off + row] = v[h][i];
        }
    }
    __syncthreads();  // the next phase overwrites the sums
  }
}

// LDS bytes of the split kernel's final sums: S tiles of MH halves per wave, four waves.
constexpr size_t red_bytes(int S, int MH) { return (size_t)4 * S * MH * 64 * 16; }

// Output of the cut tiles: the sum of a tile's partial slots in slot order (the order of the
// tile's stage units), written like the staged kernel's own output.  Grid: (patch, tile);
// workgroups of tiles that were not cut return at once.
template <int BR, int BC, int MH>
__global__ __launch_bounds__(256) void k_add_slots(const int2* __restrict__ tile_split,
                                                   const float* __restrict__ partial,
                                                   float* __restrict__ out, int n_patches,
                                                   int ncc, int nx, int ny, int out_len) {
  constexpr int TPR = BC / 16, RW = BR / 4, NT = RW * TPR, TM = 16 * MH;
  constexpr long long PS = (long long)BR * BC * TM;  // floats per slot and patch
  const int tile = blockIdx.y;
  const int2 sp = tile_split[tile];
  if (sp.x < 2) return;
  const int py0 = (blockIdx.x / ncc) * BR, px0 = (blockIdx.x % ncc) * BC;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int n = lane % 16, g = lane / 16;
  const float* base = partial + ((long long)sp.y * n_patches + blockIdx.x) * PS;
  const long long stride = (long long)n_patches * PS;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int py = py0 + wave * RW + t / TPR, px = px0 + (t % TPR) * 16 + n;
    if (py >= ny || px >= nx) continue;
    const int local = (wave * RW + t / TPR) * BC + (t % TPR) * 16 + n;
    float* o = out + ((long long)py * nx + px) * out_len;
#pragma unroll
    for (int h = 0; h < MH; ++h) {
      // four consecutive rows per lane: 16-byte loads and stores
      const long long e = (long long)local * TM + 16 * h + 4 * g;
      floatx4 v = *reinterpret_cast<const floatx4*>(base + e);
      for (int j = 1; j < sp.x; ++j) v += *reinterpret_cast<const floatx4*>(base + j * stride + e);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = TM * tile + 16 * h + 4 * g + i;
        if (row < out_len) o[row] = v[i];
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// FP8 applies: e4m3 table and e4m3 operand on the block-scaled FP8 MFMA
// (v_mfma_scale_f32_16x16x128_f8f6f4).  The operand (image or signals) gets one power-of-two
// scale per chunk of 64 entries of its fast axis over all scan positions, so every K-group of a
// stage unit (one chunk) shares it; the table's scale per (offset, 16-depth block) is carried
// per scale block of a bundle (see the layout).

// NaN-carrying maximum (fmaxf drops a NaN).
__device__ inline float nan_maxf(float a, float b) { return (a > b || a != a) ? a : b; }

// part[c * nparts + p] = max |in| over the entries of chunk c (64 entries of the fast axis) of
// the scan positions p, p + nparts, ...  Grid (nparts, chunks); 256 threads = 4 positions x 64.
__global__ __launch_bounds__(256) void k_chunk_amax(const float* __restrict__ in, long long npos,
                                                    int L, float* __restrict__ part) {
  __shared__ float sh[256];
  const int c = blockIdx.y, nparts = gridDim.x;
  const int e = threadIdx.x % 64, r = threadIdx.x / 64;
  const int l = c * 64 + e;
  float m = 0.0f;
  if (l < L)
    for (long long i = blockIdx.x + (long long)nparts * r; i < npos; i += 4LL * nparts)
      m = nan_maxf(m, fabsf(in[i * L + l]));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = nan_maxf(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long long)c * nparts + blockIdx.x] = sh[0];
}

// Per chunk: the smallest power of two 2^e >= amax / 448 (e = 0 for a chunk of zeros or a
// non-finite amax, whose NaN codes then reach the output), as the E8M0 byte e + 127 and 2^-e.
// 448 = 0.875 2^9, so with amax = m 2^ea (0.5 <= m < 1): e = ea - 9 if m <= 0.875, else ea - 8.
__global__ void k_chunk_scales(const float* __restrict__ part, int nparts, int nch,
                               int* __restrict__ xexp, float* __restrict__ xinv) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nch) return;
  float a = 0.0f;
  for (int p = 0; p < nparts; ++p) a = nan_maxf(a, part[(long long)c * nparts + p]);
  int e = 0;
  if (a > 0.0f && a <= 3.402823466e38f) {
    int ea;
    const float mnt = frexpf(a, &ea);
    e = mnt <= 0.875f ? ea - 9 : ea - 8;
  }
  e = max(-126, min(127, e));
  xexp[c] = e + 127;
  xinv[c] = ldexpf(1.0f, -e);
}

// Stage an FP32 input into the zero-padded e4m3 layout [nyp][nxp][Lp] (codes of x 2^-e of its
// chunk); one workgroup of 64 threads per padded column, each thread four consecutive entries
// (one chunk, since Lp and the chunk are multiples of 4) written as one 32-bit word.  vec4: the
// input rows are 16-byte aligned (L % 4 == 0 and an aligned base), so they load as float4.
__global__ __launch_bounds__(64) void k_stage_fp8(const float* __restrict__ in,
                                                  uint8_t* __restrict__ out,
                                                  const float* __restrict__ xinv, int K, int nx,
                                                  int ny, int nxp, int L, int Lp, int vec4) {
  const int col = blockIdx.x;
  const int px = col % nxp - K, py = col / nxp - K;
  uint32_t* o = reinterpret_cast<uint32_t*>(out + (long long)col * Lp);
  const bool inside = px >= 0 && px < nx && py >= 0 && py < ny;
  const float* src = in + ((long long)py * nx + px) * L;
  for (int q = threadIdx.x; q < Lp / 4; q += blockDim.x) {
    const int l0 = 4 * q;
    uint32_t w = 0;
    if (inside && l0 < L) {
      float v[4];
      if (vec4) {
        const float4 f = *reinterpret_cast<const float4*>(src + l0);
        v[0] = f.x, v[1] = f.y, v[2] = f.z, v[3] = f.w;
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = l0 + i < L ? src[l0 + i] : 0.0f;
      }
      const float sc = xinv[l0 / 64];
#pragma unroll
      for (int i = 0; i < 4; ++i) w |= (uint32_t)f32_to_e4m3(v[i] * sc) << (8 * i);
    }
    o[q] = w;
  }
}

struct Fp8Args {
  const int4* pieces;
  const int2* tile_split;
  float* partial;
  int n_patches;
  const int4* units;
  const int2* urows;
  const u32x4* rec;   // per bundle and lane group: LDS offsets of its 4 K-groups (16 bits
                      // each), the E8M0 scale bytes of its block for the two halves; word 3
                      // of lane group 0: the 16-row halves the bundle's K-groups reach
  const int* xexp;    // per chunk of the operand: E8M0 scale byte
  int out_len, nx, ny, K, nxp, Lp;
  int ncc;
  int NCOL, CS;
};

// Table operand of one FP8 bundle for one lane: 32 bytes per half.
struct F8Frag {
  u32x4 v[2][2];
};

__device__ __forceinline__ void load_f8(const uint8_t* __restrict__ pack, int b, int lane,
                                        F8Frag& f) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const u32x4* p = reinterpret_cast<const u32x4*>(pack + (((long long)b * 2 + h) * 64 + lane) * 32);
    f.v[h][0] = p[0];
    f.v[h][1] = p[1];
  }
}

// One word of lane group g's record for bundle b: lane 4q + j of each quad loads word j, and
// rec8_word broadcasts word J within the quad (a lane needs only its own lane group's words).
// Vector loads, since a record that came through the scalar path would make every wait on the
// LDS reads wait for it as well (scalar loads complete out of order, so the shared counter can
// only be waited to zero); one word per lane, since the texture path bounds this loop.
__device__ __forceinline__ uint32_t load_rec8(const Fp8Args& a, int b, int g, int lane) {
  return reinterpret_cast<const uint32_t*>(a.rec)[((long long)b * kLaneGroups + g) * 4 + (lane & 3)];
}

// Word J of the lane group's record: lane 4q + J of each quad loaded it (quad_perm [J,J,J,J]).
template <int J>
__device__ __forceinline__ uint32_t rec8_word(uint32_t w) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)w, 0x55 * J, 0xF, 0xF, false);
}

// LDS offsets of the lane group's four K-groups in an FP8 bundle (record words 0 and 1).
struct X8Offs {
  int o[4];
};

__device__ __forceinline__ X8Offs x8_offsets(uint32_t w) {
  const uint32_t r0 = rec8_word<0>(w), r1 = rec8_word<1>(w);
  return X8Offs{{(int)(r0 & 0xffff), (int)(r0 >> 16), (int)(r1 & 0xffff), (int)(r1 >> 16)}};
}

// Position fragments of one FP8 bundle for tiles [t0, t0 + NX) of this lane: for each of the
// lane group's four K-groups, 8 bytes of the lane's position from the LDS.  Tile t sits at row
// base rb[t / TPR] plus column offset (t % TPR) * cstep.  The step is a run-time value: as an
// immediate, the compiler pairs the reads of neighbouring tiles into one instruction whose
// registers then have to be moved into each MFMA's operand order.
template <int TPR, int NX, int NR>
__device__ __forceinline__ void read_x8(const uint8_t* lds, const int (&rb)[NR], int cstep, int t0,
                                         const X8Offs& o, u32x4 (&x)[NX][2]) {
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    const int t = t0 + i;
    const uint8_t* p = lds + rb[t / TPR] + (t % TPR) * cstep;
    const u32x2 q0 = *reinterpret_cast<const u32x2*>(p + o.o[0]);
    const u32x2 q1 = *reinterpret_cast<const u32x2*>(p + o.o[1]);
    const u32x2 q2 = *reinterpret_cast<const u32x2*>(p + o.o[2]);
    const u32x2 q3 = *reinterpret_cast<const u32x2*>(p + o.o[3]);
    x[i][0] = u32x4{q0.x, q0.y, q1.x, q1.y};
    x[i][1] = u32x4{q2.x, q2.y, q3.x, q3.y};
  }
}

// The block-scaled MFMAs of half H of one FP8 bundle for tiles [t0, t0 + NX) (t0 a constant
// after unrolling) whose fragments are x[0 .. NX): 16 rows x 128 K x 16 positions each, with
// the lane's block scale byte H of sc and the unit's operand scale xs.
template <int H, int NT, int NX>
__device__ __forceinline__ void fp8_mma_h(const F8Frag& f, int sc, int xs, int t0,
                                          const u32x4 (&x)[NX][2], floatx4 (&acc)[2][NT]) {
  const intx8 av = __builtin_bit_cast(
      intx8, u32x8{f.v[H][0].x, f.v[H][0].y, f.v[H][0].z, f.v[H][0].w, f.v[H][1].x, f.v[H][1].y,
                   f.v[H][1].z, f.v[H][1].w});
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    const intx8 bv = __builtin_bit_cast(intx8, u32x8{x[i][0].x, x[i][0].y, x[i][0].z, x[i][0].w,
                                                     x[i][1].x, x[i][1].y, x[i][1].z, x[i][1].w});
    acc[H][t0 + i] =
        __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(av, bv, acc[H][t0 + i], 0, 0, H, sc, 0, xs);
  }
}

// FP8 split kernel shape: waves sharing a unit's bundle stream, position-fragment read phases
// per bundle, table-fragment ring depth.
constexpr int kSplit8 = 4, kPhases8 = 4, kRing8 = 1;

// LDS-staged FP8 kernel: the BF16 split kernel's workgroup shape, LDS row ring, unit order and
// bundle split (4 / S row groups of the BR x BC patch; the S waves of a row group take every
// S-th bundle of each stage unit; the S partial sums of a position are added in wave order
// through the LDS at the end), with bundles of 16 K-groups: per reached 16-row half and
// position tile one block-scaled MFMA of K = 128.  Lane (n, g) reads, for each of its lane
// group's four K-groups, 8 bytes of position n from the LDS (the K-group's column and run) and
// 32 bytes of table row n per half.  An FP8 position fragment takes 8 VGPRs, so a wave reads
// its NT fragments in XP phases; the table ring is PD bundles deep.
template <int BR, int BC, int S, int XP, int PD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_apply_fp8s(
    const uint8_t* __restrict__ pack, const uint8_t* __restrict__ in, float* __restrict__ out,
    Fp8Args a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  uint8_t* lds = lds_raw;
  constexpr int TPR = BC / 16;
  constexpr int P = 4 / S;
  constexpr int RW = BR / P;
  constexpr int NT = RW * TPR;
  static_assert(4 % S == 0 && BR % P == 0 && NT % S == 0 && NT % XP == 0, "split shape");
  constexpr int NX = NT / XP;          // tiles per position-fragment read phase
  constexpr int PF = 2;
  constexpr int RQ = 2;                // record ring depth (a multiple of PD; 4 measured slower)
  constexpr int MH = 2;
  const int4 piece = a.pieces[blockIdx.y];
  const int tile = piece.x;
  const int py0 = (blockIdx.x / a.ncc) * BR, px0 = (blockIdx.x % a.ncc) * BC;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int grp = wave / S, sw = wave % S;
  const int n = lane % 16, g = lane / 16;
  constexpr int nvec = 4;
  const int rowvec = a.NCOL * nvec;
  StagedArgs sa;
  sa.units = a.units;
  sa.urows = a.urows;
  sa.NCOL = a.NCOL;
  sa.CS = a.CS;
  sa.nxp = a.nxp;
  sa.Lp = a.Lp;
  floatx4 acc[MH][NT];
#pragma unroll
  for (int h = 0; h < MH; ++h)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[h][t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int u0 = piece.y, u1 = piece.z;
  if (u0 < u1) {
    constexpr int RS = BR + 1;
    u32x4 pf[PF];
    int pf_off[PF];
    F8Frag ring[PD];
    uint32_t rq[RQ];
    {
      const int4 U = a.units[u0];
#pragma unroll
      for (int j = 0; j < PD; ++j) load_f8(pack, min(U.z + sw + S * j, U.w - 1), lane, ring[j]);
#pragma unroll
      for (int j = 0; j < RQ; ++j) rq[j] = load_rec8(a, min(U.z + sw + S * j, U.w - 1), g, lane);
      stage_prefetch<uint8_t, RS, PF>(sa, in, u0, py0, px0, rowvec, nvec, pf, pf_off);
      stage_rows<uint8_t, RS, PF>(sa, in, lds, u0, py0, px0, rowvec, nvec, pf, pf_off);
      __syncthreads();
      if (u0 + 1 < u1)
        stage_prefetch<uint8_t, RS, PF>(sa, in, u0 + 1, py0, px0, rowvec, nvec, pf, pf_off);
    }
    for (int u = u0; u < u1; ++u) {
      const int4 U = a.units[u];
      const int xs = a.xexp[U.y / 64];
      const int R = U.x + a.K;
      int rb[RW];  // LDS base of this lane's position in each of the wave's rows
#pragma unroll
      for (int r = 0; r < RW; ++r) rb[r] = (((grp * RW + r + R) % RS) * a.NCOL + n) * a.CS;
      const int cstep = 16 * a.CS;
      for (int b0 = U.z + sw; b0 < U.w; b0 += S * RQ) {
#pragma unroll
        for (int j = 0; j < RQ; ++j) {
          const int b = b0 + S * j;
          const int sc = (int)rec8_word<2>(rq[j]);
          const int hm = b < U.w ? __builtin_amdgcn_readfirstlane((int)rec8_word<3>(rq[j])) : 0;
          if (hm) {
            const X8Offs o = x8_offsets(rq[j]);
#pragma unroll
            for (int ph = 0; ph < XP; ++ph) {
              u32x4 x[NX][2];
              read_x8<TPR, NX>(lds, rb, cstep, ph * NX, o, x);
              if (hm & 1) fp8_mma_h<0, NT, NX>(ring[j % PD], sc, xs, ph * NX, x, acc);
              if (hm & 2) fp8_mma_h<1, NT, NX>(ring[j % PD], sc, xs, ph * NX, x, acc);
            }
          }
          load_f8(pack, min(b + S * PD, U.w - 1), lane, ring[j % PD]);
          rq[j] = load_rec8(a, min(b + S * RQ, U.w - 1), g, lane);
        }
      }
      if (u + 1 < u1) {
        const int4 Un = a.units[u + 1];
        const int2 Rn = a.urows[u + 1];
#pragma unroll
        for (int j = 0; j < PD; ++j)
          load_f8(pack, min(Un.z + sw + S * j, Un.w - 1), lane, ring[j]);
#pragma unroll
        for (int j = 0; j < RQ; ++j)
          rq[j] = load_rec8(a, min(Un.z + sw + S * j, Un.w - 1), g, lane);
        const bool free_slot = Rn.y - Rn.x == 1 && Rn.x == R + BR;
        if (!free_slot) __syncthreads();
        stage_rows<uint8_t, RS, PF>(sa, in, lds, u + 1, py0, px0, rowvec, nvec, pf, pf_off);
        __syncthreads();
        if (u + 2 < u1)
          stage_prefetch<uint8_t, RS, PF>(sa, in, u + 2, py0, px0, rowvec, nvec, pf, pf_off);
      }
    }
  }
  constexpr int PS = BR * BC * 16 * MH;
  float* slot =
      piece.w >= 0 ? a.partial + ((long long)piece.w * a.n_patches + blockIdx.x) * PS : nullptr;
  floatx4* red = reinterpret_cast<floatx4*>(lds_raw);
  __syncthreads();
#pragma unroll
  for (int p = 0; p < NT; p += S) {
#pragma unroll
    for (int k = 0; k < S; ++k)
#pragma unroll
      for (int h = 0; h < MH; ++h) red[((wave * S + k) * MH + h) * 64 + lane] = acc[h][p + k];
    __syncthreads();
    floatx4 v[MH];
#pragma unroll
    for (int h = 0; h < MH; ++h) {
      v[h] = red[(((grp * S) * S + sw) * MH + h) * 64 + lane];
#pragma unroll
      for (int s = 1; s < S; ++s) v[h] += red[(((grp * S + s) * S + sw) * MH + h) * 64 + lane];
    }
    const int t = p + sw;
    const int py = py0 + grp * RW + t / TPR, px = px0 + (t % TPR) * 16 + n;
    if (py < a.ny && px < a.nx) {
      const int local = (grp * RW + t / TPR) * BC + (t % TPR) * 16 + n;
      float* dst = slot ? slot : out;
      const long long off = slot ? (long long)local * (16 * MH) - 16 * MH * tile
                                 : ((long long)py * a.nx + px) * a.out_len;
#pragma unroll
      for (int h = 0; h < MH; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * MH * tile + 16 * h + 4 * g + i;
          if (row < a.out_len) dst[off + row] = v[h][i];
        }
    }
    __syncthreads();
  }
}

ApplyArgs make_args(const Layout& lay) {
  ApplyArgs a;
  a.tile_start = lay.d_tile_start;
  a.meta = lay.d_meta;
  a.out_len = lay.out_len;
  a.n_ntiles = lay.in.ny * lay.in.ntx;
  a.ntx = lay.in.ntx;
  a.nx = lay.in.nx;
  a.K = lay.in.K;
  a.nxp = lay.in.nxp;
  a.Lp = lay.in.Lp;
  return a;
}

size_t elem_bytes(int dtype) {
  switch (dtype) {
    case AROAM_FP64: return 8;
    case AROAM_FP32: return 4;
    case AROAM_BF16: return 2;
    default: return 1;  // e4m3
  }
}

constexpr int kAmaxParts = 512;  // position slices of the FP8 operand's chunk maxima

}  // namespace

const Layout& layout_for(const Model& m, bool adjoint, int dtype) {
  if (dtype == AROAM_FP64) return adjoint ? m.g4a : m.g4f;
  if (dtype == AROAM_FP32) return adjoint ? m.s4a : m.s4f;
  if (dtype == AROAM_BF16) return adjoint ? m.s8a : m.s8f;
  return adjoint ? m.f8a : m.f8f;
}

namespace {

// The stage buffer of an apply: the padded input, then, for a staged layout with cut tiles,
// the partial slots [slot][patch][position of the patch][TM rows] (FP32), then for FP8 the
// operand's chunk scales: partial maxima [chunk][kAmaxParts] (FP32), E8M0 bytes [chunk] (int)
// and inverse scales [chunk] (FP32).
struct StageParts {
  size_t input = 0, partial = 0, scales = 0;
  int chunks = 0;
};

StageParts stage_parts(const Model& m, bool adjoint, int dtype) {
  const Layout& lay = layout_for(m, adjoint, dtype);
  StageParts p;
  p.input = (size_t)round_up(lay.in.elems() * elem_bytes(dtype), 256);
  if (dtype != AROAM_FP64 && lay.n_slots > 0) {
    p.partial = (size_t)lay.n_slots * lay.n_patches * lay.TM * kPatchRows * kPatchCols *
                sizeof(float);
  }
  if (dtype == AROAM_FP8E4M3) {
    p.chunks = (int)ceil_div(lay.in.L, 64);
    p.scales = (size_t)round_up((size_t)p.chunks * (kAmaxParts + 2) * 4, 256);
  }
  return p;
}

}  // namespace

size_t stage_bytes(const Model& m, bool adjoint, int dtype) {
  const StageParts p = stage_parts(m, adjoint, dtype);
  return p.input + p.partial + p.scales;
}

namespace {

// Allow the full LDS of a CU for a kernel, once per device.
template <typename F>
int allow_full_lds(F kern, std::atomic<unsigned long long>& done) {
  int dev = 0;
  AROAM_HIP(hipGetDevice(&dev));
  const unsigned long long bit = 1ull << (dev & 63);
  if (!(done.load() & bit)) {
    AROAM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)kLdsBytes));
    done.fetch_or(bit);
  }
  return AROAM_OK;
}

// Arguments of the staged kernels for a layout (and the partial slots of its cut tiles).
int staged_args(const Layout& lay, float* partial, int elem_size, StagedArgs& a) {
  AROAM_CHECK(lay.lds_bytes <= kLdsBytes, AROAM_EINVAL,
              "lateral footprint too wide for the LDS stage (%zu bytes)", lay.lds_bytes);
  a.pieces = lay.d_pieces;
  a.tile_split = lay.d_tile_split;
  a.partial = partial;
  a.n_patches = lay.n_patches;
  a.units = lay.d_units;
  a.urows = lay.d_ucols;
  a.meta = lay.d_meta;
  a.out_len = lay.out_len;
  a.nx = lay.in.nx;
  a.ny = lay.in.ny;
  a.K = lay.in.K;
  a.nxp = lay.in.nxp;
  a.Lp = lay.in.Lp;
  a.ncc = (int)ceil_div(lay.in.nx, kPatchCols);
  a.NCOL = lay.NCOL;
  a.CS = lay.CS;
  AROAM_CHECK(lay.CH == 4 * (16 / elem_size), AROAM_EINVAL, "chunk length mismatch");
  AROAM_CHECK(lay.n_patches == ceil_div(lay.in.ny, kPatchRows) * a.ncc, AROAM_EINVAL,
              "patch count mismatch");
  AROAM_CHECK(lay.n_slots == 0 || partial, AROAM_EINVAL, "no partial slots for a cut layout");
  return AROAM_OK;
}

// BF16 apply: the split kernel, then the slot sums of cut tiles.
template <int MH>
int launch_split(const Layout& lay, const Pack& pk, const void* buf, float* partial, void* out,
                 hipStream_t st) {
  AROAM_CHECK(lay.TM == 16 * MH, AROAM_EINVAL, "tile height mismatch");
  auto kern = k_apply_split<kPatchRows, kPatchCols, MH, kSplit>;
  static std::atomic<unsigned long long> attr_set{0};
  AROAM_TRY(allow_full_lds(kern, attr_set));
  StagedArgs a;
  AROAM_TRY(staged_args(lay, partial, 2, a));
  AROAM_CHECK(lay.CS * 2 == kColumnBytes, AROAM_EINVAL, "BF16 layout column stride mismatch");
  const size_t lds = std::max(lay.lds_bytes, red_bytes(kSplit, MH));
  const dim3 grid((unsigned)lay.n_patches, (unsigned)lay.n_pieces);
  hipLaunchKernelGGL(kern, grid, dim3(256), lds, st, (const void*)pk.d, (const uint16_t*)buf,
                     (float*)out, a);
  if (lay.n_slots > 0)
    hipLaunchKernelGGL((k_add_slots<kPatchRows, kPatchCols, MH>),
                       dim3((unsigned)lay.n_patches, (unsigned)lay.n_tiles), dim3(256), 0, st,
                       lay.d_tile_split, (const float*)partial, (float*)out, lay.n_patches, a.ncc,
                       a.nx, a.ny, a.out_len);
  return AROAM_OK;
}

template <typename T, int MH>
int launch_staged(const Layout& lay, const Pack& pk, const void* buf, float* partial, void* out,
                  hipStream_t st) {
  static_assert(kPatchRows % 4 == 0 && kPatchCols % 16 == 0, "patch shape");
  AROAM_CHECK(lay.TM == 16 * MH, AROAM_EINVAL, "tile height mismatch");
  auto kern = k_apply_staged<T, kPatchRows, kPatchCols, MH>;
  static std::atomic<unsigned long long> attr_set{0};
  AROAM_TRY(allow_full_lds(kern, attr_set));
  StagedArgs a;
  AROAM_TRY(staged_args(lay, partial, (int)sizeof(T), a));
  const dim3 grid((unsigned)lay.n_patches, (unsigned)lay.n_pieces);
  hipLaunchKernelGGL(kern, grid, dim3(256), lay.lds_bytes, st, (const void*)pk.d, (const T*)buf,
                     (float*)out, a);
  if (lay.n_slots > 0)
    hipLaunchKernelGGL((k_add_slots<kPatchRows, kPatchCols, MH>),
                       dim3((unsigned)lay.n_patches, (unsigned)lay.n_tiles), dim3(256), 0, st,
                       lay.d_tile_split, (const float*)partial, (float*)out, lay.n_patches, a.ncc,
                       a.nx, a.ny, a.out_len);
  return AROAM_OK;
}

}  // namespace

namespace {

// FP8 apply: chunk maxima and scales of the operand, the e4m3 staging, the staged FP8 kernel,
// and the slot sums of cut tiles.
int launch_fp8(const Model& m, const Layout& lay, const Pack& pk, const float* in, void* buf,
               const StageParts& sp, void* out, hipStream_t st) {
  auto kern = k_apply_fp8s<kPatchRows, kPatchCols, kSplit8, kPhases8, kRing8>;
  static std::atomic<unsigned long long> attr_set{0};
  AROAM_TRY(allow_full_lds(kern, attr_set));
  AROAM_CHECK(lay.TM == kTileRows8 && lay.CH == 64 && lay.CS == kColumnBytes, AROAM_EINVAL,
              "FP8 layout shape mismatch");
  const PadGeom& pg = lay.in;
  char* base = static_cast<char*>(buf);
  uint8_t* staged = reinterpret_cast<uint8_t*>(base);
  float* partial = sp.partial > 0 ? reinterpret_cast<float*>(base + sp.input) : nullptr;
  float* amax = reinterpret_cast<float*>(base + sp.input + sp.partial);
  int* xexp = reinterpret_cast<int*>(amax + (size_t)sp.chunks * kAmaxParts);
  float* xinv = reinterpret_cast<float*>(xexp + sp.chunks);
  const long long npos = (long long)pg.nx * pg.ny;
  hipLaunchKernelGGL(k_chunk_amax, dim3(kAmaxParts, (unsigned)sp.chunks), dim3(256), 0, st, in,
                     npos, pg.L, amax);
  hipLaunchKernelGGL(k_chunk_scales, dim3((unsigned)ceil_div(sp.chunks, 64)), dim3(64), 0, st,
                     (const float*)amax, kAmaxParts, sp.chunks, xexp, xinv);
  AROAM_CHECK(pg.Lp % 64 == 0, AROAM_EINVAL, "FP8 staging needs whole 64-entry chunks");
  const int vec4 = pg.L % 4 == 0 && reinterpret_cast<uintptr_t>(in) % 16 == 0;
  hipLaunchKernelGGL(k_stage_fp8, dim3((unsigned)(pg.nyp * pg.nxp)), dim3(64), 0, st, in, staged,
                     (const float*)xinv, pg.K, pg.nx, pg.ny, pg.nxp, pg.L, pg.Lp, vec4);
  Fp8Args a;
  a.pieces = lay.d_pieces;
  a.tile_split = lay.d_tile_split;
  a.partial = partial;
  a.n_patches = lay.n_patches;
  a.units = lay.d_units;
  a.urows = lay.d_ucols;
  a.rec = reinterpret_cast<const u32x4*>(lay.d_meta);
  a.xexp = xexp;
  a.out_len = lay.out_len;
  a.nx = pg.nx;
  a.ny = pg.ny;
  a.K = pg.K;
  a.nxp = pg.nxp;
  a.Lp = pg.Lp;
  a.ncc = (int)ceil_div(pg.nx, kPatchCols);
  a.NCOL = lay.NCOL;
  a.CS = lay.CS;
  AROAM_CHECK(lay.n_patches == ceil_div(pg.ny, kPatchRows) * a.ncc, AROAM_EINVAL,
              "patch count mismatch");
  AROAM_CHECK(lay.n_slots == 0 || partial, AROAM_EINVAL, "no partial slots for a cut layout");
  const dim3 grid((unsigned)lay.n_patches, (unsigned)lay.n_pieces);
  hipLaunchKernelGGL(kern, grid, dim3(256), std::max(lay.lds_bytes, red_bytes(kSplit8, 2)), st,
                     (const uint8_t*)pk.d, (const uint8_t*)staged, (float*)out, a);
  if (lay.n_slots > 0)
    hipLaunchKernelGGL((k_add_slots<kPatchRows, kPatchCols, 2>),
                       dim3((unsigned)lay.n_patches, (unsigned)lay.n_tiles), dim3(256), 0, st,
                       lay.d_tile_split, (const float*)partial, (float*)out, lay.n_patches, a.ncc,
                       a.nx, a.ny, a.out_len);
  return AROAM_OK;
}

// The launches of one apply into the stage buffer `buf` (stage_bytes() bytes).
int launch_apply(const Model& m, bool adjoint, int dtype, const void* in, void* out, void* buf,
                 hipStream_t st) {
  const Layout& lay = layout_for(m, adjoint, dtype);
  const Pack& pk = adjoint ? m.adj_pack[dtype] : m.fwd_pack[dtype];
  const PadGeom& pg = lay.in;
  const dim3 sgrid((unsigned)(pg.nyp * pg.nxp));
  if (dtype == AROAM_FP8E4M3) {
    AROAM_TRY(launch_fp8(m, lay, pk, (const float*)in, buf, stage_parts(m, adjoint, dtype), out,
                         st));
    AROAM_HIP(hipGetLastError());
    return AROAM_OK;
  }
  if (dtype == AROAM_FP64)
    hipLaunchKernelGGL((k_stage<double, double>), sgrid, dim3(256), 0, st, (const double*)in,
                       (double*)buf, pg.K, pg.nx, pg.ny, pg.nxp, pg.L, pg.Lp);
  else if (dtype == AROAM_FP32)
    hipLaunchKernelGGL((k_stage<float, float>), sgrid, dim3(256), 0, st, (const float*)in,
                       (float*)buf, pg.K, pg.nx, pg.ny, pg.nxp, pg.L, pg.Lp);
  else
    hipLaunchKernelGGL((k_stage<float, uint16_t>), sgrid, dim3(256), 0, st, (const float*)in,
                       (uint16_t*)buf, pg.K, pg.nx, pg.ny, pg.nxp, pg.L, pg.Lp);
  if (dtype == AROAM_FP64) {
    const ApplyArgs a = make_args(lay);
    const dim3 grid((unsigned)a.n_ntiles, (unsigned)lay.n_tiles);
    hipLaunchKernelGGL(k_apply_fma<double>, grid, dim3(256), 0, st, (const double*)pk.d,
                       (const double*)buf, (double*)out, a, lay.G);
  } else {
    const StageParts sp = stage_parts(m, adjoint, dtype);
    float* partial =
        sp.partial > 0 ? reinterpret_cast<float*>(static_cast<char*>(buf) + sp.input) : nullptr;
    if (dtype == AROAM_FP32)
      AROAM_TRY((launch_staged<float, 1>(lay, pk, buf, partial, out, st)));
    else
      AROAM_TRY((launch_split<kTileRows8 / 16>(lay, pk, buf, partial, out, st)));
  }
  AROAM_HIP(hipGetLastError());
  return AROAM_OK;
}

}  // namespace

int apply(const Model& m, bool adjoint, int dtype, const void* in, void* out, void* stage,
          hipStream_t st) {
  AROAM_CHECK(dtype >= AROAM_FP64 && dtype <= AROAM_FP8E4M3, AROAM_EINVAL, "bad dtype %d", dtype);
  AROAM_CHECK(in && out, AROAM_EINVAL, "NULL vector");
  AROAM_CHECK((m.dtype_mask >> dtype) & 1u, AROAM_EUNSUPPORTED,
              "model was not packed for dtype %d", dtype);
  const Layout& lay = layout_for(m, adjoint, dtype);
  AROAM_CHECK(!lay.staged || lay.lds_bytes <= kLdsBytes, AROAM_EINVAL,
              "lateral footprint too wide for the LDS stage (%zu bytes)", lay.lds_bytes);
  if (stage) return launch_apply(m, adjoint, dtype, in, out, stage, st);
  // a stage buffer of its own from the pool, returned to the pool on every path
  void* buf = nullptr;
  AROAM_TRY(pool_alloc(&buf, stage_bytes(m, adjoint, dtype), st));
  const int rc = launch_apply(m, adjoint, dtype, in, out, buf, st);
  const hipError_t e = hipFreeAsync(buf, st);
  if (rc != AROAM_OK) return rc;
  AROAM_CHECK(e == hipSuccess, AROAM_EDEVICE, "hipFreeAsync failed: %s", hipGetErrorString(e));
  return AROAM_OK;
}

// Stage buffer of the allocation-free applies: a static device array, one copy per GPU the
// library runs on, held until the process ends.  In host code `scratch` names a host-side
// stand-in, so its device address is looked up once per device and only that address is
// passed to kernels.
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

int static_scratch(void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  AROAM_HIP(hipGetDevice(&dev));
  AROAM_CHECK(dev >= 0 && dev < kMaxDevices, AROAM_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    AROAM_CHECK(e == hipSuccess && p, AROAM_EDEVICE,
                "hipGetSymbolAddress of the static scratch buffer failed: %s", hipGetErrorString(e));
    addr[dev] = p;
  }
  *out = addr[dev];
  return AROAM_OK;
}

}  // namespace

int apply_noalloc(const Model& m, bool adjoint, int dtype, const void* in, void* out,
                  hipStream_t st) {
  AROAM_CHECK(dtype >= AROAM_FP64 && dtype <= AROAM_FP8E4M3, AROAM_EINVAL, "bad dtype %d", dtype);
  AROAM_CHECK(in && out, AROAM_EINVAL, "NULL vector");
  AROAM_CHECK((m.dtype_mask >> dtype) & 1u, AROAM_EUNSUPPORTED,
              "model was not packed for dtype %d", dtype);
  const Layout& lay = layout_for(m, adjoint, dtype);
  AROAM_CHECK(!lay.staged || lay.lds_bytes <= kLdsBytes, AROAM_EINVAL,
              "lateral footprint too wide for the LDS stage (%zu bytes)", lay.lds_bytes);
  const size_t need = stage_bytes(m, adjoint, dtype);
  AROAM_CHECK(need <= kStaticScratchBytes, AROAM_EINVAL,
              "the apply needs %zu bytes of scratch; the static buffer holds %zu", need,
              (size_t)kStaticScratchBytes);
  void* buf = nullptr;
  AROAM_TRY(static_scratch(&buf));
  return launch_apply(m, adjoint, dtype, in, out, buf, st);
}

int apply_batch(int n, const Model* const* ms, bool adjoint, int dtype, const float* const* in,
                float* const* out, hipStream_t st) {
  AROAM_CHECK(n >= 0 && (n == 0 || (ms && in && out)), AROAM_EINVAL, "bad batch arguments");
  // the batch's vectors are FP32: FP64 applies would read and write doubles
  AROAM_CHECK(dtype == AROAM_FP32 || dtype == AROAM_BF16 || dtype == AROAM_FP8E4M3, AROAM_EINVAL,
              "batched applies take FP32, BF16 or FP8 (dtype %d)", dtype);
  for (int i = 0; i < n; ++i) {
    AROAM_CHECK(ms[i], AROAM_EINVAL, "NULL model in batch");
    AROAM_TRY(apply(*ms[i], adjoint, dtype, in[i], out[i], nullptr, st));
  }
  return AROAM_OK;
}

}  // namespace aroam
