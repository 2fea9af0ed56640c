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
// K-groups.  Kernels: a plain FP64/FP32 FMA kernel, FP32 MFMA (v_mfma_f32_16x16x4f32) and
// BF16 MFMA (v_mfma_f32_16x16x32_bf16) on gfx950.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "internal.h"

namespace aroam {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx2 __attribute__((ext_vector_type(2)));


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
  const int* tile_units;
  const int4* units;
  const int2* ucols;
  const int* meta;
  int out_len, nx, ny, K, nxp, Lp;
  int ncc;         // patch column chunks
  int NCOL, CS, CH;
};

// LDS-staged MFMA kernel.  A workgroup (4 waves) owns one output tile (16 rows) and one patch
// of BR scan rows x BC scan columns; each wave owns BR/4 rows x BC columns = NT 16-position
// tiles.  Per stage unit (dy, chunk) the patch's input rows shifted by dy, the unit's column
// window and the chunk's CH inner entries are copied to LDS; then every bundle of the unit
// multiplies the 16 x (4 G) table block (from global memory, shared by the 4 waves through
// L1) with the NT position tiles read from LDS.  Lane (n = lane % 16, g = lane / 16) holds
// row n of K-group g of the table and the entries of K-group g for position n.
template <typename T, int BR, int BC, bool FP8A>
__global__ __launch_bounds__(256) void k_apply_staged(const void* __restrict__ pack_raw,
                                                      const float* __restrict__ gscale,
                                                      const T* __restrict__ in,
                                                      float* __restrict__ out, StagedArgs a) {
  const T* pack = reinterpret_cast<const T*>(pack_raw);
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  T* lds = reinterpret_cast<T*>(lds_raw);
  constexpr int VEC = 16 / sizeof(T);  // entries per 16-byte vector == K-group width G
  constexpr int TPR = BC / 16;
  constexpr int RW = BR / 4;
  constexpr int NT = RW * TPR;
  const int tile = blockIdx.y;
  const int py0 = (blockIdx.x / a.ncc) * BR, px0 = (blockIdx.x % a.ncc) * BC;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int n = lane % 16, g = lane / 16;
  int lbase[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int r = wave * RW + t / TPR, c = (t % TPR) * 16 + n;
    lbase[t] = (r * a.NCOL + c) * a.CS;
  }
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int u0 = a.tile_units[tile], u1 = a.tile_units[tile + 1];
  const int nvec = a.CH / VEC;
  for (int u = u0; u < u1; ++u) {
    const int4 U = a.units[u];   // (row offset, chunk start, bundle begin, bundle end)
    const int2 C = a.ucols[u];   // staged columns [C.x, C.y)
    const int ncols = C.y - C.x;
    const int total = BR * ncols * nvec;
    __syncthreads();
    for (int idx = threadIdx.x; idx < total; idx += 256) {
      const int v = idx % nvec;
      const int rc = idx / nvec;
      const int c = C.x + rc % ncols, r = rc / ncols;
      const long long src =
          ((long long)(py0 + r + U.x + a.K) * a.nxp + (px0 + c)) * a.Lp + U.y + v * VEC;
      *reinterpret_cast<uint4*>(lds + (r * a.NCOL + c) * a.CS + v * VEC) =
          *reinterpret_cast<const uint4*>(in + src);
    }
    __syncthreads();
    for (int b = U.z; b < U.w; ++b) {
      const int q = b * kLaneGroups + g;
      uint4 araw;
      if constexpr (FP8A) {
        // e4m3 table entries: decode 8 values, apply the K-group's scale, round to BF16
        const uint2 r8 = *reinterpret_cast<const uint2*>(
            reinterpret_cast<const uint8_t*>(pack_raw) + ((long long)q * 16 + n) * 8);
        const float sc = gscale[q];
        bf16x8 av;
        const floatx2 f0 = __builtin_amdgcn_cvt_pk_f32_fp8((int)r8.x, false);
        const floatx2 f1 = __builtin_amdgcn_cvt_pk_f32_fp8((int)r8.x, true);
        const floatx2 f2 = __builtin_amdgcn_cvt_pk_f32_fp8((int)r8.y, false);
        const floatx2 f3 = __builtin_amdgcn_cvt_pk_f32_fp8((int)r8.y, true);
        av[0] = (__bf16)(f0.x * sc);
        av[1] = (__bf16)(f0.y * sc);
        av[2] = (__bf16)(f1.x * sc);
        av[3] = (__bf16)(f1.y * sc);
        av[4] = (__bf16)(f2.x * sc);
        av[5] = (__bf16)(f2.y * sc);
        av[6] = (__bf16)(f3.x * sc);
        av[7] = (__bf16)(f3.y * sc);
        araw = *reinterpret_cast<const uint4*>(&av);
      } else {
        araw = *reinterpret_cast<const uint4*>(pack + ((long long)q * 16 + n) * VEC);
      }
      const int mo = a.meta[q];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const uint4 xraw = *reinterpret_cast<const uint4*>(lds + lbase[t] + mo);
        if constexpr (sizeof(T) == 4) {
          const float4 av = *reinterpret_cast<const float4*>(&araw);
          const float4 xv = *reinterpret_cast<const float4*>(&xraw);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.x, xv.x, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.y, xv.y, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.z, xv.z, acc[t], 0, 0, 0);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av.w, xv.w, acc[t], 0, 0, 0);
        } else {
          const bf16x8 av = *reinterpret_cast<const bf16x8*>(&araw);
          const bf16x8 xv = *reinterpret_cast<const bf16x8*>(&xraw);
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, xv, acc[t], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int py = py0 + wave * RW + t / TPR, px = px0 + (t % TPR) * 16 + n;
    if (py >= a.ny || px >= a.nx) continue;
    float* o = out + ((long long)py * a.nx + px) * a.out_len;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = kTile * tile + 4 * g + i;
      if (row < a.out_len) o[row] = acc[t][i];
    }
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
    default: return 2;  // BF16 and FP8 stage their vector operand as BF16
  }
}

}  // namespace

const Layout& layout_for(const Model& m, bool adjoint, int dtype) {
  if (dtype == AROAM_FP64) return adjoint ? m.g4a : m.g4f;
  if (dtype == AROAM_FP32) return adjoint ? m.s4a : m.s4f;
  return adjoint ? m.s8a : m.s8f;
}

size_t stage_bytes(const Model& m, bool adjoint, int dtype) {
  const Layout& lay = layout_for(m, adjoint, dtype);
  return (size_t)round_up(lay.in.elems() * elem_bytes(dtype), 256);
}

namespace {

template <typename T, bool FP8A>
int launch_staged(const Layout& lay, const Pack& pk, const void* buf, void* out, hipStream_t st) {
  static_assert(kPatchRows % 4 == 0 && kPatchCols % 16 == 0, "patch shape");
  auto kern = k_apply_staged<T, kPatchRows, kPatchCols, FP8A>;
  static bool attr_set = false;  // allow the full LDS of a CU for wide footprints
  if (!attr_set) {
    AROAM_HIP(hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  160 * 1024));
    attr_set = true;
  }
  AROAM_CHECK(lay.lds_bytes <= 160 * 1024, AROAM_EINVAL,
              "lateral footprint too wide for the LDS stage (%zu bytes)", lay.lds_bytes);
  StagedArgs a;
  a.tile_units = lay.d_tile_units;
  a.units = lay.d_units;
  a.ucols = lay.d_ucols;
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
  a.CH = lay.CH;
  const dim3 grid((unsigned)(ceil_div(lay.in.ny, kPatchRows) * a.ncc), (unsigned)lay.n_tiles);
  hipLaunchKernelGGL(kern, grid, dim3(256), lay.lds_bytes, st, (const void*)pk.d,
                     (const float*)pk.d_scale, (const T*)buf, (float*)out, a);
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
  const Pack& pk = adjoint ? m.adj_pack[dtype] : m.fwd_pack[dtype];
  const PadGeom& pg = lay.in;
  void* buf = stage;
  if (!buf) AROAM_HIP(hipMallocAsync(&buf, stage_bytes(m, adjoint, dtype), st));
  const dim3 sgrid((unsigned)(pg.nyp * pg.nxp));
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
  } else if (dtype == AROAM_FP32) {
    AROAM_TRY((launch_staged<float, false>(lay, pk, buf, out, st)));
  } else if (dtype == AROAM_BF16) {
    AROAM_TRY((launch_staged<uint16_t, false>(lay, pk, buf, out, st)));
  } else {
    AROAM_TRY((launch_staged<uint16_t, true>(lay, pk, buf, out, st)));
  }
  AROAM_HIP(hipGetLastError());
  if (!stage) AROAM_HIP(hipFreeAsync(buf, st));
  return AROAM_OK;
}

int apply_batch(int n, const Model* const* ms, bool adjoint, int dtype, const float* const* in,
                float* const* out, hipStream_t st) {
  AROAM_CHECK(n >= 0 && (n == 0 || (ms && in && out)), AROAM_EINVAL, "bad batch arguments");
  for (int i = 0; i < n; ++i) {
    AROAM_CHECK(ms[i], AROAM_EINVAL, "NULL model in batch");
    AROAM_TRY(apply(*ms[i], adjoint, dtype, in[i], out[i], nullptr, st));
  }
  return AROAM_OK;
}

}  // namespace aroam
