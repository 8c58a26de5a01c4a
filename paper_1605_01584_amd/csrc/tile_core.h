// Device core of the all-pairs tile computation, shared by the uniform
// kernels (tiles.hip) and the uneven-batch kernel (batched.hip).
//
// One call computes one TILE x TILE tile (yt, xt) of Z Z^T (Eq. (5)) with a
// 256-thread workgroup: 4 waves in a 2 x 2 grid, each wave a (TILE/2)^2
// block of 32 x 32 MFMA blocks with FP32 accumulators in registers for the
// whole K loop.  K loop: one 128-byte chunk of every row per stage (32 FP32
// samples, 32 split hi+lo samples, or 64 BF16/FP16 samples), staged
// global -> VGPR -> LDS, double buffered with one barrier per stage.  In LDS
// a row is 8 units of 16 bytes, unit u of row r at slot u ^ (r & 7), so the
// ds_read_b128 of 32 rows by a half-wave hit distinct banks.
//
// Sample assignment inside a chunk (any assignment works as long as both
// operands use the same one, since the contraction sums over all samples):
//   FP32   step t = 0..3, lane half g reads unit 2t+g (4 samples) and feeds
//          them to 4 consecutive 32x32x2 MFMAs (K = 2: one sample per half);
//   BF16/FP16  step t = 0..3, half g reads unit 2t+g (8 samples), one
//          32x32x16 MFMA;
//   SPLIT  step t = 0..1, half g reads hi unit 2t+g and lo unit 4+2t+g of
//          the same 8 samples; three 32x32x16 MFMAs lo.hi + hi.lo + hi.hi
//          into one FP32 accumulator (the lo.lo term, ~2^-16 of r, dropped).
#pragma once

#include "pcc_internal.h"

namespace pcc {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

enum { EPI_PACKED = 0, EPI_EDGES = 1 };

// Z operand of one tile computation.
struct ZView {
  const unsigned char *z;
  int64_t row_bytes;
  int64_t n;
  int32_t nchunks;
  float scale;  // accumulator -> r (FP16 layout: 1/l)
};

// Output of one tile computation.
struct EpiArgs {
  float *r;                 // packed strict upper triangle
  float thr;                // edges: |r| >= thr
  int32_t *ij;
  float *rv;
  int64_t cap;
  unsigned long long *count;
};

template <int TILE> struct TileShape {
  static constexpr int WT = TILE / 2;    // wave tile side
  static constexpr int NB = WT / 32;     // MFMA blocks per wave side
  static constexpr int OPU = TILE * 8;   // LDS units per operand per stage
  static constexpr int LPT = OPU / 256;  // units per thread per operand
  static constexpr int LDS_UNITS = 2 * 2 * OPU;  // [buffer][A | B]
};

__device__ __forceinline__ float clamp_unit(float r) {
  // NaN passes through (both comparisons false).
  return r > 1.0f ? 1.0f : (r < -1.0f ? -1.0f : r);
}

template <int MODE, int NB>
__device__ __forceinline__ void mma_stage(const u32x4 *__restrict__ sa, const u32x4 *__restrict__ sb,
                                          int i, int g, f32x16 (&acc)[NB][NB]) {
  const int sw = i & 7;
  if constexpr (MODE == PCC_FP32) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int uu = (2 * t + g) ^ sw;
      f32x4 a[NB], b[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        a[q] = __builtin_bit_cast(f32x4, sa[(q * 32 + i) * 8 + uu]);
        b[q] = __builtin_bit_cast(f32x4, sb[(q * 32 + i) * 8 + uu]);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int p = 0; p < NB; ++p)
#pragma unroll
          for (int q = 0; q < NB; ++q)
            acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p][e], b[q][e], acc[p][q], 0, 0, 0);
    }
  } else if constexpr (MODE == PCC_SPLIT_BF16X3) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int uh = (2 * t + g) ^ sw;
      const int ul = (4 + 2 * t + g) ^ sw;
      bf16x8 ah[NB], al[NB], bh[NB], bl[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        ah[q] = __builtin_bit_cast(bf16x8, sa[(q * 32 + i) * 8 + uh]);
        al[q] = __builtin_bit_cast(bf16x8, sa[(q * 32 + i) * 8 + ul]);
        bh[q] = __builtin_bit_cast(bf16x8, sb[(q * 32 + i) * 8 + uh]);
        bl[q] = __builtin_bit_cast(bf16x8, sb[(q * 32 + i) * 8 + ul]);
      }
#pragma unroll
      for (int p = 0; p < NB; ++p)
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[p], bh[q], acc[p][q], 0, 0, 0);
          acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[p], bl[q], acc[p][q], 0, 0, 0);
          acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[p], bh[q], acc[p][q], 0, 0, 0);
        }
    }
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int uu = (2 * t + g) ^ sw;
      u32x4 a[NB], b[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        a[q] = sa[(q * 32 + i) * 8 + uu];
        b[q] = sb[(q * 32 + i) * 8 + uu];
      }
#pragma unroll
      for (int p = 0; p < NB; ++p)
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if constexpr (MODE == PCC_BF16)
            acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, a[p]), __builtin_bit_cast(bf16x8, b[q]), acc[p][q], 0, 0, 0);
          else
            acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                __builtin_bit_cast(f16x8, a[p]), __builtin_bit_cast(f16x8, b[q]), acc[p][q], 0, 0, 0);
        }
    }
  }
}

// Compute tile (yt, xt) and write its strict-upper-triangle pairs.
// Requires: all 256 threads of the workgroup call it together; smem holds
// TileShape<TILE>::LDS_UNITS units; rows yt*TILE .. +TILE and xt*TILE ..
// +TILE exist in Z (n_pad is a multiple of 256).
template <int MODE, int TILE, int EPI>
__device__ __forceinline__ void do_tile(const ZView &zv, const EpiArgs &ea, int64_t yt, int64_t xt,
                                        u32x4 *__restrict__ smem) {
  using S = TileShape<TILE>;
  constexpr int WT = S::WT, NB = S::NB, OPU = S::OPU, LPT = S::LPT;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int i = lane & 31, g = lane >> 5;

  const unsigned char *za = zv.z + yt * TILE * zv.row_bytes;
  const unsigned char *zb = zv.z + xt * TILE * zv.row_bytes;

  f32x16 acc[NB][NB];
#pragma unroll
  for (int p = 0; p < NB; ++p)
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[p][q][v] = 0.0f;

  // Thread tid stages rows tid/8 + 32 s (s < LPT), unit tid % 8: eight
  // threads cover one 128-byte row chunk, so each load reads whole lines.
  // Row r0 + 32 s keeps the swizzle of row r0, so slot and offset advance by
  // constants with s.
  const int u0 = tid & 7, r0 = tid >> 3;
  const int64_t goff = (int64_t)r0 * zv.row_bytes + u0 * 16;
  const int64_t gstep = 32 * zv.row_bytes;
  const int lslot = r0 * 8 + (u0 ^ (r0 & 7));
  u32x4 ra[LPT], rb[LPT];
#pragma unroll
  for (int s = 0; s < LPT; ++s) {
    ra[s] = *reinterpret_cast<const u32x4 *>(za + goff + s * gstep);
    rb[s] = *reinterpret_cast<const u32x4 *>(zb + goff + s * gstep);
  }
  __syncthreads();  // the previous tile's last reads of smem are done
#pragma unroll
  for (int s = 0; s < LPT; ++s) {
    smem[lslot + 256 * s] = ra[s];
    smem[OPU + lslot + 256 * s] = rb[s];
  }
  __syncthreads();
  for (int c = 0; c < zv.nchunks; ++c) {
    const int buf = c & 1;
    const bool more = c + 1 < zv.nchunks;
    if (more) {
      const int64_t cb = (int64_t)(c + 1) * 128;
#pragma unroll
      for (int s = 0; s < LPT; ++s) {
        ra[s] = *reinterpret_cast<const u32x4 *>(za + goff + s * gstep + cb);
        rb[s] = *reinterpret_cast<const u32x4 *>(zb + goff + s * gstep + cb);
      }
    }
    const u32x4 *base = smem + buf * 2 * OPU;
    mma_stage<MODE, NB>(base + (wr * WT) * 8, base + OPU + (wc * WT) * 8, i, g, acc);
    if (more) {
      u32x4 *nb = smem + (buf ^ 1) * 2 * OPU;
#pragma unroll
      for (int s = 0; s < LPT; ++s) {
        nb[lslot + 256 * s] = ra[s];
        nb[OPU + lslot + 256 * s] = rb[s];
      }
    }
    __syncthreads();
  }

  // Epilogue.  Lane holds column x0 + 32q + i of block (p, q); accumulator
  // register v holds row 8*(v/4) + 4*g + (v%4) of the block.  Row y of the
  // packed triangle starts at F_{n-1}(y) - y - 1 + x.
  const int64_t n = zv.n;
  const int64_t y0 = yt * TILE + wr * WT;
  const int64_t x0 = xt * TILE + wc * WT;
#pragma unroll
  for (int p = 0; p < NB; ++p) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t y = y0 + p * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
      const int64_t rowbase = tri_F(n - 1, y) - 1 - y;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int64_t x = x0 + q * 32 + i;
        if (y < x && x < n) {
          const float rv = clamp_unit(acc[p][q][v] * zv.scale);
          if constexpr (EPI == EPI_PACKED) {
            __builtin_nontemporal_store(rv, ea.r + rowbase + x);
          } else {
            if (fabsf(rv) >= ea.thr) {
              const unsigned long long s = atomicAdd(ea.count, 1ull);
              if ((int64_t)s < ea.cap) {
                ea.ij[2 * s] = (int32_t)y;
                ea.ij[2 * s + 1] = (int32_t)x;
                ea.rv[s] = rv;
              }
            }
          }
        }
      }
    }
  }
}

__device__ __forceinline__ int64_t xcd_slot(int64_t b, int64_t G) {
  // Workgroups are dispatched to the 8 XCDs round robin (b % 8); give the
  // workgroups of one XCD consecutive job ids so they share L2 lines.
  return (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
}

}  // namespace pcc
