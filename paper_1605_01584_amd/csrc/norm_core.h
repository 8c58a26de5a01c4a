// Device core of the variable transformation, Eq. (4), shared by the
// single-matrix kernel (normalize.hip) and the uneven-batch kernel
// (batched.hip).
//
// A group of G lanes (16, 32 or 64: a whole wave by default, several short
// rows per wave in a batch) owns one row.  The row is read once from HBM with
// coalesced 16-byte loads, kept in registers in its input type (units of 4
// or 8 consecutive samples per lane, up to kCache units per lane; longer rows
// are re-read, from L2, by the later passes), and reduced across the wave in
// FP64:
//   pass 1  mean = sum x / l
//   pass 2  M2   = sum (x - mean)^2          (sum of squared deviations, as
//                                             the transformation algorithm
//                                             computes it: no division by l)
//   pass 3  z    = (x - mean) / sqrt(M2)     in FP64, rounded to the mode's
//                                             format, stored as 16-byte units
//                                             of the Z layout.
#pragma once

#include <math.h>

#include "pcc_internal.h"

namespace pcc {

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Sum over the G lanes of a group (G a power of two dividing 64; every lane
// of the group takes part).
__device__ __forceinline__ double group_sum(double v, int G) {
  for (int off = G >> 1; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Lanes that own one row in the variable transformation: the fewest of 4,
// 8, ..., 64 whose registers hold a padded row at 32 samples per lane, so
// short rows share a wave (at least 4 lanes, so that a row's loads still
// cover 64 contiguous bytes or more).  One rule for the single-matrix and the
// batched kernels: the lane count fixes the order of the FP64 sums, and both
// must produce the same Z.
inline int norm_lanes(int64_t l_pad) {
  int g = 4;
  while (g < 64 && (int64_t)g * 32 < l_pad) g *= 2;
  return g;
}

// Samples per 16-byte output unit.
template <int MODE> struct UnitOf {
  static constexpr int E = (MODE == PCC_FP64) ? 2 : ((MODE == PCC_FP32) ? 4 : 8);
};

// Input units cached in registers per lane: 32 samples, so a row of up to
// 2048 samples held by a whole wave stays in registers for all three passes
// (more would cost occupancy: 64 samples halve the waves per SIMD and
// measured slower); the rest of a longer row is staged in LDS.
template <typename TIn, int MODE> struct CacheOf {
  static constexpr int C = 32 / UnitOf<MODE>::E;
};

template <typename TIn, int E, bool VEC>
__device__ __forceinline__ void load_unit(const TIn *row, int l, int k0, TIn (&v)[E]) {
  if (!VEC && k0 + E <= l) {
    // a whole unit of a row that need not start 16-byte aligned: copied at
    // the element type's alignment, which gfx950 loads with 16-byte (or
    // 8-byte) vector loads just the same
    __builtin_memcpy(v, row + k0, E * sizeof(TIn));
  } else if (VEC && k0 + E <= l) {
    if constexpr (sizeof(TIn) == 4 && E == 2) {
      const float2 f = *reinterpret_cast<const float2 *>(row + k0);
      v[0] = f.x; v[1] = f.y;
    } else if constexpr (sizeof(TIn) == 4) {
#pragma unroll
      for (int q = 0; q < E / 4; ++q) {
        const float4 f = *reinterpret_cast<const float4 *>(row + k0 + 4 * q);
        v[4 * q + 0] = f.x; v[4 * q + 1] = f.y; v[4 * q + 2] = f.z; v[4 * q + 3] = f.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < E / 2; ++q) {
        const double2 d = *reinterpret_cast<const double2 *>(row + k0 + 2 * q);
        v[2 * q + 0] = d.x; v[2 * q + 1] = d.y;
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = (k0 + e < l) ? row[k0 + e] : (TIn)0;
  }
}

// Store one unit of E transformed samples (FP64 values) into row `zr`.
template <int MODE, int E>
__device__ __forceinline__ void store_unit(unsigned char *zr, int64_t u, const double (&z)[E]) {
  if constexpr (MODE == PCC_FP64) {
    *reinterpret_cast<double2 *>(zr + u * 16) = make_double2(z[0], z[1]);
  } else if constexpr (MODE == PCC_FP32) {
    float4 o = make_float4((float)z[0], (float)z[1], (float)z[2], (float)z[3]);
    *reinterpret_cast<float4 *>(zr + u * 16) = o;
  } else if constexpr (MODE == PCC_BF16) {
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      w[q] = (uint32_t)f32_to_bf16_bits((float)z[2 * q]) |
             ((uint32_t)f32_to_bf16_bits((float)z[2 * q + 1]) << 16);
    *reinterpret_cast<uint4 *>(zr + u * 16) = make_uint4(w[0], w[1], w[2], w[3]);
  } else if constexpr (MODE == PCC_FP16) {
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const _Float16 a = (_Float16)(float)z[2 * q];
      const _Float16 b = (_Float16)(float)z[2 * q + 1];
      w[q] = (uint32_t)__builtin_bit_cast(uint16_t, a) |
             ((uint32_t)__builtin_bit_cast(uint16_t, b) << 16);
    }
    *reinterpret_cast<uint4 *>(zr + u * 16) = make_uint4(w[0], w[1], w[2], w[3]);
  } else {  // split: hi = bf16(z), lo = bf16(z - hi), hi and lo halves of a chunk
    // Each value is rounded to FP32 first, then to BF16 (round to nearest
    // even, two values per v_cvt_pk_bf16_f32).  The empty asm keeps the FP32
    // value: the compiler would otherwise fuse the two roundings into one.
    uint32_t wh[4], wl[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      f32x2_t zf = {(float)z[2 * q], (float)z[2 * q + 1]};
      asm volatile("" : "+v"(zf));
      const bf16x2_t h = __builtin_convertvector(zf, bf16x2_t);
      const uint32_t hw = __builtin_bit_cast(uint32_t, h);
      f32x2_t rf = {(float)(z[2 * q] - (double)__builtin_bit_cast(float, hw << 16)),
                    (float)(z[2 * q + 1] - (double)__builtin_bit_cast(float, hw & 0xffff0000u))};
      asm volatile("" : "+v"(rf));
      wh[q] = hw;
      wl[q] = __builtin_bit_cast(uint32_t, __builtin_convertvector(rf, bf16x2_t));
    }
    const int64_t c = u >> 2, part = u & 3;
    *reinterpret_cast<uint4 *>(zr + c * 128 + part * 16) = make_uint4(wh[0], wh[1], wh[2], wh[3]);
    *reinterpret_cast<uint4 *>(zr + c * 128 + 64 + part * 16) =
        make_uint4(wl[0], wl[1], wl[2], wl[3]);
  }
}

// Unit u of a row, from the group's LDS staging area when it holds it (slot
// < spill_units), else from memory.
template <typename TIn, int E, bool VEC>
__device__ __forceinline__ void reload_unit(const TIn *row, int l, int u, int slot,
                                            const TIn *spill, int spill_units, TIn (&v)[E]) {
  if (slot < spill_units) {
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = spill[slot * E + e];
  } else {
    load_unit<TIn, E, VEC>(row, l, u * E, v);
  }
}

// Transform row `row` (< n) of x into row zr of Z.  Called by the G lanes
// of a group (G = 64: a whole wave).  Lane j owns units j, j + G, j + 2G, ...
// of the padded row; the first kCache of them stay in registers (in the
// input type) for all three passes.  The rest (rows longer than the
// registers hold) are staged in the group's own LDS region `spill` during
// the first pass, up to spill_units units, and read back from there by the
// later passes; units beyond that are read from memory again.  Each lane
// reads back only the units it wrote, so no barrier is needed.  Sample indices
// are 32-bit (l <= 2^21).  A cached unit the row does not have (at or past
// l_pad) reads as zeros: adding +0.0 leaves the FP64 sums unchanged, and the
// third pass stores only the units the row has.
// VEC: the row starts 16-byte aligned, so a unit of E samples is read with
// aligned 16-byte loads (the caller checks the pointer and the pitch);
// otherwise whole units are read at the element type's alignment.
template <typename TIn, int MODE, int kCache, bool VEC>
__device__ __forceinline__ void normalize_row(const TIn *__restrict__ xr, int64_t l64,
                                              int64_t l_pad, unsigned char *__restrict__ zr,
                                              double *stats_row, int32_t *n_degenerate,
                                              double out_scale, int G = 64,
                                              TIn *__restrict__ spill = nullptr,
                                              int spill_units = 0) {
  constexpr int E = UnitOf<MODE>::E;
  const int l = (int)l64;
  const int units = (int)(l_pad / E);
  const int lane = threadIdx.x & (G - 1);
  // cached units the row has at all: the same for every lane of the wave
  // (all its rows have length l), so the bound is a scalar branch
  const int nc = (units + G - 1) / G;
  TIn cache[kCache][E];  // the row stays in registers in its input type
  // pass 1: sum.  All loads of a group of units are issued before any of
  // them is used, so their latencies overlap (summed afterwards in the same
  // order).
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < kCache; ++c)
    if (c < nc) load_unit<TIn, E, VEC>(xr, l, (lane + G * c) * E, cache[c]);
#pragma unroll
  for (int c = 0; c < kCache; ++c) {
    if (c < nc) {
#pragma unroll
      for (int e = 0; e < E; ++e) s += (double)cache[c][e];
    }
  }
  constexpr int kTailGroup = 2;  // tail units loaded together
  for (int u0 = lane + G * kCache; u0 < units; u0 += kTailGroup * G) {
    TIn v[kTailGroup][E];
#pragma unroll
    for (int j = 0; j < kTailGroup; ++j)
      if (u0 + j * G < units) load_unit<TIn, E, VEC>(xr, l, (u0 + j * G) * E, v[j]);
#pragma unroll
    for (int j = 0; j < kTailGroup; ++j) {
      const int u = u0 + j * G;
      if (u < units) {
        const int slot = u - G * kCache;
        if (slot < spill_units) {
#pragma unroll
          for (int e = 0; e < E; ++e) spill[slot * E + e] = v[j][e];
        }
#pragma unroll
        for (int e = 0; e < E; ++e) s += (double)v[j][e];
      }
    }
  }
  const double mean = group_sum(s, G) / (double)l;
  // The cache is re-converted in each pass rather than kept in FP64 (which
  // would double its registers): the empty asm hides that the values did not
  // change.
#pragma unroll
  for (int c = 0; c < kCache; ++c)
#pragma unroll
    for (int e = 0; e < E; ++e) asm volatile("" : "+v"(cache[c][e]));
  // pass 2: sum of squared deviations (padding samples excluded)
  double q = 0.0;
#pragma unroll
  for (int c = 0; c < kCache; ++c) {
    if (c < nc) {
      const int k0 = (lane + G * c) * E;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const double d = (double)cache[c][e] - mean;
        q += (k0 + e < l) ? d * d : 0.0;
      }
    }
  }
  for (int u = lane + G * kCache; u < units; u += G) {
    TIn v[E];
    reload_unit<TIn, E, VEC>(xr, l, u, u - G * kCache, spill, spill_units, v);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const double d = (double)v[e] - mean;
      q += (u * E + e < l) ? d * d : 0.0;
    }
  }
  const double m2 = group_sum(q, G);
  const bool degenerate = !(m2 > 0.0) || !(m2 < INFINITY);
  if (lane == 0) {
    if (stats_row) {
      stats_row[0] = mean;
      stats_row[1] = m2;
    }
    if (degenerate && n_degenerate) atomicAdd(n_degenerate, 1);
  }
  const double inv = degenerate ? (double)NAN : out_scale / sqrt(m2);
#pragma unroll
  for (int c = 0; c < kCache; ++c)
#pragma unroll
    for (int e = 0; e < E; ++e) asm volatile("" : "+v"(cache[c][e]));
  // pass 3: transformed samples, zero padding
#pragma unroll
  for (int c = 0; c < kCache; ++c) {
    if (c < nc) {
      const int u = lane + G * c;
      double o[E];
#pragma unroll
      for (int e = 0; e < E; ++e)
        o[e] = (u * E + e < l) ? ((double)cache[c][e] - mean) * inv : 0.0;
      if (u < units) store_unit<MODE, E>(zr, u, o);
    }
  }
  for (int u = lane + G * kCache; u < units; u += G) {
    TIn v[E];
    double o[E];
    reload_unit<TIn, E, VEC>(xr, l, u, u - G * kCache, spill, spill_units, v);
#pragma unroll
    for (int e = 0; e < E; ++e) o[e] = (u * E + e < l) ? ((double)v[e] - mean) * inv : 0.0;
    store_unit<MODE, E>(zr, u, o);
  }
}

// NG rows of one matrix whose padded length fits the registers of their G
// lanes (l_pad / E <= G * kCache), transformed exactly as normalize_row
// transforms each of them (every sum in the same order), with the loads of
// all NG rows issued before any row is summed, so NG rows are in flight at
// once.  No statistics and no degenerate count (the batch keeps neither).
template <typename TIn, int MODE, int kCache, bool VEC, int NG>
__device__ __forceinline__ void normalize_rows_cached(const TIn *const (&xr)[NG], int64_t l64,
                                                      int64_t l_pad,
                                                      unsigned char *const (&zr)[NG],
                                                      double out_scale, int G) {
  constexpr int E = UnitOf<MODE>::E;
  const int l = (int)l64;
  const int units = (int)(l_pad / E);
  const int lane = threadIdx.x & (G - 1);
  const int nc = (units + G - 1) / G;
  TIn cache[NG][kCache][E];
#pragma unroll
  for (int r = 0; r < NG; ++r)
#pragma unroll
    for (int c = 0; c < kCache; ++c)
      if (c < nc) load_unit<TIn, E, VEC>(xr[r], l, (lane + G * c) * E, cache[r][c]);
  double mean[NG], inv[NG];
#pragma unroll
  for (int r = 0; r < NG; ++r) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kCache; ++c) {
      if (c < nc) {
#pragma unroll
        for (int e = 0; e < E; ++e) s += (double)cache[r][c][e];
      }
    }
    mean[r] = group_sum(s, G) / (double)l;
  }
#pragma unroll
  for (int r = 0; r < NG; ++r)
#pragma unroll
    for (int c = 0; c < kCache; ++c)
#pragma unroll
      for (int e = 0; e < E; ++e) asm volatile("" : "+v"(cache[r][c][e]));
#pragma unroll
  for (int r = 0; r < NG; ++r) {
    double q = 0.0;
#pragma unroll
    for (int c = 0; c < kCache; ++c) {
      if (c < nc) {
        const int k0 = (lane + G * c) * E;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const double d = (double)cache[r][c][e] - mean[r];
          q += (k0 + e < l) ? d * d : 0.0;
        }
      }
    }
    const double m2 = group_sum(q, G);
    const bool degenerate = !(m2 > 0.0) || !(m2 < INFINITY);
    inv[r] = degenerate ? (double)NAN : out_scale / sqrt(m2);
  }
#pragma unroll
  for (int r = 0; r < NG; ++r)
#pragma unroll
    for (int c = 0; c < kCache; ++c)
#pragma unroll
      for (int e = 0; e < E; ++e) asm volatile("" : "+v"(cache[r][c][e]));
#pragma unroll
  for (int r = 0; r < NG; ++r) {
#pragma unroll
    for (int c = 0; c < kCache; ++c) {
      if (c < nc) {
        const int u = lane + G * c;
        double o[E];
#pragma unroll
        for (int e = 0; e < E; ++e)
          o[e] = (u * E + e < l) ? ((double)cache[r][c][e] - mean[r]) * inv[r] : 0.0;
        if (u < units) store_unit<MODE, E>(zr[r], u, o);
      }
    }
  }
}

// Zero one padding row of Z (rows n .. n_pad-1).
__device__ __forceinline__ void zero_row(unsigned char *__restrict__ zr, int64_t row_bytes,
                                         int G = 64) {
  const int lane = threadIdx.x & (G - 1);
  for (int64_t u = lane; u < row_bytes / 16; u += G)
    *reinterpret_cast<uint4 *>(zr + u * 16) = make_uint4(0u, 0u, 0u, 0u);
}

}  // namespace pcc
