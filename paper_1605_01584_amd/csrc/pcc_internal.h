// Internal definitions shared by the HIP sources of libpcc (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pcc.h"

#define PCC_HD __host__ __device__ __forceinline__

namespace pcc {

// ---------------------------------------------------------------------------
// Job maps (Sec. III-B/C).  F_m(y) = y(2m - y + 1)/2 counts the cells of the
// inclusive upper triangle above row y, Eq. (10)/(17).  All integer work is
// int64: y(2m-y+1) passes INT32_MAX already for m around 46341.

PCC_HD int64_t tri_F(int64_t m, int64_t y) { return (y * (2 * m - y + 1)) >> 1; }

struct Cell {
  int64_t y, x;
};

// Inverse of J = F_m(y) + x - y, Eq. (14)-(15)/(18)-(19).  The ceiling of
// Eq. (14) is evaluated in FP64; the guess is then corrected in int64 until
// F_m(y) <= J < F_m(y+1) holds, so the result is exact for every m < 2^31
// whatever the rounding of sqrt (a 1-ulp-low sqrt would otherwise move the
// last id of every row to the next row).
PCC_HD Cell tri_cell(int64_t m, int64_t J) {
  const double dm = (double)m;
  double t = dm * dm + dm + 0.25 - 2.0 * ((double)J + 1.0);
  t = t > 0.0 ? t : 0.0;
  int64_t g = (int64_t)ceil(dm - 0.5 - sqrt(t));
  g = g < 0 ? 0 : (g > m - 1 ? m - 1 : g);
  while (g + 1 < m && tri_F(m, g + 1) <= J) ++g;
  while (g > 0 && tri_F(m, g) > J) --g;
  return Cell{g, J + g - tri_F(m, g)};
}

// Strict upper triangle over n profiles: cells y < x < n are the inclusive
// triangle over n - 1 with x shifted by one (the diagonal-free adaptation the
// framework allows).  J' = F_{n-1}(y) + (x - 1) - y.
PCC_HD int64_t packed_index(int64_t n, int64_t y, int64_t x) {
  return tri_F(n - 1, y) + (x - 1) - y;
}
PCC_HD Cell packed_cell(int64_t n, int64_t Jp) {
  const Cell c = tri_cell(n - 1, Jp);
  return Cell{c.y, c.x + 1};
}

// Column of offset o in a small triangle walked column by column (column c
// holds c + 1 cells): the largest c with c(c+1)/2 <= o.
PCC_HD int64_t small_tri_col(int64_t o) {
  int64_t c = (int64_t)((sqrt(8.0 * (double)o + 1.0) - 1.0) * 0.5);
  if (c < 0) c = 0;
  while ((c + 1) * (c + 2) / 2 <= o) ++c;
  while (c > 0 && c * (c + 1) / 2 > o) --c;
  return c;
}

// Banded tile order: the m x m tile triangle is cut into bands of H tile
// rows; band b covers rows [bH, bH + h), h = min(H, m - bH), and is walked
// column by column, top to bottom inside a column.  The jobs before band b
// are exactly the cells of the rows above it, F_m(bH), so the band of id J is
// the row-major row of J (Eq. (18)) divided by H.  A bijection from
// [0, m(m+1)/2) onto the inclusive tile triangle.
PCC_HD Cell band_cell(int64_t m, int64_t H, int64_t J) {
  const Cell rm = tri_cell(m, J);
  const int64_t r0 = (rm.y / H) * H;
  const int64_t h = (m - r0) < H ? (m - r0) : H;
  const int64_t o = J - tri_F(m, r0);
  const int64_t T = h * (h + 1) / 2;
  if (o < T) {
    const int64_t c = small_tri_col(o);
    return Cell{r0 + (o - c * (c + 1) / 2), r0 + c};
  }
  const int64_t q = o - T;
  return Cell{r0 + q % h, r0 + h + q / h};
}

PCC_HD Cell tile_of_job(int64_t m, int order, int64_t H, int64_t J) {
  return (order == 1 && H > 1) ? band_cell(m, H, J) : tri_cell(m, J);
}

// Non-symmetric all-pairs over an mr x mc tile rectangle, Eq. (7)-(8): every
// cell is a job, J = y mc + x, x = J % mc, y = J / mc.  Banded order: bands
// of H tile rows, band b = [bH, bH + h) with h = min(H, mr - bH), starts at
// id bH mc and is walked column by column, top to bottom.
PCC_HD Cell rect_cell(int64_t mr, int64_t mc, int order, int64_t H, int64_t J) {
  if (order != 1 || H <= 1) return Cell{J / mc, J % mc};
  const int64_t r0 = (J / mc) / H * H;
  const int64_t h = (mr - r0) < H ? (mr - r0) : H;
  const int64_t o = J - r0 * mc;
  return Cell{r0 + o % h, o / h};
}

// ---------------------------------------------------------------------------
// Number formats.

// float -> bf16 bits, round to nearest even; NaN stays a quiet NaN.
PCC_HD uint16_t f32_to_bf16_bits(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
PCC_HD float bf16_bits_to_f32(uint16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// The last HIP error a library call met on this thread (for
// pcc_last_hip_error); returns e so call sites can wrap a HIP call.
hipError_t note_hip(hipError_t e);

// Layout constants.
constexpr int kChunkBytes = 128;
constexpr int kRowPadMultiple = 256;

inline int kchunk_of(int mode) {
  if (mode == PCC_FP64) return 16;
  return (mode == PCC_FP32 || mode == PCC_SPLIT_BF16X3) ? 32 : 64;
}

// Arithmetic of the split-BF16 layout on short rows.  Two BF16 terms carry z
// to about 2^-16 relative and the lo.lo product is dropped, so a product
// z_i[k] z_j[k] is off by up to 3 * 2^-16 |z_i[k] z_j[k]|; over many samples
// these errors have random signs and average out, over a handful they do not
// (|dr| above 1e-5 at l <= 8 on Gaussian rows).  Rows of at most two chunks
// (l_pad <= 64) therefore hold z in FP32 and are contracted on FP32 MFMA:
// the FP32 and split layouts both pack 32 samples into a 128-byte chunk, so
// the row size is the same and only the arithmetic changes.  At such l a
// tile does 2 l flops per pair against 4 bytes of r stored, so the FP32
// tiles cost about what the split ones do.
constexpr int64_t kSplitFp32MaxLPad = 64;

inline int arith_mode(int mode, int64_t l_pad) {
  return (mode == PCC_SPLIT_BF16X3 && l_pad <= kSplitFp32MaxLPad) ? (int)PCC_FP32 : mode;
}
inline int arith_mode(const pcc_zdesc &zd) { return arith_mode(zd.mode, zd.l_pad); }

}  // namespace pcc
