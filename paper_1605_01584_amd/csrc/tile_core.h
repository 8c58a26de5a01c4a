// Device core of the all-pairs tile computation, shared by the uniform
// kernels (tiles.hip) and the uneven-batch kernel (batched.hip).
//
// One call computes one TILE x TILE tile (yt, xt) of Z Z^T (Eq. (5)) with a
// 512-thread workgroup: 8 waves, two per SIMD, in a 4 x 2 grid, each wave a
// (TILE/4) x (TILE/2) block of 32 x 32 MFMA blocks whose FP32 accumulators
// stay in registers for the whole K loop.  Two waves per SIMD let one wave's
// LDS reads and barrier waits overlap the other's MFMAs.
//
// K loop: one 128-byte chunk of every row per stage (32 FP32 samples, 32
// split hi+lo samples, or 64 BF16/FP16 samples).  Stages are copied global ->
// LDS directly by buffer_load ... lds (no VGPR staging), double buffered.
// In LDS a row is 8 units of 16 bytes, unit u of row r at slot
// u ^ ((r & 7) ^ ((r >> 3) & 1)): the ds_read_b128 of 16 consecutive rows hit
// 16 distinct bank groups, so fragment reads are conflict free.
//
// Each stage is split in two halves of fragments; the second half is read
// while the first half's MFMAs run, and the next stage's first half is read
// (after the stage barrier) while the second half's MFMAs run:
//   read h1(c) | MFMA h0(c) | wait DMA(c+1), barrier, read h0(c+1),
//   DMA(c+2) into the buffer stage c used | MFMA h1(c)
//
// Sample assignment inside a chunk (any assignment works as long as both
// operands use the same one, since the contraction sums over all samples):
//   FP32   fragment (h, s) = unit 2(2h+s)+g, 4 samples feeding 4 consecutive
//          32x32x2 MFMAs (K = 2: one sample per lane half g);
//   BF16/FP16  fragment (h, s) = unit 2(2h+s)+g (8 samples), one 32x32x16
//          MFMA each;
//   SPLIT  half h: hi unit 2h+g and lo unit 4+2h+g of the same 8 samples;
//          three 32x32x16 MFMAs lo.hi + hi.lo + hi.hi into one FP32
//          accumulator (the lo.lo term, about 2^-16 of r, is dropped).
//   FP64   (do_tile_f64, 128-wide tiles, 16 x 16 blocks) lane (j, g4),
//          j = lane % 16, g4 = lane / 16, reads units g4 and g4 + 4 of row j
//          (4 doubles); k-step (h, e) takes double e of unit g4 + 4h, i.e.
//          sample 8h + 2g4 + e, as its k index g4.
//
// The same core serves the symmetric job matrix (column operand = row
// operand, strict upper triangle kept, Eq. (5)) and the non-symmetric one of
// two variable sets (Eq. (7)-(8), every cell kept); the epilogue kind EPI
// selects the mask and where r goes.
#pragma once

#include "pcc_internal.h"

namespace pcc {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

// Epilogue kinds:
//   EPI_PACKED      symmetric, packed strict upper triangle, FP32 r
//   EPI_EDGES       symmetric, |r| >= thr appended to an edge list
//   EPI_RECT        non-symmetric, r[y * ldr + x], FP32
//   EPI_RECT_EDGES  non-symmetric edge list
//   EPI_PACKED_F64  symmetric, packed, FP64 r (FP64 mode only)
//   EPI_PERM        symmetric job matrix of Z against a column-permuted copy
//                   of Z: cnt[J'] += 1 where |r| >= |robs[J']| (permutation
//                   test; the job owning a tile is the only writer of its
//                   counts in a launch, so an atomic add with no return
//                   value serves as the increment and saves the load of a
//                   read-modify-write)
enum { EPI_PACKED = 0, EPI_EDGES = 1, EPI_RECT = 2, EPI_RECT_EDGES = 3, EPI_PACKED_F64 = 4,
       EPI_PERM = 5 };

constexpr int kTileThreads = 512;  // 8 waves
// num_records of the panel buffer descriptors: 2^32 - 1 bytes.  A panel is at
// most 256 rows of at most 2^21 samples x 4 bytes (or 128 rows x 8 bytes),
// 2 GiB, so every load of a tile lies inside it and its 32-bit offset.
constexpr int kPanelRange = (int)0xffffffffu;
constexpr int kWavesR = 4, kWavesC = 2;

// Z operands of one tile computation.
struct ZView {
  const unsigned char *z;   // row operand (profiles y)
  int64_t row_bytes;        // both operands
  int64_t n;                // profiles of the row operand
  int32_t nchunks;
  float scale;              // accumulator -> r (FP16 layout: 1/l)
  const unsigned char *zc;  // column operand (profiles x); == z when symmetric
  int64_t nc;               // profiles of the column operand
};

// Output of one tile computation.
struct EpiArgs {
  float *r;                 // packed triangle, or nx x ldr rectangle
  double *r64;              // packed triangle in FP64
  int64_t roff;             // packed: index of r[0] in the whole triangle (a slice)
  int64_t ldr;              // rectangle row pitch
  float thr;                // edges: |r| >= thr
  int32_t *ij;
  float *rv;
  int64_t cap;
  unsigned long long *count;
  const float *robs;        // permutation test: observed r, packed
  int32_t *cnt;             // permutation test: counts, packed
};

template <int TILE> struct TileShape {
  static constexpr int WTR = TILE / kWavesR;  // wave tile rows
  static constexpr int WTC = TILE / kWavesC;  // wave tile columns
  static constexpr int NBR = WTR / 32;        // MFMA blocks per wave, rows
  static constexpr int NBC = WTC / 32;        // MFMA blocks per wave, columns
  static constexpr int OPU = TILE * 8;        // LDS units per operand per stage
  static constexpr int IPW = OPU / 64 / (kWavesR * kWavesC);  // DMA per wave per operand
  static constexpr int LDS_UNITS = 2 * 2 * OPU;               // [buffer][A | B]
};

__device__ __forceinline__ float clamp_unit(float r) {
  // median of (r, -1, 1), then NaN restored (the median of a NaN and two
  // numbers need not be NaN): three instructions, NaN passes through
  const float c = __builtin_amdgcn_fmed3f(r, -1.0f, 1.0f);
  return r == r ? c : r;
}

__device__ __forceinline__ double clamp_unit(double r) {
  return r > 1.0 ? 1.0 : (r < -1.0 ? -1.0 : r);
}

// Accumulator -> r: the FP16 layout holds z * sqrt(l), so its products are
// scaled by 1/l; every other layout's accumulator is r itself.
template <int MODE>
__device__ __forceinline__ float acc_to_r(float a, float scale) {
  if constexpr (MODE == PCC_FP16)
    return clamp_unit(a * scale);
  else
    return clamp_unit(a);
}

// Mask, output row base and store of one r value for epilogue kind EPI.
template <int EPI> struct Epi {
  static constexpr bool kRect = EPI == EPI_RECT || EPI == EPI_RECT_EDGES;
  static constexpr bool kEdges = EPI == EPI_EDGES || EPI == EPI_RECT_EDGES;
  // Packed: row y of the strict upper triangle starts at F_{n-1}(y) - y - 1 + x.
  // Profile indices are below 2^31, so the products are 32 x 32 -> 64 bits
  // (one multiply-add) and the masks compare 32-bit values.
  static __device__ __forceinline__ int64_t rowbase(const ZView &zv, const EpiArgs &ea,
                                                    uint32_t y) {
    if constexpr (kRect) {
      return (int64_t)((uint64_t)y * (uint64_t)ea.ldr);
    } else {
      // F_{n-1}(y) = y (2(n-1) - y + 1) / 2, both factors below 2^32
      const uint32_t f = 2u * (uint32_t)zv.n - 1u - y;
      return (int64_t)(((uint64_t)y * (uint64_t)f) >> 1) - 1 - (int64_t)y - ea.roff;
    }
  }
  // rowbase(y + 1) - rowbase(y): the row pitch, or the length n - 1 - y of
  // packed row y less the one-column shift of the next row
  static __device__ __forceinline__ int64_t row_step(const ZView &zv, const EpiArgs &ea,
                                                     uint32_t y) {
    if constexpr (kRect)
      return ea.ldr;
    else
      return (int64_t)(int32_t)((uint32_t)zv.n - 2u - y);
  }
  static __device__ __forceinline__ bool keep(const ZView &zv, uint32_t y, uint32_t x) {
    if constexpr (kRect)
      return y < (uint32_t)zv.n && x < (uint32_t)zv.nc;
    else
      return y < x && x < (uint32_t)zv.n;
  }
  // Every cell of the TILE x TILE tile at rows ya.., columns xa.. is kept.
  static __device__ __forceinline__ bool full(const ZView &zv, int64_t ya, int64_t xa, int TILE) {
    if constexpr (kRect)
      return ya + TILE <= zv.n && xa + TILE <= zv.nc;
    else
      return ya + TILE <= xa && xa + TILE <= zv.n;
  }
  // rv is already clamped (NaN kept: it fails |rv| >= thr).  r is stored
  // with ordinary (L2 write-back) stores: nontemporal ones measured about 1%
  // slower on the packed triangle and the uneven batch, whose short jobs
  // wait for their stores at the next job's first copy.
  template <typename T>
  static __device__ __forceinline__ void emit(const EpiArgs &ea, int64_t rb, int64_t y, int64_t x,
                                              T rv) {
    if constexpr (EPI == EPI_PACKED_F64) {
      ea.r64[rb + x] = (double)rv;
    } else if constexpr (kEdges) {
      if ((rv < (T)0 ? -rv : rv) >= (T)ea.thr) {
        const unsigned long long s = atomicAdd(ea.count, 1ull);
        if ((int64_t)s < ea.cap) {
          ea.ij[2 * s] = (int32_t)y;
          ea.ij[2 * s + 1] = (int32_t)x;
          ea.rv[s] = (float)rv;
        }
      }
    } else {
      ea.r[rb + x] = (float)rv;
    }
  }
};

__device__ __forceinline__ int64_t xcd_slot(int64_t b, int64_t G) {
  // Workgroups are dispatched to the 8 XCDs round robin (b % 8); give the
  // workgroups of one XCD consecutive job ids so they share L2 lines.
  return (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
}

__device__ __forceinline__ int lds_swz(int r) { return (r & 7) ^ ((r >> 3) & 1); }

// Swizzle of the FP64 tile's LDS rows, whose fragment reads take 16 rows by
// four 16-byte units per instruction.  Measured: the swizzle above, which
// also flips the unit of rows 8-15, costs these reads four bank-conflict
// cycles each; the row index mod 8 alone (or (r / 2) mod 8) none.
__device__ __forceinline__ int lds_swz64(int r) { return r & 7; }

// LDS unit of fragment s of half h for lane half g.
template <int MODE> __device__ __forceinline__ int frag_unit(int h, int s, int g) {
  if constexpr (MODE == PCC_SPLIT_BF16X3)
    return s * 4 + 2 * h + g;  // s = 0: hi, s = 1: lo
  else
    return 2 * (2 * h + s) + g;
}

template <int MODE, int NB>
__device__ __forceinline__ void read_half(const u32x4 *__restrict__ base, int i, int g, int h,
                                          u32x4 (&f)[2][NB]) {
  const int sw = lds_swz(i);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int u = frag_unit<MODE>(h, s, g) ^ sw;
#pragma unroll
    for (int q = 0; q < NB; ++q) f[s][q] = base[(q * 32 + i) * 8 + u];
  }
}

template <int MODE, int NBR, int NBC>
__device__ __forceinline__ void mfma_half(const u32x4 (&fa)[2][NBR], const u32x4 (&fb)[2][NBC],
                                          f32x16 (&acc)[NBR][NBC]) {
  if constexpr (MODE == PCC_FP32) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      // cast whole vectors, then index the floats
      f32x4 a[NBR], b[NBC];
#pragma unroll
      for (int q = 0; q < NBR; ++q) a[q] = __builtin_bit_cast(f32x4, fa[s][q]);
#pragma unroll
      for (int q = 0; q < NBC; ++q) b[q] = __builtin_bit_cast(f32x4, fb[s][q]);
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int p = 0; p < NBR; ++p)
#pragma unroll
          for (int q = 0; q < NBC; ++q)
            acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p][e], b[q][e], acc[p][q], 0, 0, 0);
    }
  } else if constexpr (MODE == PCC_SPLIT_BF16X3) {
#pragma unroll
    for (int p = 0; p < NBR; ++p)
#pragma unroll
      for (int q = 0; q < NBC; ++q) {
        const bf16x8 ah = __builtin_bit_cast(bf16x8, fa[0][p]);
        const bf16x8 al = __builtin_bit_cast(bf16x8, fa[1][p]);
        const bf16x8 bh = __builtin_bit_cast(bf16x8, fb[0][q]);
        const bf16x8 bl = __builtin_bit_cast(bf16x8, fb[1][q]);
        acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[p][q], 0, 0, 0);
        acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[p][q], 0, 0, 0);
        acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[p][q], 0, 0, 0);
      }
  } else {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int p = 0; p < NBR; ++p)
#pragma unroll
        for (int q = 0; q < NBC; ++q) {
          if constexpr (MODE == PCC_BF16)
            acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, fa[s][p]), __builtin_bit_cast(bf16x8, fb[s][q]), acc[p][q], 0, 0, 0);
          else
            acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                __builtin_bit_cast(f16x8, fa[s][p]), __builtin_bit_cast(f16x8, fb[s][q]), acc[p][q], 0, 0, 0);
        }
  }
}

// Copy stage (byte offset cb within every row) of both panels into LDS at dst.
// DMA instruction inst fills LDS units [64 inst, 64 inst + 64) of an operand:
// rows 8 inst .. 8 inst + 7, lane l taking row 8 inst + l/8 and the unit that
// belongs in slot l % 8.  Wave w issues instructions w * IPW .. + IPW - 1.
template <int TILE>
__device__ __forceinline__ void dma_stage(__amdgpu_buffer_rsrc_t ra, __amdgpu_buffer_rsrc_t rbs,
                                          uint32_t lane_row_off, uint32_t uoff_even,
                                          uint32_t uoff_odd, uint32_t row8_bytes, uint32_t cb,
                                          u32x4 *dst, int w) {
  using S = TileShape<TILE>;
#pragma unroll
  for (int k = 0; k < S::IPW; ++k) {
    const int inst = w * S::IPW + k;
    const uint32_t voff = lane_row_off + ((inst & 1) ? uoff_odd : uoff_even);
    const uint32_t soff = (uint32_t)k * row8_bytes + cb;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_void *)(dst + inst * 64), 16, voff, soff, 0, 0);
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rbs, (lds_void *)(dst + S::OPU + inst * 64), 16, voff,
                                             soff, 0, 0);
  }
}

// Compute tile (yt, xt) and write its strict-upper-triangle pairs.
// The last stage copy of a call may still be in flight when it returns (it
// fills LDS units that the same wave fills first at the next call with the
// same TILE); a workgroup that switches TILE between calls waits for its
// outstanding loads (vmcnt(0)) before the next call.
// Requires: all 512 threads of the workgroup call it together; smem holds
// TileShape<TILE>::LDS_UNITS units; rows yt*TILE .. +TILE and xt*TILE .. +TILE
// exist in Z (n_pad is a multiple of 256); TILE * row_bytes <= 2^32.
template <int MODE, int TILE, int EPI>
__device__ __forceinline__ void do_tile(const ZView &zv, const EpiArgs &ea, int64_t yt, int64_t xt,
                                        u32x4 *__restrict__ smem) {
  using S = TileShape<TILE>;
  constexpr int WTR = S::WTR, WTC = S::WTC, NBR = S::NBR, NBC = S::NBC, OPU = S::OPU;
  constexpr int IPW = S::IPW;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = w / kWavesC, wc = w % kWavesC;
  const int i = lane & 31, g = lane >> 5;
  const int64_t rb = zv.row_bytes;
  const unsigned char *za = zv.z + yt * TILE * rb;
  const unsigned char *zb = zv.zc + xt * TILE * rb;
  const __amdgpu_buffer_rsrc_t rsa =
      __builtin_amdgcn_make_buffer_rsrc((void *)za, (short)0, kPanelRange, 0x00020000);
  const __amdgpu_buffer_rsrc_t rsb =
      __builtin_amdgcn_make_buffer_rsrc((void *)zb, (short)0, kPanelRange, 0x00020000);
  const int ro = lane >> 3;
  const uint32_t lane_row_off = (uint32_t)((8 * IPW * w + ro) * rb);
  const uint32_t uoff_even = (uint32_t)(((lane & 7) ^ lds_swz(ro)) * 16);
  const uint32_t uoff_odd = (uint32_t)(((lane & 7) ^ lds_swz(ro + 8)) * 16);
  const uint32_t row8 = (uint32_t)(8 * rb);
  const int nch = zv.nchunks;
  const int aoff = (wr * WTR) * 8, boff = OPU + (wc * WTC) * 8;

  f32x16 acc[NBR][NBC];
#pragma unroll
  for (int p = 0; p < NBR; ++p)
#pragma unroll
    for (int q = 0; q < NBC; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[p][q][v] = 0.0f;

  u32x4 f0a[2][NBR], f0b[2][NBC], f1a[2][NBR], f1b[2][NBC];
  __syncthreads();  // every wave is done reading the previous tile's stages
  dma_stage<TILE>(rsa, rsb, lane_row_off, uoff_even, uoff_odd, row8, 0u, smem, w);
  if (nch > 1) {
    dma_stage<TILE>(rsa, rsb, lane_row_off, uoff_even, uoff_odd, row8, 128u, smem + 2 * OPU, w);
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * IPW) : "memory");  // stage 0 landed
  } else {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  __syncthreads();
  read_half<MODE, NBR>(smem + aoff, i, g, 0, f0a);
  read_half<MODE, NBC>(smem + boff, i, g, 0, f0b);
  // Every stage but the last.  The last one is peeled off below, so the
  // loop body has a single path: were the barrier conditional, the compiler
  // would merge a path with the second-half reads still in flight into the
  // one without, and make the second-half MFMAs wait for the next stage's
  // first-half reads issued right after the barrier.
  for (int c = 0; c + 1 < nch; ++c) {
    const u32x4 *cur = smem + (c & 1) * 2 * OPU;
    read_half<MODE, NBR>(cur + aoff, i, g, 1, f1a);
    read_half<MODE, NBC>(cur + boff, i, g, 1, f1b);
    mfma_half<MODE, NBR, NBC>(f0a, f0b, acc);
    // own DMA of stage c+1 landed and own reads of stage c returned; the
    // barrier makes both true for every wave
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    __syncthreads();
    const u32x4 *nxt = smem + ((c + 1) & 1) * 2 * OPU;
    read_half<MODE, NBR>(nxt + aoff, i, g, 0, f0a);
    read_half<MODE, NBC>(nxt + boff, i, g, 0, f0b);
    // Stage c + 2 into the buffer stage c used.  Issued unconditionally (the
    // last stage is loaded again when c + 2 == nch, into a buffer nobody
    // reads any more), so the loads sit in the same block as the MFMAs and
    // the scheduler interleaves them.  A wave's DMA always fills the same
    // LDS units and its loads complete in order, so that extra load lands
    // before the next tile's first stage overwrites the buffer.
    {
      const int cn = (c + 2 < nch) ? c + 2 : nch - 1;
      dma_stage<TILE>(rsa, rsb, lane_row_off, uoff_even, uoff_odd, row8, (uint32_t)cn * 128u,
                      smem + (c & 1) * 2 * OPU, w);
    }
    mfma_half<MODE, NBR, NBC>(f1a, f1b, acc);
  }
  {
    const u32x4 *cur = smem + ((nch - 1) & 1) * 2 * OPU;
    read_half<MODE, NBR>(cur + aoff, i, g, 1, f1a);
    read_half<MODE, NBC>(cur + boff, i, g, 1, f1b);
    mfma_half<MODE, NBR, NBC>(f0a, f0b, acc);
    mfma_half<MODE, NBR, NBC>(f1a, f1b, acc);
  }

  // Epilogue.  Lane holds column x0 + 32q + i of block (p, q); accumulator
  // register v holds row 8*(v/4) + 4*g + (v%4) of the block.
  const int64_t y0 = yt * TILE + wr * WTR;
  const int64_t x0 = xt * TILE + wc * WTC;
  // Tiles wholly inside the kept region (all but the diagonal ones and the
  // last column or row) store every value without a per-value mask.
  const bool whole = Epi<EPI>::full(zv, yt * TILE, xt * TILE, TILE);
  if constexpr (EPI == EPI_PERM) {
    // Counting epilogue: the observed r of half a block row (8 rows) is
    // loaded whole before any of its counts is touched, so the loads share
    // one wait (one after each count update would wait for that update to
    // complete as well).  Half rows keep the loaded values within registers.
#pragma unroll
    for (int p = 0; p < NBR; ++p) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        float ro[8][NBC];
#pragma unroll
        for (int vv = 0; vv < 8; ++vv) {
          const int v = 8 * h + vv;
          const uint32_t y = (uint32_t)(y0 + p * 32 + 8 * (v >> 2) + 4 * g + (v & 3));
          const float *rrow = ea.robs + Epi<EPI>::rowbase(zv, ea, y) + x0 + i;
#pragma unroll
          for (int q = 0; q < NBC; ++q) {
            const uint32_t x = (uint32_t)(x0 + q * 32 + i);
            ro[vv][q] = (whole || Epi<EPI>::keep(zv, y, x)) ? rrow[q * 32] : __builtin_nanf("");
          }
        }
#pragma unroll
        for (int vv = 0; vv < 8; ++vv) {
          const int v = 8 * h + vv;
          const uint32_t y = (uint32_t)(y0 + p * 32 + 8 * (v >> 2) + 4 * g + (v & 3));
          int32_t *crow = ea.cnt + Epi<EPI>::rowbase(zv, ea, y) + x0 + i;
#pragma unroll
          for (int q = 0; q < NBC; ++q) {
            // NaN (masked cells, degenerate pairs) never counts
            const float rv = acc_to_r<MODE>(acc[p][q][v], zv.scale);
            if (fabsf(rv) >= fabsf(ro[vv][q]))
              (void)__hip_atomic_fetch_add(crow + q * 32, 1, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
    }
  } else {
#pragma unroll
    for (int p = 0; p < NBR; ++p) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        // rows y4 .. y4 + 3 (registers v = 4j .. 4j + 3): the first row's
        // start computed, the next ones stepped by the row lengths
        const uint32_t y4 = (uint32_t)(y0 + p * 32 + 8 * j + 4 * g);
        int64_t rbase = Epi<EPI>::rowbase(zv, ea, y4);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int v = 4 * j + t;
          const uint32_t y = y4 + t;
          if (t > 0) rbase += Epi<EPI>::row_step(zv, ea, y - 1);
          if (whole) {
#pragma unroll
            for (int q = 0; q < NBC; ++q)
              Epi<EPI>::emit(ea, rbase, y, x0 + q * 32 + i, acc_to_r<MODE>(acc[p][q][v], zv.scale));
          } else {
#pragma unroll
            for (int q = 0; q < NBC; ++q) {
              const uint32_t x = (uint32_t)(x0 + q * 32 + i);
              if (Epi<EPI>::keep(zv, y, x))
                Epi<EPI>::emit(ea, rbase, y, x, acc_to_r<MODE>(acc[p][q][v], zv.scale));
            }
          }
        }
      }
    }
  }
}

// FP64 tile (yt, xt), 128 x 128, same workgroup shape, LDS stages and DMA as
// do_tile, with its own row swizzle (lds_swz64); each wave owns 32 x 64 =
// 2 x 4 blocks of 16 x 16 FP64 accumulators (v_mfma_f64_16x16x4_f64).  One
// FP64 MFMA is long, so whole stages are pipelined: stage c + 1's fragments
// are read (after the stage barrier) before stage c's 32 MFMAs are issued.
template <int EPI>
__device__ __forceinline__ void do_tile_f64(const ZView &zv, const EpiArgs &ea, int64_t yt,
                                            int64_t xt, u32x4 *__restrict__ smem) {
  constexpr int TILE = 128;
  using S = TileShape<TILE>;
  constexpr int WTR = S::WTR, WTC = S::WTC, OPU = S::OPU, IPW = S::IPW;
  constexpr int FR = WTR / 16, FC = WTC / 16;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = w / kWavesC, wc = w % kWavesC;
  const int j = lane & 15, g4 = lane >> 4;
  const int64_t rb = zv.row_bytes;
  const unsigned char *za = zv.z + yt * TILE * rb;
  const unsigned char *zb = zv.zc + xt * TILE * rb;
  const __amdgpu_buffer_rsrc_t rsa =
      __builtin_amdgcn_make_buffer_rsrc((void *)za, (short)0, kPanelRange, 0x00020000);
  const __amdgpu_buffer_rsrc_t rsb =
      __builtin_amdgcn_make_buffer_rsrc((void *)zb, (short)0, kPanelRange, 0x00020000);
  const int ro = lane >> 3;
  const uint32_t lane_row_off = (uint32_t)((8 * IPW * w + ro) * rb);
  const uint32_t uoff_even = (uint32_t)(((lane & 7) ^ lds_swz64(ro)) * 16);
  const uint32_t uoff_odd = (uint32_t)(((lane & 7) ^ lds_swz64(ro + 8)) * 16);
  const uint32_t row8 = (uint32_t)(8 * rb);
  const int nch = zv.nchunks;
  // rows 16p + j of a wave's band sit at row offsets that are multiples of
  // 16 plus j, so their swizzle is lds_swz64(j)
  const int sw = lds_swz64(j);
  const int aoff = (wr * WTR + j) * 8, boff = OPU + (wc * WTC + j) * 8;
  const int u0 = g4 ^ sw, u1 = (g4 + 4) ^ sw;

  f64x4 acc[FR][FC];
#pragma unroll
  for (int p = 0; p < FR; ++p)
#pragma unroll
    for (int q = 0; q < FC; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[p][q][v] = 0.0;

  // Two fragment sets alternate between stages (the loop body runs twice
  // per iteration with the sets' roles swapped), so no fragment is copied.
  u32x4 a0[2][FR], b0[2][FC], a1[2][FR], b1[2][FC];
  __syncthreads();  // every wave is done reading the previous tile's stages
  dma_stage<TILE>(rsa, rsb, lane_row_off, uoff_even, uoff_odd, row8, 0u, smem, w);
  if (nch > 1) {
    dma_stage<TILE>(rsa, rsb, lane_row_off, uoff_even, uoff_odd, row8, 128u, smem + 2 * OPU, w);
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(2 * IPW) : "memory");  // stage 0 landed
  } else {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
  __syncthreads();
  auto read_stage = [&](const u32x4 *buf, u32x4(&fa)[2][FR], u32x4(&fb)[2][FC]) {
#pragma unroll
    for (int p = 0; p < FR; ++p) {
      fa[0][p] = buf[aoff + p * 128 + u0];
      fa[1][p] = buf[aoff + p * 128 + u1];
    }
#pragma unroll
    for (int q = 0; q < FC; ++q) {
      fb[0][q] = buf[boff + q * 128 + u0];
      fb[1][q] = buf[boff + q * 128 + u1];
    }
  };
  auto mfma_stage = [&](const u32x4(&fa)[2][FR], const u32x4(&fb)[2][FC]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      f64x2 a[FR], b[FC];
#pragma unroll
      for (int p = 0; p < FR; ++p) a[p] = __builtin_bit_cast(f64x2, fa[h][p]);
#pragma unroll
      for (int q = 0; q < FC; ++q) b[q] = __builtin_bit_cast(f64x2, fb[h][q]);
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int p = 0; p < FR; ++p)
#pragma unroll
          for (int q = 0; q < FC; ++q)
            acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p][e], b[q][e], acc[p][q], 0, 0, 0);
    }
  };
  // Stage c with a stage after it: after the barrier read stage c + 1 into
  // the other set and copy stage c + 2 (if any) into the buffer stage c used,
  // then stage c's MFMAs.  Every stage in the loop reads its successor (the
  // last one is peeled off), so the waits for those reads stay exact.
  auto stage = [&](int c, const u32x4(&fa)[2][FR], const u32x4(&fb)[2][FC], u32x4(&ga)[2][FR],
                   u32x4(&gb)[2][FC]) {
    // The MFMAs touch registers only, so the scheduler would sink the
    // previous stage's MFMAs below this wait, which then finds the copy of
    // stage c + 1 still in flight with nothing left to cover it: keep them
    // above it.
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    __syncthreads();  // stage c + 1 landed everywhere; stage c's buffer is free
    read_stage(smem + ((c + 1) & 1) * 2 * OPU, ga, gb);
    if (c + 2 < nch)
      dma_stage<TILE>(rsa, rsb, lane_row_off, uoff_even, uoff_odd, row8,
                      (uint32_t)(c + 2) * 128u, smem + (c & 1) * 2 * OPU, w);
    mfma_stage(fa, fb);
  };
  read_stage(smem, a0, b0);
  int c = 0;
  for (; c + 2 < nch; c += 2) {
    stage(c, a0, b0, a1, b1);
    stage(c + 1, a1, b1, a0, b0);
  }
  if (c + 1 < nch) {  // two stages left
    stage(c, a0, b0, a1, b1);
    mfma_stage(a1, b1);
  } else {            // one stage left
    mfma_stage(a0, b0);
  }

  // Epilogue.  Lane (j, g4) holds column 16q + j of block (p, q); its
  // accumulator element v is row g4 + 4v (the FP64 form interleaves rows
  // across the four lane groups, unlike the FP32 16 x 16 forms).
  const int64_t y0 = yt * TILE + wr * WTR;
  const int64_t x0 = xt * TILE + wc * WTC;
#pragma unroll
  for (int p = 0; p < FR; ++p) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t y = y0 + p * 16 + g4 + 4 * v;
      const int64_t rbase = Epi<EPI>::rowbase(zv, ea, y);
#pragma unroll
      for (int q = 0; q < FC; ++q) {
        const int64_t x = x0 + q * 16 + j;
        if (Epi<EPI>::keep(zv, y, x)) Epi<EPI>::emit(ea, rbase, y, x, clamp_unit(acc[p][q][v]));
      }
    }
  }
}

}  // namespace pcc
