// Batched permutation test: for every pair y < x, the observed r and the r
// of P permutations of the second profile's samples, counting the
// permutations whose |r| reaches the observed |r| (significance by
// permutation testing, which the evaluation section motivates with at least
// 1,000 iterations of all-pairs r on permuted data).
//
// One persistent launch for all P permutations, in one of two kernels by
// Z's layout.  FP32 (v_mfma_f32_32x32x2_f32, r within about 1e-7: the test
// decides integers from |r| differences): a job is one 32 x 32 block of the
// pair matrix, placed by the bijection of Eq. (16)-(19) over 32-wide tiles,
// with both 32-profile panels in LDS for every sample, so a permutation
// costs no global traffic: permuting the column profile is only a different
// LDS read index, B[k][j] = Z_x[pi(k)] is a ds_read_b32 at column j, sample
// pi(k).  The 16 waves of a workgroup share the job and split the
// permutations two at a time (two accumulators sharing each A read), with no
// barrier until the job ends; after each pass a wave adds its hits to the
// job's counts in LDS, which are stored once.  Every wave first computes the
// observed r itself, by the same code path as a permutation with the
// identity index, so an identity permutation reproduces it bit for bit.
// Split-BF16x3 (three v_mfma_f32_32x32x16_bf16 per 16 samples, r within
// split's 1e-5) uses 64 x 32 jobs, further below.
#include <algorithm>

#include "pcc_internal.h"

namespace pcc {
hipError_t launch_allpairs(const pcc_zdesc &zd, const void *z, float *r, const pcc_tile_cfg &cfg,
                           int grid, hipStream_t st);
hipError_t launch_perm_tiles(const pcc_zdesc &zd, const void *z, const unsigned char *zp,
                             int64_t zp_stride, const float *robs, int32_t *cnt,
                             int64_t cnt_stride, int slots, const pcc_tile_cfg &cfg, int cus,
                             hipStream_t st);
int tile_occupancy(int mode, int tile, int epi);

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kBlk = 32;  // profiles per side of a job

__device__ __forceinline__ float clamp_unit(float r) {
  return r > 1.0f ? 1.0f : (r < -1.0f ? -1.0f : r);
}

__device__ __forceinline__ int64_t xcd_slot(int64_t b, int64_t G) {
  return (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
}

// LDS pitches (floats): A rows padded by one 16-byte unit (odd number of
// units: ds_read_b128 of 16 rows hit distinct bank groups); B rows by one
// float (the 32 lanes of a gather hit 32 distinct banks).
__host__ __device__ __forceinline__ int64_t pitch_a(int64_t l_pad) { return l_pad + 4; }
__host__ __device__ __forceinline__ int64_t pitch_b(int64_t l_pad) { return l_pad + 1; }

size_t lds_bytes(int64_t l_pad) {
  const size_t a = (size_t)kBlk * pitch_a(l_pad) * 4;
  const size_t b = ((size_t)kBlk * pitch_b(l_pad) * 4 + 15) / 16 * 16;
  return a + b + (size_t)kBlk * kBlk * 4;
}

// ---------------------------------------------------------------------------
// FP32 LDS layout: A rows as stored (pitch l_pad + 4 floats), B rows at pitch
// l_pad + 1 floats.
//
// Samples k >= l (padding) are zero in A, so whatever finite B value their
// index selects adds exactly zero: the permutation indices are loaded through
// a buffer descriptor that spans the row's l entries, and a load past them
// returns index 0.  (The split kernel relies on the same.)
//
// NP permutations per pass share every A read; WAVES waves split the
// permutations, wave w taking p = w, w + WAVES, ...; slot 0 of a wave's first
// pass is the identity (the observed r).

__device__ __forceinline__ bool bf16_is_nan(uint32_t h) { return (h & 0x7fffu) > 0x7f80u; }

// Indices of samples k0 .. k0 + 7 of one permutation row (byte offset off of
// k0).  The row's buffer descriptor spans exactly its l entries: a load past
// them returns 0, a valid index (see above).  Rows start on any 4-byte
// boundary unless ALIGNED (l % 4 == 0 and a 16-byte aligned matrix).
template <bool ALIGNED>
__device__ __forceinline__ void idx_load(__amdgpu_buffer_rsrc_t rs, uint32_t off, i32x4 (&d)[2]) {
  if constexpr (ALIGNED) {
    d[0] = __builtin_bit_cast(i32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
    d[1] = __builtin_bit_cast(i32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, off + 16, 0, 0));
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e)
      d[e >> 2][e & 3] = (int)__builtin_amdgcn_raw_buffer_load_b32(rs, off + 4 * e, 0, 0);
  }
}

// FP32 pass: a step is 8 samples, lane (i, g) taking k = 8t + 4g + e,
// e = 0..3, one sample per 32x32x2 MFMA (K = 2 across the lane halves); the
// indices go a step ahead as in the split pass.
template <bool ALIGNED>
__device__ __forceinline__ void idx_load4(__amdgpu_buffer_rsrc_t rs, uint32_t off, i32x4 &d) {
  if constexpr (ALIGNED) {
    d = __builtin_bit_cast(i32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0));
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) d[e] = (int)__builtin_amdgcn_raw_buffer_load_b32(rs, off + 4 * e, 0, 0);
  }
}

template <int NP, bool IDENT0>
__device__ __forceinline__ void step_f32(const float *__restrict__ arow,
                                         const float *__restrict__ brow, int t, int g,
                                         const i32x4 (&idx)[NP], f32x16 (&acc)[NP]) {
  const int k0 = 8 * t + 4 * g;
  const f32x4 a = *reinterpret_cast<const f32x4 *>(arow + k0);
  float b[NP][4];
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int e = 0; e < 4; ++e) b[j][e] = (IDENT0 && j == 0) ? brow[k0 + e] : brow[idx[j][e]];
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int j = 0; j < NP; ++j)
      acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], b[j][e], acc[j], 0, 0, 0);
}

template <bool ALIGNED, int NP, bool IDENT0>
__device__ __forceinline__ void pass_f32(const float *__restrict__ arow,
                                         const float *__restrict__ brow,
                                         const __amdgpu_buffer_rsrc_t (&rs)[NP], int nt, int g,
                                         f32x16 (&acc)[NP]) {
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[j][v] = 0.0f;
  i32x4 even[NP], odd[NP];
  const uint32_t o0 = 16 * g;  // byte offset of sample 4g
#pragma unroll
  for (int j = 0; j < NP; ++j)
    if (!(IDENT0 && j == 0)) idx_load4<ALIGNED>(rs[j], o0, even[j]);
  for (int t = 0; t < nt; t += 2) {
#pragma unroll
    for (int j = 0; j < NP; ++j)
      if (!(IDENT0 && j == 0)) idx_load4<ALIGNED>(rs[j], o0 + 32 * (t + 1), odd[j]);
    __builtin_amdgcn_sched_barrier(0);
    step_f32<NP, IDENT0>(arow, brow, t, g, even, acc);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < NP; ++j)
      if (!(IDENT0 && j == 0)) idx_load4<ALIGNED>(rs[j], o0 + 32 * (t + 2), even[j]);
    __builtin_amdgcn_sched_barrier(0);
    step_f32<NP, IDENT0>(arow, brow, t + 1, g, odd, acc);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Descriptor over permutation row p (l entries).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t perm_row(const int32_t *perms, int64_t p, int l) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)(perms + p * l), (short)0, 4 * l, 0x00020000);
}

template <bool ALIGNED, int NP, int WAVES>
__global__ __launch_bounds__(64 * WAVES, 1) void permtest_f32_kernel(
    const unsigned char *__restrict__ z, int64_t row_bytes, int64_t n, int64_t l, int64_t l_pad,
    int64_t mb, const int32_t *__restrict__ perms, int32_t P, int32_t *__restrict__ counts) {
  constexpr int kT = 64 * WAVES;
  extern __shared__ __align__(16) unsigned char dyn[];
  const int64_t pa = 4 * pitch_a(l_pad);  // bytes
  const int64_t pb = pitch_b(l_pad);      // words
  unsigned char *sA = dyn;
  uint32_t *sB = reinterpret_cast<uint32_t *>(dyn + kBlk * pa);
  int32_t *sC = reinterpret_cast<int32_t *>(dyn + kBlk * pa + (kBlk * pb * 4 + 15) / 16 * 16);

  const int tid = threadIdx.x;
  // the wave index in an SGPR: permutation rows are then scalar base addresses
  const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i = lane & 31, g = lane >> 5;
  const int nt = (int)(l_pad / 8);
  const int64_t njobs = mb * (mb + 1) / 2;
  const int64_t G = gridDim.x;
  const int64_t u4 = l_pad / 4;   // 16-byte units per row

  for (int64_t J = xcd_slot(blockIdx.x, G); J < njobs; J += G) {
    const Cell cell = tri_cell(mb, J);
    const int64_t y0 = cell.y * kBlk, x0 = cell.x * kBlk;
    __syncthreads();  // the previous job is done with sA, sB, sC
    for (int64_t q = tid; q < kBlk * u4; q += kT) {
      const int64_t r = q / u4, u = q % u4;
      *reinterpret_cast<u32x4 *>(sA + r * pa + 16 * u) =
          *reinterpret_cast<const u32x4 *>(z + (y0 + r) * row_bytes + 16 * u);
    }
    for (int64_t q = tid; q < kBlk * u4; q += kT) {
      const int64_t r = q / u4, u = q % u4;
      const u32x4 v = *reinterpret_cast<const u32x4 *>(z + (x0 + r) * row_bytes + 16 * u);
      uint32_t *d = sB + r * pb + 4 * u;
      d[0] = v[0]; d[1] = v[1]; d[2] = v[2]; d[3] = v[3];
    }
    for (int q = tid; q < kBlk * kBlk; q += kT) sC[q] = 0;
    __syncthreads();

    if (w < P) {
      const unsigned char *arow = sA + (int64_t)i * pa;
      const uint32_t *brow = sB + (int64_t)i * pb;
      // accumulator register v of lane (i, g): row 8(v/4) + 4g + v%4, column
      // i; each pass adds its hits to the job's counts in LDS at once, so no
      // count stays in registers
      int32_t *crow = sC + (4 * g) * kBlk + i;
      f32x16 acc[NP], robs;
      {
        // the observed r in slot 0, permutations w, w + WAVES, ... after it;
        // a slot past P repeats permutation w and is not counted
        __amdgpu_buffer_rsrc_t rs[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) {
          const int64_t p = w + (int64_t)WAVES * (j - 1);
          rs[j] = perm_row(perms, j > 0 && p < P ? p : w, (int)l);
        }
        pass_f32<ALIGNED, NP, true>(reinterpret_cast<const float *>(arow),
                                    reinterpret_cast<const float *>(brow), rs, nt, g, acc);
#pragma unroll
        for (int v = 0; v < 16; ++v) robs[v] = fabsf(clamp_unit(acc[0][v]));
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          int c = 0;
#pragma unroll
          for (int j = 1; j < NP; ++j)
            if (w + (int64_t)WAVES * (j - 1) < P) c += (fabsf(clamp_unit(acc[j][v])) >= robs[v]) ? 1 : 0;
          atomicAdd(crow + (8 * (v >> 2) + (v & 3)) * kBlk, c);
        }
      }
      for (int64_t m0 = NP - 1; w + WAVES * m0 < P; m0 += NP) {
        __amdgpu_buffer_rsrc_t rs[NP];
        const int64_t p0 = w + WAVES * m0;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
          const int64_t p = p0 + (int64_t)WAVES * j;
          rs[j] = perm_row(perms, p < P ? p : p0, (int)l);
        }
        pass_f32<ALIGNED, NP, false>(reinterpret_cast<const float *>(arow),
                                     reinterpret_cast<const float *>(brow), rs, nt, g, acc);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          int c = 0;
#pragma unroll
          for (int j = 0; j < NP; ++j)
            if (p0 + (int64_t)WAVES * j < P) c += (fabsf(clamp_unit(acc[j][v])) >= robs[v]) ? 1 : 0;
          atomicAdd(crow + (8 * (v >> 2) + (v & 3)) * kBlk, c);
        }
      }
    }
    __syncthreads();
    for (int q = tid; q < kBlk * kBlk; q += kT) {
      const int r = q / kBlk, c = q % kBlk;
      const int64_t y = y0 + r, x = x0 + c;
      if (y < x && x < n) {
        // degenerate profiles are NaN rows of Z; sample 0 shows it
        const float a0 = *reinterpret_cast<const float *>(sA + r * pa);
        const float b0 = __builtin_bit_cast(float, sB[c * pb]);
        const bool nan = !(a0 == a0) || !(b0 == b0);
        counts[packed_index(n, y, x)] = nan ? -1 : sC[q];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Split-BF16x3 permutation test on 64 x 32 jobs.  B rows hold one 32-bit
// word per sample, hi in the low half and lo in the high half, so a single
// ds_read_b32 gather of sample pi(k) brings both BF16 operands of the
// sample; per 16 samples and slot, 8 gathers are regrouped by v_perm_b32
// into a hi and a lo operand vector.  On 32 x 32 jobs (the FP32 kernel's
// shape) each gathered word would feed one 32-row MFMA block, and at three
// BF16 MFMAs per 16 samples the gathers and the regrouping would weigh as
// much as the MFMAs.  Here a job is 64 rows by 32 columns (the two column
// halves of a 64-wide tile of the inclusive triangle, Eq. (16)-(19)), so
// every gathered word and its regrouping feed two 32-row blocks.  The 32
// permuted profiles stay in LDS for every sample, as in the FP32 kernel; the
// 64 unpermuted profiles are streamed through a ring of two segments of CS
// 32-sample chunks instead (a 64-row panel would not fit beside them), and
// all waves walk the samples in step: one barrier per segment, the next
// segment's copy in flight meanwhile.  Longer segments mean fewer barriers,
// so the launcher takes the longest that divides the row's chunks and fits
// the LDS beside the rows.
// A pass gives every wave NP slots; slot s of the job is the identity for
// s = 0 (the observed r, which wave 0 writes to LDS after the first pass)
// and permutation s - 1 after it.  The identity slot gathers through a
// table of indices 0, 1, 2, ..., so it runs the code of every other slot and
// an identity permutation reproduces the observed r bit for bit.
constexpr int kRows2 = 64;  // unpermuted profiles per job
constexpr int kIotaLen = 1024;

// A staged chunk holds 32 samples of the 64 rows, 144 bytes a row: the
// 128-byte chunk and one 16-byte unit of padding (9 units, an odd number, so
// the ds_read_b128 of 8 consecutive rows hit distinct bank groups).
constexpr int kChunkPitch = 144;
constexpr int kChunkBytes = kRows2 * kChunkPitch;

struct IotaTable {
  int32_t v[kIotaLen];
  constexpr IotaTable() : v() {
    for (int k = 0; k < kIotaLen; ++k) v[k] = k;
  }
};
__device__ const IotaTable kIota;

size_t lds_bytes_split64(int64_t l_pad, int cs) {
  const size_t b = ((size_t)kBlk * pitch_b(l_pad) * 4 + 15) / 16 * 16;
  return b + 2 * (size_t)cs * kChunkBytes + 2 * (size_t)kRows2 * kBlk * 4;
}

// One 16-sample step of NP slots on both 32-row blocks: per slot 8 gathers
// and 8 regroupings feed six MFMAs.  Every slot's gathers are issued before
// the first MFMA, so the later slots' LDS latency hides behind the earlier
// slots' MFMAs.  `ring` points at the step's staged chunk, rows kPitch bytes
// apart.
template <int NP, int kPitch>
__device__ __forceinline__ void step_split64(const unsigned char *__restrict__ ring,
                                             const uint32_t *__restrict__ brow, int t, int i,
                                             int g, const i32x4 (&idx)[NP][2],
                                             f32x16 (&acc)[NP][2]) {
  const unsigned char *ap = ring + i * kPitch + ((2 * (t & 1) + g) << 4);
  bf16x8 ah[2], al[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    ah[b] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(ap + b * 32 * kPitch));
    al[b] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(ap + b * 32 * kPitch + 64));
  }
  uint32_t wd[NP][8];
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int e = 0; e < 8; ++e) wd[j][e] = brow[idx[j][e >> 2][e & 3]];
  // (the scheduler would otherwise sink the later slots' gathers below the
  // first slot's MFMAs)
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    u32x4 h, o;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      h[q] = __builtin_amdgcn_perm(wd[j][2 * q + 1], wd[j][2 * q], 0x05040100u);
      o[q] = __builtin_amdgcn_perm(wd[j][2 * q + 1], wd[j][2 * q], 0x07060302u);
    }
    const bf16x8 bh = __builtin_bit_cast(bf16x8, h);
    const bf16x8 bl = __builtin_bit_cast(bf16x8, o);
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc[j][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[b], bh, acc[j][b], 0, 0, 0);
      acc[j][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[b], bl, acc[j][b], 0, 0, 0);
      acc[j][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[b], bh, acc[j][b], 0, 0, 0);
    }
  }
}

typedef __attribute__((address_space(3))) void lds_void;

// Copy chunk c of the job's 64 unpermuted rows (descriptor rz over those
// rows) into a staged chunk (64 rows of kChunkPitch bytes) by buffer-to-LDS
// DMA.  A DMA instruction fills 64 consecutive 16-byte LDS units; the staged
// chunk is 64 rows of 9 units (the last one padding), so instruction q fills
// linear units 64 q .. 64 q + 63, lane L the unit (row, slot) =
// divmod(64 q + L, 9), and a padding slot takes a copy of the row's first
// unit.  Wave w issues instructions w, w + W, ...
template <int W>
__device__ __forceinline__ void chunk_dma(__amdgpu_buffer_rsrc_t rz, unsigned char *dst, int c,
                                          uint32_t row_bytes, int w, int lane) {
  constexpr int kUPR = kChunkPitch / 16;  // 9 units per staged row, 9 instructions
#pragma unroll
  for (int k = 0; k < (kUPR + W - 1) / W; ++k) {
    const int q = w + k * W;
    if (q < kUPR) {
      const uint32_t m = (uint32_t)(64 * q + lane);
      const uint32_t r = m / kUPR, v0 = m % kUPR;
      const uint32_t v = v0 < 8u ? v0 : 0u;
      const uint32_t voff = r * row_bytes + (uint32_t)c * 128u + 16u * v;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rz, (lds_void *)(dst + q * 1024), 16, voff, 0, 0, 0);
    }
  }
}

template <bool ALIGNED, int W, int NP, int CS>
__global__ __launch_bounds__(64 * W, 1) void permtest_split64_kernel(
    const unsigned char *__restrict__ z, int64_t row_bytes, int64_t n, int64_t l, int64_t l_pad,
    int64_t mb, const int32_t *__restrict__ perms, int32_t P, int32_t *__restrict__ counts) {
  constexpr int kT = 64 * W;
  constexpr int kSlots = W * NP;  // slots per pass
  constexpr int kSegBytes = CS * kChunkBytes;  // one ring half
  extern __shared__ __align__(16) unsigned char dyn[];
  const int64_t pb = pitch_b(l_pad);  // words
  // observed |r| and counts first (small LDS offsets), then the ring, then
  // the permuted rows
  float *sRobs = reinterpret_cast<float *>(dyn);
  int32_t *sC = reinterpret_cast<int32_t *>(sRobs + kRows2 * kBlk);
  unsigned char *sRing = reinterpret_cast<unsigned char *>(sC + kRows2 * kBlk);
  uint32_t *sB = reinterpret_cast<uint32_t *>(sRing + 2 * kSegBytes);

  const int tid = threadIdx.x;
  const int lane = tid & 63, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i = lane & 31, g = lane >> 5;
  const int nc = (int)(l_pad / 32);  // chunks per row
  const int64_t njobs = mb * (mb + 1);  // two column halves per tile
  const int64_t G = gridDim.x;
  const int64_t g8 = l_pad / 8;
  const int npass = (P + kSlots) / kSlots;  // P + 1 slots, slot 0 the identity
  const uint32_t o0 = 32 * g;               // byte offset of sample 8g in an index row

  for (int64_t J = xcd_slot(blockIdx.x, G); J < njobs; J += G) {
    const Cell cell = tri_cell(mb, J >> 1);
    const int64_t y0 = cell.y * kRows2, x0 = cell.x * kRows2 + kBlk * (J & 1);
    if (x0 >= n) continue;  // the right half of a tile past the last profile
    __syncthreads();        // the previous job is done with the LDS
    for (int64_t q = tid; q < kBlk * g8; q += kT) {
      // samples 32c + 8s .. + 7: hi in unit s of chunk c, lo in unit s + 4
      const int64_t r = q / g8, c = (q % g8) >> 2, s = q & 3;
      const unsigned char *src = z + (x0 + r) * row_bytes + c * 128 + 16 * s;
      const u32x4 hv = *reinterpret_cast<const u32x4 *>(src);
      const u32x4 lv = *reinterpret_cast<const u32x4 *>(src + 64);
      uint32_t *d = sB + r * pb + 32 * c + 8 * s;
#pragma unroll
      for (int q2 = 0; q2 < 4; ++q2) {
        d[2 * q2] = (hv[q2] & 0xffffu) | (lv[q2] << 16);
        d[2 * q2 + 1] = (hv[q2] >> 16) | (lv[q2] & 0xffff0000u);
      }
    }
    for (int q = tid; q < kRows2 * kBlk; q += kT) sC[q] = 0;
    const __amdgpu_buffer_rsrc_t rz = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(z + y0 * row_bytes), (short)0, (int)(kRows2 * row_bytes), 0x00020000);
#pragma unroll
    for (int h = 0; h < CS; ++h) chunk_dma<W>(rz, sRing + h * kChunkBytes, h, (uint32_t)row_bytes, w, lane);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();

    const uint32_t *brow = sB + (int64_t)i * pb;
    int seq = 0;  // segments consumed in this job; the ring half is seq & 1
    for (int pass = 0; pass < npass; ++pass) {
      const int s0 = (pass * W + w) * NP;  // this wave's first slot
      const bool active = s0 <= P;
      __amdgpu_buffer_rsrc_t rs[NP];
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        // a slot past P repeats the wave's first slot and is not counted (an
        // inactive wave loads nothing, its descriptors only stay in range)
        const int s = (s0 + j <= P) ? s0 + j : (s0 <= P ? s0 : 0);
        rs[j] = s == 0 ? perm_row(kIota.v, 0, (int)l) : perm_row(perms, s - 1, (int)l);
      }
      f32x16 acc[NP][2];
#pragma unroll
      for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[j][b][v] = 0.0f;
      i32x4 even[NP][2], odd[NP][2];
      if (active) {
#pragma unroll
        for (int j = 0; j < NP; ++j) idx_load<ALIGNED>(rs[j], o0, even[j]);
      }
#pragma unroll 1
      for (int c = 0; c < nc; ++c) {
        // chunk h of the current segment is read from the ring half seq & 1
        // while chunk h of the next segment (CS chunks on, wrapping into the
        // next pass) is copied into the other half
        const int h = c % CS;
        const int cn = c + CS >= nc ? c + CS - nc : c + CS;
        chunk_dma<W>(rz, sRing + ((seq + 1) & 1) * kSegBytes + h * kChunkBytes, cn,
                  (uint32_t)row_bytes, w, lane);
        const unsigned char *ring = sRing + (seq & 1) * kSegBytes + h * kChunkBytes;
        if (active) {
          const int t = 2 * c;
#pragma unroll
          for (int j = 0; j < NP; ++j) idx_load<ALIGNED>(rs[j], o0 + 64 * (t + 1), odd[j]);
          __builtin_amdgcn_sched_barrier(0);
          step_split64<NP, kChunkPitch>(ring, brow, t, i, g, even, acc);
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int j = 0; j < NP; ++j) idx_load<ALIGNED>(rs[j], o0 + 64 * (t + 2), even[j]);
          __builtin_amdgcn_sched_barrier(0);
          step_split64<NP, kChunkPitch>(ring, brow, t + 1, i, g, odd, acc);
          __builtin_amdgcn_sched_barrier(0);
        }
        if (h == CS - 1) {
          asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's copies landed
          __syncthreads();
          ++seq;
        }
      }
      if (pass == 0) {
        // slot 0 of wave 0 is the observed r
        if (w == 0) {
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v)
              sRobs[(32 * b + 8 * (v >> 2) + 4 * g + (v & 3)) * kBlk + i] =
                  fabsf(clamp_unit(acc[0][b][v]));
        }
        __syncthreads();
      }
      if (active) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int q = (32 * b + 8 * (v >> 2) + 4 * g + (v & 3)) * kBlk + i;
            const float ro = sRobs[q];
            int cnt = 0;
#pragma unroll
            for (int j = 0; j < NP; ++j)
              if (s0 + j >= 1 && s0 + j <= P) cnt += (fabsf(clamp_unit(acc[j][b][v])) >= ro) ? 1 : 0;
            atomicAdd(sC + q, cnt);
          }
      }
    }
    __syncthreads();
    for (int q = tid; q < kRows2 * kBlk; q += kT) {
      const int r = q / kBlk, c = q % kBlk;
      const int64_t y = y0 + r, x = x0 + c;
      if (y < x && x < n) {
        // degenerate profiles are NaN rows of Z; sample 0 shows it
        const bool nan = bf16_is_nan(*reinterpret_cast<const uint16_t *>(z + y * row_bytes)) ||
                         bf16_is_nan(sB[c * pb] & 0xffffu);
        counts[packed_index(n, y, x)] = nan ? -1 : sC[q];
      }
    }
  }
}

// LDS one workgroup may allocate: the device's figure when a device is
// present, else gfx950's 160 KiB.
int64_t max_lds_per_block() {
  constexpr int64_t kGfx950Lds = 160 * 1024;
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return kGfx950Lds;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
      v <= 0)
    return kGfx950Lds;
  return v;
}

}  // namespace

// ---------------------------------------------------------------------------
// Permutation test on tiles, for rows of any length (the LDS kernel above
// holds both panels for every sample, which caps l_pad).  Per group of S
// permutations: S column-permuted copies of Z are gathered into the
// workspace, then one tile launch runs the symmetric tile schedule of Z
// against each copy (the all-pairs tile core, so an identity permutation
// reproduces the observed r bit for bit) and adds |r_p| >= |r_obs| to the
// copy's slot of counts; the slots are summed at the end.  The observed r
// comes first, from the all-pairs kernel on the same schedule.

// Row x of copy s: sample k of the copy is sample perms[p0 + s][k] of row x
// of Z (k < l); padding samples stay zero.  FP32 rows are l_pad floats in
// sample order; a split row is 128-byte chunks of 32 BF16 hi values and the
// 32 matching lo values.
//
// A workgroup of 16 waves takes R rows and every copy of the launch (with
// only 128 KB of LDS free for one workgroup per compute unit, 16 waves keep
// more of the gather's memory accesses in flight than 4).  The R rows are
// first staged in LDS as one 32-bit word per sample (the FP32 value, or the
// sample's hi in the low half and lo in the high half), so every gathered
// sample is one LDS read and each row is read from memory once per launch;
// each index of a permutation serves R rows.  A thread then writes 16-byte
// units of the copies: 4 samples (FP32), or the hi unit and lo unit of 8
// samples (split).
template <bool SPLIT>
__global__ __launch_bounds__(1024) void perm_gather_lds_kernel(
    const unsigned char *__restrict__ z, int64_t row_bytes, int64_t n_pad, int64_t l,
    int64_t l_pad, int R, const int32_t *__restrict__ perms, int64_t p0, int copies,
    unsigned char *__restrict__ zp, int64_t zp_stride) {
  extern __shared__ __align__(16) uint32_t rows[];  // R x l_pad words
  const int64_t x0 = (int64_t)blockIdx.x * R;
  const int nr = (int)((n_pad - x0) < R ? (n_pad - x0) : R);
  const int64_t u4 = l_pad / 4;  // 16-byte units of a staged row
  for (int64_t q = threadIdx.x; q < (int64_t)nr * u4; q += blockDim.x) {
    const int64_t r = q / u4, u = q - r * u4;
    u32x4 v;
    if constexpr (SPLIT) {
      // samples 4u .. 4u + 3: hi at chunk c, position 4u % 32, lo 64 bytes on
      const int64_t k = 4 * u, c = k >> 5, o = k & 31;
      const unsigned char *src = z + (x0 + r) * row_bytes + c * 128 + 2 * o;
      const uint2 h = *reinterpret_cast<const uint2 *>(src);
      const uint2 lo = *reinterpret_cast<const uint2 *>(src + 64);
      v[0] = (h.x & 0xffffu) | (lo.x << 16);
      v[1] = (h.x >> 16) | (lo.x & 0xffff0000u);
      v[2] = (h.y & 0xffffu) | (lo.y << 16);
      v[3] = (h.y >> 16) | (lo.y & 0xffff0000u);
    } else {
      v = *reinterpret_cast<const u32x4 *>(z + (x0 + r) * row_bytes + 16 * u);
    }
    *reinterpret_cast<u32x4 *>(rows + r * l_pad + 4 * u) = v;
  }
  __syncthreads();
  constexpr int kS = SPLIT ? 8 : 4;  // samples per thread step
  const int64_t steps = l_pad / kS;
  for (int s = 0; s < copies; ++s) {
    const int32_t *pr = perms + (p0 + s) * l;
    unsigned char *dst = zp + s * zp_stride + x0 * row_bytes;
    for (int64_t q = threadIdx.x; q < steps; q += blockDim.x) {
      const int64_t k0 = kS * q;
      int32_t idx[kS];
#pragma unroll
      for (int e = 0; e < kS; ++e) idx[e] = (k0 + e < l) ? pr[k0 + e] : -1;
      for (int r = 0; r < nr; ++r) {
        const uint32_t *row = rows + r * l_pad;
        uint32_t w[kS];
#pragma unroll
        for (int e = 0; e < kS; ++e) w[e] = idx[e] >= 0 ? row[idx[e]] : 0u;
        unsigned char *d = dst + r * row_bytes;
        if constexpr (SPLIT) {
          const int64_t c = k0 >> 5, u = (k0 & 31) >> 3;  // chunk, unit of 8 samples
          u32x4 hv, lv;
#pragma unroll
          for (int e2 = 0; e2 < 4; ++e2) {
            hv[e2] = (w[2 * e2] & 0xffffu) | (w[2 * e2 + 1] << 16);
            lv[e2] = (w[2 * e2] >> 16) | (w[2 * e2 + 1] & 0xffff0000u);
          }
          *reinterpret_cast<u32x4 *>(d + c * 128 + 16 * u) = hv;
          *reinterpret_cast<u32x4 *>(d + c * 128 + 64 + 16 * u) = lv;
        } else {
          *reinterpret_cast<u32x4 *>(d + 16 * q) = u32x4{w[0], w[1], w[2], w[3]};
        }
      }
    }
  }
}

// The same gather for rows too long to stage (one workgroup per row and
// copy, every sample read from memory).
template <bool SPLIT>
__global__ __launch_bounds__(256) void perm_gather_kernel(const unsigned char *__restrict__ z,
                                                         int64_t row_bytes, int64_t l,
                                                         int64_t l_pad,
                                                         const int32_t *__restrict__ perms,
                                                         int64_t p0, unsigned char *__restrict__ zp,
                                                         int64_t zp_stride) {
  const int64_t x = blockIdx.x, s = blockIdx.y;
  const unsigned char *src = z + x * row_bytes;
  unsigned char *dst = zp + s * zp_stride + x * row_bytes;
  const int32_t *pr = perms + (p0 + s) * l;
  if constexpr (SPLIT) {
    const int64_t units = l_pad / 8;  // groups of 8 samples
    for (int64_t q = threadIdx.x; q < units; q += blockDim.x) {
      const int64_t c = q >> 2, u = q & 3, k0 = 8 * q;
      uint32_t hw[4], lw[4];
#pragma unroll
      for (int e2 = 0; e2 < 4; ++e2) {
        uint32_t hv[2], lv[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int64_t k = k0 + 2 * e2 + h;
          hv[h] = lv[h] = 0u;
          if (k < l) {
            const int64_t pk = pr[k];
            const unsigned char *sp = src + (pk >> 5) * 128 + (pk & 31) * 2;
            hv[h] = *reinterpret_cast<const uint16_t *>(sp);
            lv[h] = *reinterpret_cast<const uint16_t *>(sp + 64);
          }
        }
        hw[e2] = hv[0] | (hv[1] << 16);
        lw[e2] = lv[0] | (lv[1] << 16);
      }
      unsigned char *d = dst + c * 128 + 16 * u;
      *reinterpret_cast<u32x4 *>(d) = u32x4{hw[0], hw[1], hw[2], hw[3]};
      *reinterpret_cast<u32x4 *>(d + 64) = u32x4{lw[0], lw[1], lw[2], lw[3]};
    }
  } else {
    const int64_t units = l_pad / 4;
    const float *sf = reinterpret_cast<const float *>(src);
    for (int64_t q = threadIdx.x; q < units; q += blockDim.x) {
      f32x4 v;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t k = 4 * q + e;
        v[e] = k < l ? sf[pr[k]] : 0.0f;
      }
      *reinterpret_cast<f32x4 *>(dst + 16 * q) = v;
    }
  }
}

__global__ void fill_i32_kernel(int32_t *p, int64_t count, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// counts[J] = -1 where the observed r is NaN (a degenerate profile), else the
// sum of the slots' counts (slots == 0: counts already holds them).
__global__ void perm_finalize_kernel(int32_t *__restrict__ counts, const float *__restrict__ robs,
                                     const int32_t *__restrict__ slot0, int slots, int64_t stride,
                                     int64_t np) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float ro = robs[i];
    int32_t c = 0;
    if (slots == 0) {
      c = counts[i];
    } else {
      for (int s = 0; s < slots; ++s) c += slot0[s * stride + i];
    }
    counts[i] = (ro == ro) ? c : -1;
  }
}

// Copies of Z (and count slots) per launch of the tiled permutation test:
// enough tile jobs per launch to fill the grid for a few rounds (about 2^27
// pair-copies), at most 32.
int permtest_slots(int64_t npairs) {
  if (npairs <= 0) return 1;
  int64_t s = ((int64_t)1 << 27) / npairs;
  if (s < 1) s = 1;
  if (s > 32) s = 32;
  return (int)s;
}

// Workspace of the tiled permutation test: [observed r | count slots (when
// more than one) | permuted copies of Z], each part 256-byte aligned.
struct PermWs {
  float *robs;
  int32_t *slots;
  int64_t slot_stride;  // counts between slots
  unsigned char *zp;
  size_t bytes;
};

PermWs perm_ws(const pcc_zdesc &zd, void *base) {
  const int64_t np = zd.n * (zd.n - 1) / 2;
  const int S = permtest_slots(np);
  const size_t rb = ((size_t)np * 4 + 255) / 256 * 256;
  unsigned char *b = (unsigned char *)base;
  PermWs w;
  w.robs = (float *)b;
  w.slots = S > 1 ? (int32_t *)(b + rb) : nullptr;
  w.slot_stride = (int64_t)(rb / 4);
  const size_t sb = S > 1 ? (size_t)S * rb : 0;
  w.zp = b + rb + sb;
  w.bytes = rb + sb + (size_t)S * (size_t)zd.bytes;
  return w;
}

size_t permtest_tiles_workspace(const pcc_zdesc &zd) { return perm_ws(zd, nullptr).bytes; }

hipError_t launch_permtest_tiles(const pcc_zdesc &zd, const void *z, const int32_t *perms,
                                 int32_t P, int32_t *counts, void *ws, const pcc_tile_cfg &cfg,
                                 int cus, hipStream_t st) {
  const int64_t np = zd.n * (zd.n - 1) / 2;
  const int S = permtest_slots(np);
  const PermWs w = perm_ws(zd, ws);
  const int amode = arith_mode(zd);
  int occ = tile_occupancy(amode, cfg.tile, 0);
  if (occ < 1) occ = 1;
  const int64_t m = (zd.n + cfg.tile - 1) / cfg.tile;
  // persistent workgroups of a tile launch (the observed r's launch has no
  // more than its tiles)
  const int64_t g0 = cfg.grid > 0 ? cfg.grid : (int64_t)(cus > 0 ? cus : 256) * occ;
  const int64_t grid = std::min<int64_t>(g0, m * (m + 1) / 2);
  hipError_t e = launch_allpairs(zd, z, w.robs, cfg, (int)grid, st);
  if (e != hipSuccess) return e;
  int32_t *cnt0 = S > 1 ? w.slots : counts;
  const int64_t cnt_stride = S > 1 ? w.slot_stride : 0;
  const int64_t nfill = S > 1 ? (int64_t)S * w.slot_stride : np;
  const int fblocks = (int)std::min<int64_t>((nfill + 255) / 256, 4096);
  if (nfill > 0) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(fblocks), dim3(256), 0, st, cnt0, nfill, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const bool split = amode == PCC_SPLIT_BF16X3;
  // rows staged per gather workgroup: as many as 128 KiB of LDS holds, at most 8
  const int64_t row_lds = zd.l_pad * 4;
  const int R = (int)std::min<int64_t>(8, ((int64_t)128 * 1024) / row_lds);
  if (R >= 1) {
    const size_t lds = (size_t)R * (size_t)row_lds;
    const void *gk = split ? (const void *)perm_gather_lds_kernel<true>
                           : (const void *)perm_gather_lds_kernel<false>;
    if ((e = hipFuncSetAttribute(gk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
        hipSuccess)
      return e;
  }
  // tile jobs of one copy, and workgroups of a tile launch
  const int64_t T = m * (m + 1) / 2;
  const int64_t G = std::max<int64_t>(1, g0);
  for (int64_t p0 = 0, sc = 0; p0 < P; p0 += sc) {
    // copies in this launch: the count (at most S) whose jobs fill the
    // grid's rounds best, the larger one on a tie
    sc = 1;
    double best = 0.0;
    for (int64_t c = 1; c <= std::min<int64_t>(S, P - p0); ++c) {
      const int64_t jobs = c * T;
      const double fill = (double)jobs / (double)(((jobs + G - 1) / G) * G);
      if (fill >= best) {
        best = fill;
        sc = c;
      }
    }
    if (R >= 1) {
      const size_t lds = (size_t)R * (size_t)row_lds;
      const unsigned blocks = (unsigned)((zd.n_pad + R - 1) / R);
      if (split)
        hipLaunchKernelGGL(perm_gather_lds_kernel<true>, dim3(blocks), dim3(1024), lds, st,
                           (const unsigned char *)z, zd.row_bytes, zd.n_pad, zd.l, zd.l_pad, R,
                           perms, p0, (int)sc, w.zp, zd.bytes);
      else
        hipLaunchKernelGGL(perm_gather_lds_kernel<false>, dim3(blocks), dim3(1024), lds, st,
                           (const unsigned char *)z, zd.row_bytes, zd.n_pad, zd.l, zd.l_pad, R,
                           perms, p0, (int)sc, w.zp, zd.bytes);
    } else if (split) {
      hipLaunchKernelGGL(perm_gather_kernel<true>, dim3((unsigned)zd.n_pad, (unsigned)sc), dim3(256),
                         0, st, (const unsigned char *)z, zd.row_bytes, zd.l, zd.l_pad, perms, p0,
                         w.zp, zd.bytes);
    } else {
      hipLaunchKernelGGL(perm_gather_kernel<false>, dim3((unsigned)zd.n_pad, (unsigned)sc),
                         dim3(256), 0, st, (const unsigned char *)z, zd.row_bytes, zd.l, zd.l_pad,
                         perms, p0, w.zp, zd.bytes);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = launch_perm_tiles(zd, z, w.zp, zd.bytes, w.robs, cnt0, cnt_stride, (int)sc, cfg, cus, st);
    if (e != hipSuccess) return e;
  }
  const int nblocks = (int)std::min<int64_t>((np + 255) / 256, 4096);
  if (np > 0) {
    hipLaunchKernelGGL(perm_finalize_kernel, dim3(nblocks), dim3(256), 0, st, counts, w.robs,
                       cnt0, S > 1 ? S : 0, cnt_stride, np);
    e = hipGetLastError();
  }
  return e;
}

int64_t permtest_max_l(int mode) {
  if (mode != PCC_FP32 && mode != PCC_SPLIT_BF16X3) return 0;
  // largest multiple of 32 whose LDS footprint fits one workgroup
  const int64_t cap = max_lds_per_block();
  int64_t lp = 0;
  if (mode == PCC_SPLIT_BF16X3) {
    while (lp + 32 <= kIotaLen && lds_bytes_split64(lp + 32, 1) <= (size_t)cap) lp += 32;
  } else {
    while (lds_bytes(lp + 32) <= (size_t)cap) lp += 32;
  }
  return lp;
}

// Kernel shapes: waves per workgroup and permutations per wave and pass; the
// split kernel's longest segment (chunks per barrier).
constexpr int kSplitWaves = 12;
constexpr int kSplitNP = 2;
constexpr int kSplitMaxCS = 4;
constexpr int kF32NP = 2;
constexpr int kF32Waves = 16;

template <int CS>
const void *split64_kernel(bool aligned) {
  return aligned ? (const void *)permtest_split64_kernel<true, kSplitWaves, kSplitNP, CS>
                 : (const void *)permtest_split64_kernel<false, kSplitWaves, kSplitNP, CS>;
}

hipError_t launch_permtest(const pcc_zdesc &zd, const void *z, const int32_t *perms, int32_t P,
                           int32_t *counts, int cus, hipStream_t st) {
  const bool aligned = (zd.l % 4) == 0 && ((reinterpret_cast<uintptr_t>(perms) & 15) == 0);
  const bool split = arith_mode(zd) == PCC_SPLIT_BF16X3;
  // split: 64-wide tiles, two jobs each; FP32: 32 x 32 jobs
  const int64_t mb = split ? (zd.n + kRows2 - 1) / kRows2 : (zd.n + kBlk - 1) / kBlk;
  const int64_t jobs = split ? mb * (mb + 1) : mb * (mb + 1) / 2;
  size_t lds;
  const void *k;
  int threads;
  if (split) {
    // the longest segment whose ring fits beside the rows
    const size_t cap = (size_t)max_lds_per_block();
    const int64_t nc = zd.l_pad / 32;
    int cs = kSplitMaxCS;
    while (cs > 1 && (nc % cs != 0 || lds_bytes_split64(zd.l_pad, cs) > cap)) --cs;
    lds = lds_bytes_split64(zd.l_pad, cs);
    k = cs >= 4 ? split64_kernel<4>(aligned)
        : cs == 3 ? split64_kernel<3>(aligned)
        : cs == 2 ? split64_kernel<2>(aligned) : split64_kernel<1>(aligned);
    threads = 64 * kSplitWaves;
  } else {
    lds = lds_bytes(zd.l_pad);
    k = aligned ? (const void *)permtest_f32_kernel<true, kF32NP, kF32Waves>
                : (const void *)permtest_f32_kernel<false, kF32NP, kF32Waves>;
    threads = 64 * kF32Waves;
  }
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int64_t grid = cus;
  if (grid > jobs) grid = jobs;
  const unsigned char *zp = (const unsigned char *)z;
  int64_t rb = zd.row_bytes, n = zd.n, l = zd.l, lp = zd.l_pad;
  void *args[] = {(void *)&zp, (void *)&rb, (void *)&n, (void *)&l, (void *)&lp, (void *)&mb,
                  (void *)&perms, (void *)&P, (void *)&counts};
  return hipLaunchKernel(k, dim3((unsigned)grid), dim3(threads), args, lds, st);
}

}  // namespace pcc
