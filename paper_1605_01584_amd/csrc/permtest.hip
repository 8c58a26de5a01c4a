// Batched permutation test: for every pair y < x, the observed r and the r
// of P permutations of the second profile's samples, counting the
// permutations whose |r| reaches the observed |r| (significance by
// permutation testing, which the evaluation section motivates with at least
// 1,000 iterations of all-pairs r on permuted data).
//
// One persistent launch for all P permutations.  A job is one 32 x 32 block
// of the pair matrix, placed by the bijection of Eq. (16)-(19) over 32-wide
// tiles.  Both 32-profile panels stay in LDS for every sample, so a
// permutation costs no global traffic at all: permuting the column profile
// is only a different LDS read index, B[k][j] = Z_x[pi(k)] is a ds_read_b32
// at column j, sample pi(k).  The 16 waves of a workgroup share the job and
// split the permutations (wave w takes p = w, w + 16, ...), two at a time
// (two independent accumulators), with no barrier until the job ends; their
// counts are summed with LDS atomics and stored once.
//
// Every wave first computes the observed r itself, by the same code path as
// a permutation with the identity index, so an identity permutation
// reproduces it bit for bit.  Two kernels, by Z's layout: FP32 MFMA
// (v_mfma_f32_32x32x2_f32, r within about 1e-7: the test decides integers
// from |r| differences) and split-BF16x3 (three v_mfma_f32_32x32x16_bf16 per
// 16 samples, about 5x the FP32 rate, r within split's 1e-5).
#include "pcc_internal.h"

namespace pcc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kBlk = 32;       // profiles per side of a job
constexpr int kWaves = 16;
constexpr int kThreads = 64 * kWaves;

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

// Permutation indices of samples k0..k0+3 for the permutation whose row is
// `row`, in two steps.  perm_load reads them branch-free (the address is
// clamped into the row), so the loads stay in the MFMA block instead of
// being fenced by divergent branches; perm_fix then gives samples at or
// beyond l (padding: A and B are zero there) their own index, exactly as
// the identity does.
template <bool ALIGNED>
__device__ __forceinline__ i32x4 perm_load(const int32_t *__restrict__ row, int l, int k0) {
  if constexpr (ALIGNED) {  // l % 4 == 0: a group is wholly inside or outside
    return *reinterpret_cast<const i32x4 *>(row + (k0 < l ? k0 : 0));
  } else {
    i32x4 r;
#pragma unroll
    for (int e = 0; e < 4; ++e) r[e] = row[k0 + e < l ? k0 + e : 0];
    return r;
  }
}

__device__ __forceinline__ i32x4 perm_fix(i32x4 raw, int64_t l, int k0) {
  i32x4 r;
#pragma unroll
  for (int e = 0; e < 4; ++e) r[e] = (k0 + e < l) ? raw[e] : k0 + e;
  return r;
}

// One pass of a wave: accumulators for two permutations (rows ra, rb of the
// permutation matrix; IDENT_*: the identity instead) over all samples.
// Lane (i, g) supplies A[i][k] and B[k][i] for its half's samples
// k = 8t + 4g + e, e = 0..3, at MFMA step (t, e).  The identity gathers
// through the same LDS read as a permutation, so an identity permutation
// reproduces the observed r bit for bit.  The indices of step t + 1 are
// loaded at the start of step t and first used after its MFMAs, so the
// gathers never wait for a global load issued in the same step.
template <bool ALIGNED, bool IDENT_A, bool IDENT_B>
__device__ __forceinline__ void pass2(const float *__restrict__ sA, const float *__restrict__ sB,
                                      int64_t pa_l, int64_t pb_l, const int32_t *__restrict__ ra,
                                      const int32_t *__restrict__ rb, int64_t l, int nt, int i,
                                      int g, f32x16 &accA, f32x16 &accB) {
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    accA[v] = 0.0f;
    accB[v] = 0.0f;
  }
  const float *arow = sA + (int64_t)i * pa_l;
  const float *bcol = sB + (int64_t)i * pb_l;
  i32x4 na = {}, nb = {};  // raw indices of the next step
  if constexpr (!IDENT_A) na = perm_load<ALIGNED>(ra, l, 4 * g);
  if constexpr (!IDENT_B) nb = perm_load<ALIGNED>(rb, l, 4 * g);
  for (int t = 0; t < nt; ++t) {
    const int k0 = 8 * t + 4 * g;
    const f32x4 a = *reinterpret_cast<const f32x4 *>(arow + k0);
    const i32x4 own = {k0, k0 + 1, k0 + 2, k0 + 3};
    const i32x4 ia = IDENT_A ? own : perm_fix(na, l, k0);
    const i32x4 ib = IDENT_B ? own : perm_fix(nb, l, k0);
    const int kn = (t + 1 < nt) ? k0 + 8 : k0;  // the last step reloads its own
    if constexpr (!IDENT_A) na = perm_load<ALIGNED>(ra, l, kn);
    if constexpr (!IDENT_B) nb = perm_load<ALIGNED>(rb, l, kn);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      accA = __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], bcol[ia[e]], accA, 0, 0, 0);
      accB = __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], bcol[ib[e]], accB, 0, 0, 0);
    }
    if constexpr (!IDENT_A || !IDENT_B) {
      // the index loads first in the block, then the gathers and the MFMAs;
      // the loaded values are first used here, after the MFMAs (an empty asm,
      // no load in it), so the wait for them falls at the end of the step
      __builtin_amdgcn_sched_group_barrier(0x020, (IDENT_A || IDENT_B) ? 1 : 2, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 9, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
      __builtin_amdgcn_sched_barrier(0);  // nothing moves across: the asm stays last
      asm volatile("" : "+v"(na), "+v"(nb));
    }
  }
}

template <bool ALIGNED>
__global__ __launch_bounds__(kThreads, 1) void permtest_kernel(
    const unsigned char *__restrict__ z, int64_t row_bytes, int64_t n, int64_t l, int64_t l_pad,
    int64_t mb, const int32_t *__restrict__ perms, int32_t P, int32_t *__restrict__ counts) {
  extern __shared__ __align__(16) unsigned char dyn[];
  const int64_t pa_l = pitch_a(l_pad), pb_l = pitch_b(l_pad);
  float *sA = reinterpret_cast<float *>(dyn);
  float *sB = sA + kBlk * pa_l;
  int32_t *sC = reinterpret_cast<int32_t *>(
      dyn + (size_t)kBlk * pa_l * 4 + ((size_t)kBlk * pb_l * 4 + 15) / 16 * 16);

  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int i = lane & 31, g = lane >> 5;
  const int nt = (int)(l_pad / 8);
  const int64_t njobs = mb * (mb + 1) / 2;
  const int64_t G = gridDim.x;
  const int64_t u4 = l_pad / 4;  // 16-byte units per row

  for (int64_t J = xcd_slot(blockIdx.x, G); J < njobs; J += G) {
    const Cell cell = tri_cell(mb, J);
    const int64_t y0 = cell.y * kBlk, x0 = cell.x * kBlk;
    __syncthreads();  // the previous job is done with sA, sB, sC
    for (int64_t q = tid; q < kBlk * u4; q += kThreads) {
      const int64_t r = q / u4, u = q % u4;
      const f32x4 va = *reinterpret_cast<const f32x4 *>(z + (y0 + r) * row_bytes + u * 16);
      *reinterpret_cast<f32x4 *>(sA + r * pa_l + 4 * u) = va;
      const f32x4 vb = *reinterpret_cast<const f32x4 *>(z + (x0 + r) * row_bytes + u * 16);
      float *d = sB + r * pb_l + 4 * u;
      d[0] = vb[0]; d[1] = vb[1]; d[2] = vb[2]; d[3] = vb[3];
    }
    for (int q = tid; q < kBlk * kBlk; q += kThreads) sC[q] = 0;
    __syncthreads();

    // Wave w: the observed r, then permutations w, w + 16, w + 32, ...
    f32x16 robs, accA, accB;
    int cnt[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) cnt[v] = 0;
    {
      if (w < P)
        pass2<ALIGNED, true, false>(sA, sB, pa_l, pb_l, perms, perms + (int64_t)w * l, l, nt, i,
                                    g, accA, accB);
      else
        pass2<ALIGNED, true, true>(sA, sB, pa_l, pb_l, perms, perms, l, nt, i, g, accA, accB);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        robs[v] = fabsf(clamp_unit(accA[v]));
        if (w < P) cnt[v] += (fabsf(clamp_unit(accB[v])) >= robs[v]) ? 1 : 0;
      }
    }
    for (int p = w + kWaves; p < P; p += 2 * kWaves) {
      // the second permutation of the last pass may not exist: the pass then
      // repeats the first one and its result is not counted
      const int p2 = p + kWaves;
      const bool two = p2 < P;
      pass2<ALIGNED, false, false>(sA, sB, pa_l, pb_l, perms + (int64_t)p * l,
                                   perms + (int64_t)(two ? p2 : p) * l, l, nt, i, g, accA, accB);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        cnt[v] += (fabsf(clamp_unit(accA[v])) >= robs[v]) ? 1 : 0;
        if (two) cnt[v] += (fabsf(clamp_unit(accB[v])) >= robs[v]) ? 1 : 0;
      }
    }
    // accumulator register v of lane (i, g): row 8(v/4) + 4g + v%4, column i
#pragma unroll
    for (int v = 0; v < 16; ++v)
      atomicAdd(&sC[(8 * (v >> 2) + 4 * g + (v & 3)) * kBlk + i], cnt[v]);
    __syncthreads();
    for (int q = tid; q < kBlk * kBlk; q += kThreads) {
      const int r = q / kBlk, c = q % kBlk;
      const int64_t y = y0 + r, x = x0 + c;
      if (y < x && x < n) {
        // degenerate profiles are NaN rows of Z (observed r is NaN)
        const bool nan = !(sA[r * pa_l] == sA[r * pa_l]) || !(sB[c * pb_l] == sB[c * pb_l]);
        counts[packed_index(n, y, x)] = nan ? -1 : sC[q];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Split-BF16x3 variant.  Z in the split layout (per 128-byte chunk the BF16
// hi parts of 32 samples, then their lo parts); r = sum of lo.hi + hi.lo +
// hi.hi products (v_mfma_f32_32x32x16_bf16), the arithmetic of the split
// all-pairs tiles.
//
// LDS: A rows are the chunks as stored (pitch 4 l_pad + 16 bytes, an odd
// number of 16-byte units); B rows hold one 32-bit word per sample, hi in
// the low half and lo in the high half (pitch l_pad + 1 words), so a single
// ds_read_b32 gather of sample pi(k) brings both BF16 operands of the
// sample.  Lane (i, g) at step t takes samples k = 16t + 8g + e, e = 0..7:
// its A hi and lo operands are one 16-byte unit each (unit 2(t mod 2) + g
// of chunk t/2, and the unit four further on), its B operands come from 8
// gathers regrouped into a hi and a lo vector.
//
// Samples k >= l (padding) are zero in A, so whatever finite B value their
// index selects adds exactly zero: the permutation indices are loaded through
// a buffer descriptor that spans the row's l entries, and a load past them
// returns index 0.
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

// One step (16 samples) of NP accumulators: gathers, hi/lo regrouping
// (v_perm_b32: the low halves of two words, then their high halves) and the
// three products per accumulator.
template <int NP, bool IDENT0>
__device__ __forceinline__ void step_split(const unsigned char *__restrict__ arow,
                                           const uint32_t *__restrict__ brow, int t, int g,
                                           const i32x4 (&idx)[NP][2], f32x16 (&acc)[NP]) {
  const int kb = 16 * t + 8 * g;
  const unsigned char *ap = arow + (t >> 1) * 128 + ((2 * (t & 1) + g) << 4);
  const bf16x8 ah = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(ap));
  const bf16x8 al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(ap + 64));
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    uint32_t wd[8];
#pragma unroll
    for (int e = 0; e < 8; ++e)
      wd[e] = (IDENT0 && j == 0) ? brow[kb + e] : brow[idx[j][e >> 2][e & 3]];
    u32x4 h, o;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      h[q] = __builtin_amdgcn_perm(wd[2 * q + 1], wd[2 * q], 0x05040100u);
      o[q] = __builtin_amdgcn_perm(wd[2 * q + 1], wd[2 * q], 0x07060302u);
    }
    const bf16x8 bh = __builtin_bit_cast(bf16x8, h);
    const bf16x8 bl = __builtin_bit_cast(bf16x8, o);
    acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc[j], 0, 0, 0);
    acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc[j], 0, 0, 0);
    acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc[j], 0, 0, 0);
  }
}

// One pass over all samples.  The indices of step t + 1 are loaded before
// step t runs, into the other of two register sets (steps go in pairs: nt
// is even), so a step never waits for a load it issued itself.
template <bool ALIGNED, int NP, bool IDENT0>
__device__ __forceinline__ void pass_split(const unsigned char *__restrict__ arow,
                                           const uint32_t *__restrict__ brow,
                                           const __amdgpu_buffer_rsrc_t (&rs)[NP], int nt, int g,
                                           f32x16 (&acc)[NP]) {
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[j][v] = 0.0f;
  i32x4 even[NP][2], odd[NP][2];
  const uint32_t o0 = 32 * g;  // byte offset of sample 8g
#pragma unroll
  for (int j = 0; j < NP; ++j)
    if (!(IDENT0 && j == 0)) idx_load<ALIGNED>(rs[j], o0, even[j]);
  // (scheduling barriers keep each group of loads ahead of the step it
  // overlaps: the compiler would otherwise sink them next to their use)
  for (int t = 0; t < nt; t += 2) {
#pragma unroll
    for (int j = 0; j < NP; ++j)
      if (!(IDENT0 && j == 0)) idx_load<ALIGNED>(rs[j], o0 + 64 * (t + 1), odd[j]);
    __builtin_amdgcn_sched_barrier(0);
    step_split<NP, IDENT0>(arow, brow, t, g, even, acc);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < NP; ++j)
      if (!(IDENT0 && j == 0)) idx_load<ALIGNED>(rs[j], o0 + 64 * (t + 2), even[j]);
    __builtin_amdgcn_sched_barrier(0);
    step_split<NP, IDENT0>(arow, brow, t + 1, g, odd, acc);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Descriptor over permutation row p (l entries).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t perm_row(const int32_t *perms, int64_t p, int l) {
  return __builtin_amdgcn_make_buffer_rsrc((void *)(perms + p * l), (short)0, 4 * l, 0x00020000);
}

template <bool ALIGNED, int NP, int WAVES>
__global__ __launch_bounds__(64 * WAVES, 1) void permtest_split_kernel(
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
  const int nt = (int)(l_pad / 16);
  const int64_t njobs = mb * (mb + 1) / 2;
  const int64_t G = gridDim.x;
  const int64_t u4 = l_pad / 4;   // 16-byte units per row
  const int64_t g8 = l_pad / 8;   // groups of 8 samples per row

  for (int64_t J = xcd_slot(blockIdx.x, G); J < njobs; J += G) {
    const Cell cell = tri_cell(mb, J);
    const int64_t y0 = cell.y * kBlk, x0 = cell.x * kBlk;
    __syncthreads();  // the previous job is done with sA, sB, sC
    for (int64_t q = tid; q < kBlk * u4; q += kT) {
      const int64_t r = q / u4, u = q % u4;
      *reinterpret_cast<u32x4 *>(sA + r * pa + 16 * u) =
          *reinterpret_cast<const u32x4 *>(z + (y0 + r) * row_bytes + 16 * u);
    }
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
        pass_split<ALIGNED, NP, true>(arow, brow, rs, nt, g, acc);
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
        pass_split<ALIGNED, NP, false>(arow, brow, rs, nt, g, acc);
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
        // degenerate profiles are NaN rows of Z; sample 0's hi part shows it
        const bool nan = bf16_is_nan(*reinterpret_cast<const uint16_t *>(sA + r * pa)) ||
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

int64_t permtest_max_l(int mode) {
  if (mode != PCC_FP32 && mode != PCC_SPLIT_BF16X3) return 0;
  // largest multiple of 32 whose LDS footprint fits one workgroup (both
  // modes store 4 bytes per sample)
  const int64_t cap = max_lds_per_block();
  int64_t lp = 0;
  while (lds_bytes(lp + 32) <= (size_t)cap) lp += 32;
  return lp;
}

// Split kernel shape: permutations per pass and waves per workgroup.
constexpr int kSplitNP = 2;
constexpr int kSplitWaves = 16;

hipError_t launch_permtest(const pcc_zdesc &zd, const void *z, const int32_t *perms, int32_t P,
                           int32_t *counts, int cus, hipStream_t st) {
  const int64_t mb = (zd.n + kBlk - 1) / kBlk;
  const int64_t jobs = mb * (mb + 1) / 2;
  const size_t lds = lds_bytes(zd.l_pad);
  const bool aligned = (zd.l % 4) == 0 && ((reinterpret_cast<uintptr_t>(perms) & 15) == 0);
  const bool split = zd.mode == PCC_SPLIT_BF16X3;
  const void *k;
  int threads;
  if (split) {
    k = aligned ? (const void *)permtest_split_kernel<true, kSplitNP, kSplitWaves>
                : (const void *)permtest_split_kernel<false, kSplitNP, kSplitWaves>;
    threads = 64 * kSplitWaves;
  } else {
    k = aligned ? (const void *)permtest_kernel<true> : (const void *)permtest_kernel<false>;
    threads = kThreads;
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
