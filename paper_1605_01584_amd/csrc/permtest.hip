// Batched permutation test: for every pair y < x, the observed r and the r
// of P permutations of the second profile's samples, counting the
// permutations whose |r| reaches the observed |r| (significance by
// permutation testing, as the evaluation section motivates: at least 1,000
// iterations of all-pairs r on permuted data).
//
// One persistent launch for all P permutations.  A job is one 256 x 32 block
// of the pair matrix: tile J_t of the 256-wide tile triangle (Eq. (16)-(19))
// times one of its eight 32-column slices.  The job keeps the 32 column
// profiles resident in LDS for the whole sample range, so permuting them is
// only a different LDS read index: B[k][j] = Z_x[pi(k)] is a ds_read_b32 at
// column j, sample pi(k).  The 256 row profiles stream through a double
// buffered LDS stage as in the all-pairs kernel.  Observed r (identity
// permutation, same code path and same summation order, so an identity
// permutation reproduces it bit for bit), |r| comparisons and the counts stay
// in registers; counts are stored once per job.  FP32 MFMA
// (v_mfma_f32_32x32x2_f32): the test decides integers from differences of
// r that can be far below 1e-5, so it uses the most accurate tile path.
#include "pcc_internal.h"

namespace pcc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kRows = 256;    // row profiles per job
constexpr int kCols = 32;     // column profiles per job (one MFMA block wide)
constexpr int kAUnits = kRows * 8;  // LDS units (16 B) of one A stage
constexpr int kStaticLds = 2 * kAUnits * 16;  // double-buffered A stages

__device__ __forceinline__ float clamp_unit(float r) {
  return r > 1.0f ? 1.0f : (r < -1.0f ? -1.0f : r);
}

__device__ __forceinline__ int64_t xcd_slot(int64_t b, int64_t G) {
  return (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
}

// Dynamic LDS: [A stages | perm buffers (2 x l_pad int32) | B panel
// (32 x (l_pad + 1) floats; the odd pitch spreads the 32 columns over all
// banks)].
__global__ __launch_bounds__(256, 1) void permtest_kernel(
    const unsigned char *__restrict__ z, int64_t row_bytes, int64_t n, int64_t l, int64_t l_pad,
    int64_t m, const int32_t *__restrict__ perms, int32_t P, int32_t *__restrict__ counts) {
  extern __shared__ __align__(16) unsigned char dyn[];
  u32x4 *sA = reinterpret_cast<u32x4 *>(dyn);                       // [2][kAUnits]
  int32_t *sP = reinterpret_cast<int32_t *>(dyn + kStaticLds);      // [2][l_pad]
  float *sB = reinterpret_cast<float *>(dyn + kStaticLds + 2 * l_pad * 4);  // [32][l_pad+1]
  const int64_t pitch = l_pad + 1;

  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int i = lane & 31, g = lane >> 5;
  const int nchunks = (int)(l_pad / 32);
  const int64_t njobs = 8 * (m * (m + 1) / 2);
  const int64_t G = gridDim.x;

  const int u0 = tid & 7, r0 = tid >> 3;
  const int64_t goff = (int64_t)r0 * row_bytes + u0 * 16;
  const int64_t gstep = 32 * row_bytes;
  const int lslot = r0 * 8 + (u0 ^ (r0 & 7));

  for (int64_t J = xcd_slot(blockIdx.x, G); J < njobs; J += G) {
    const Cell tc = tri_cell(m, J >> 3);
    const int64_t y0 = tc.y * kRows;
    const int64_t x0 = tc.x * kRows + (J & 7) * kCols;
    const unsigned char *za = z + y0 * row_bytes;

    // Resident column panel: 32 rows of Z starting at x0, all l_pad samples.
    __syncthreads();  // the previous job's last reads of sB are done
    for (int64_t q = tid; q < (int64_t)kCols * (l_pad / 4); q += 256) {
      const int64_t j = q / (l_pad / 4), k4 = q % (l_pad / 4);
      const f32x4 v = *reinterpret_cast<const f32x4 *>(z + (x0 + j) * row_bytes + k4 * 16);
      float *dst = sB + j * pitch + 4 * k4;
      dst[0] = v[0]; dst[1] = v[1]; dst[2] = v[2]; dst[3] = v[3];
    }

    f32x16 robs[2];
    int cnt[2][16];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) cnt[b][v] = 0;

    for (int p = -1; p < P; ++p) {
      int32_t *perm = sP + (p & 1) * l_pad;
      const int32_t *src = perms + (int64_t)(p < 0 ? 0 : p) * l;
      for (int64_t k = tid; k < l_pad; k += 256) perm[k] = (p >= 0 && k < l) ? src[k] : (int32_t)k;

      f32x16 acc[2];
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[b][v] = 0.0f;

      u32x4 ra[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) ra[s] = *reinterpret_cast<const u32x4 *>(za + goff + s * gstep);
#pragma unroll
      for (int s = 0; s < 8; ++s) sA[lslot + 256 * s] = ra[s];
      __syncthreads();

      for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        const bool more = c + 1 < nchunks;
        if (more) {
          const int64_t cb = (int64_t)(c + 1) * 128;
#pragma unroll
          for (int s = 0; s < 8; ++s)
            ra[s] = *reinterpret_cast<const u32x4 *>(za + goff + s * gstep + cb);
        }
        const u32x4 *stage = sA + buf * kAUnits + (w * 64) * 8;
        const float *bcol = sB + i * pitch;  // this lane's column x0 + i
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int uu = (2 * t + g) ^ (i & 7);
          const f32x4 a0 = __builtin_bit_cast(f32x4, stage[(0 * 32 + i) * 8 + uu]);
          const f32x4 a1 = __builtin_bit_cast(f32x4, stage[(1 * 32 + i) * 8 + uu]);
          // samples 32c + 4(2t+g) + e, e = 0..3, the same ones the A unit holds
          const u32x4 pk = *reinterpret_cast<const u32x4 *>(perm + 32 * c + 4 * (2 * t + g));
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float bv = bcol[pk[e]];
            acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0[e], bv, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1[e], bv, acc[1], 0, 0, 0);
          }
        }
        if (more) {
#pragma unroll
          for (int s = 0; s < 8; ++s) sA[(buf ^ 1) * kAUnits + lslot + 256 * s] = ra[s];
        }
        __syncthreads();
      }

      if (p < 0) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 16; ++v) robs[b][v] = clamp_unit(acc[b][v]);
      } else {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 16; ++v)
            cnt[b][v] += (fabsf(clamp_unit(acc[b][v])) >= fabsf(robs[b][v])) ? 1 : 0;
      }
    }

    // rows of the wave: y0 + 64w + 32b + 8(v/4) + 4g + v%4; column x0 + i
    const int64_t x = x0 + i;
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t y = y0 + w * 64 + b * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
        if (y < x && x < n) {
          const int32_t c = (robs[b][v] == robs[b][v]) ? cnt[b][v] : -1;
          counts[packed_index(n, y, x)] = c;
        }
      }
  }
}

size_t permtest_lds_bytes(int64_t l_pad) {
  return (size_t)kStaticLds + 2 * (size_t)l_pad * 4 + (size_t)kCols * (size_t)(l_pad + 1) * 4;
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
  if (mode != PCC_FP32) return 0;
  // largest multiple of 32 whose LDS footprint fits one workgroup
  const int64_t cap = max_lds_per_block();
  int64_t lp = 32;
  while (permtest_lds_bytes(lp + 32) <= (size_t)cap) lp += 32;
  return permtest_lds_bytes(lp) <= (size_t)cap ? lp : 0;
}

hipError_t launch_permtest(const pcc_zdesc &zd, const void *z, const int32_t *perms, int32_t P,
                           int32_t *counts, int cus, hipStream_t st) {
  const int64_t m = (zd.n + kRows - 1) / kRows;
  const int64_t jobs = 8 * (m * (m + 1) / 2);
  const size_t lds = permtest_lds_bytes(zd.l_pad);
  hipError_t e = hipFuncSetAttribute((const void *)permtest_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int64_t grid = cus;
  if (grid > jobs) grid = jobs;
  hipLaunchKernelGGL(permtest_kernel, dim3((unsigned)grid), dim3(256), lds, st,
                     (const unsigned char *)z, zd.row_bytes, zd.n, zd.l, zd.l_pad, m, perms, P,
                     counts);
  return hipGetLastError();
}

}  // namespace pcc
