// Variable transformation, Eq. (4), of one matrix: a grid-stride loop of
// waves over the n_pad rows of Z (padding rows are zeroed).  HBM-bound: it
// reads n*l input elements and writes n_pad*row_bytes bytes; the FP64
// arithmetic (about 5 operations per sample) is far below the vector FP64
// rate.
#include <algorithm>

#include "norm_core.h"

namespace pcc {
namespace {

constexpr int kWaves = 4;  // waves (rows) per workgroup
// LDS per wave for the part of a row its registers do not hold (2048 FP32
// samples: rows of up to 4096 samples are read from memory once).
constexpr int kSpillBytesPerWave = 8192;

// Wave w of the grid-stride loop owns row group w: rows w * (64 / lanes) ..,
// one row per `lanes` lanes.
template <typename TIn, int MODE, bool VEC>
__global__ __launch_bounds__(64 * kWaves) void normalize_kernel(
    const TIn *__restrict__ x, int64_t ldx, int64_t n, int64_t l, int64_t n_pad, int64_t l_pad,
    int64_t row_bytes, unsigned char *__restrict__ z, double *__restrict__ stats,
    int32_t *__restrict__ n_degenerate, double out_scale, int lanes, int spill_units) {
  extern __shared__ __align__(16) unsigned char norm_lds[];
  TIn *spill = reinterpret_cast<TIn *>(norm_lds) +
               (size_t)(threadIdx.x >> 6) * spill_units * UnitOf<MODE>::E;
  const int64_t rpw = 64 / lanes;
  const int64_t groups = n_pad / rpw;
  const int64_t stride = (int64_t)gridDim.x * kWaves;
  for (int64_t w = (int64_t)blockIdx.x * kWaves + (threadIdx.x >> 6); w < groups; w += stride) {
    const int64_t row = w * rpw + (threadIdx.x & 63) / lanes;
    unsigned char *zr = z + row * row_bytes;
    if (row >= n) {
      zero_row(zr, row_bytes, lanes);
      continue;
    }
    normalize_row<TIn, MODE, CacheOf<TIn, MODE>::C, VEC>(x + row * ldx, l, l_pad, zr,
                                                         stats ? stats + 2 * row : nullptr,
                                                         n_degenerate, out_scale, lanes, spill,
                                                         spill_units);
  }
}

__global__ void fill_i32_kernel(int32_t *p, int32_t v) { *p = v; }

template <typename TIn, int MODE>
hipError_t launch_norm(const TIn *x, int64_t ldx, const pcc_zdesc &zd, void *z, double *stats,
                       int32_t *ndeg, hipStream_t st) {
  const bool vec = ((ldx * (int64_t)sizeof(TIn)) % 16 == 0) &&
                   ((reinterpret_cast<uintptr_t>(x) & 15) == 0);
  const double out_scale = (MODE == PCC_FP16) ? sqrt((double)zd.l) : 1.0;
  const int lanes = norm_lanes(zd.l_pad);
  const int64_t groups = zd.n_pad / (64 / lanes);  // n_pad is a multiple of 256
  int64_t blocks = (groups + kWaves - 1) / kWaves;
  if (blocks > 65536) blocks = 65536;
  // units past the registers' share, staged in LDS (only whole-wave rows
  // have them: a narrower group's row fits its registers by construction)
  constexpr int E = UnitOf<MODE>::E, kc = CacheOf<TIn, MODE>::C;
  int64_t tail = lanes == 64 ? zd.l_pad / E - 64 * kc : 0;
  if (tail < 0) tail = 0;
  const int spill_units = (int)std::min<int64_t>(tail, kSpillBytesPerWave / (E * sizeof(TIn)));
  const size_t lds = (size_t)kWaves * spill_units * E * sizeof(TIn);
  if (vec)
    hipLaunchKernelGGL((normalize_kernel<TIn, MODE, true>), dim3((unsigned)blocks),
                       dim3(64 * kWaves), lds, st, x, ldx, zd.n, zd.l, zd.n_pad, zd.l_pad,
                       zd.row_bytes, (unsigned char *)z, stats, ndeg, out_scale, lanes,
                       spill_units);
  else
    hipLaunchKernelGGL((normalize_kernel<TIn, MODE, false>), dim3((unsigned)blocks),
                       dim3(64 * kWaves), lds, st, x, ldx, zd.n, zd.l, zd.n_pad, zd.l_pad,
                       zd.row_bytes, (unsigned char *)z, stats, ndeg, out_scale, lanes,
                       spill_units);
  return hipGetLastError();
}

template <typename TIn>
hipError_t dispatch_mode(const TIn *x, int64_t ldx, const pcc_zdesc &zd, void *z, double *stats,
                         int32_t *ndeg, hipStream_t st) {
  // a split layout of short rows holds FP32 z (its tiles compute in FP32)
  switch (arith_mode(zd)) {
    case PCC_FP32: return launch_norm<TIn, PCC_FP32>(x, ldx, zd, z, stats, ndeg, st);
    case PCC_SPLIT_BF16X3: return launch_norm<TIn, PCC_SPLIT_BF16X3>(x, ldx, zd, z, stats, ndeg, st);
    case PCC_BF16: return launch_norm<TIn, PCC_BF16>(x, ldx, zd, z, stats, ndeg, st);
    case PCC_FP16: return launch_norm<TIn, PCC_FP16>(x, ldx, zd, z, stats, ndeg, st);
    case PCC_FP64: return launch_norm<TIn, PCC_FP64>(x, ldx, zd, z, stats, ndeg, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_normalize(const void *x, int xt, int64_t ldx, const pcc_zdesc &zd, void *z,
                            double *stats, int32_t *ndeg, hipStream_t st) {
  if (ndeg) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(1), 0, st, ndeg, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (xt == PCC_IN_F64)
    return dispatch_mode<double>((const double *)x, ldx, zd, z, stats, ndeg, st);
  return dispatch_mode<float>((const float *)x, ldx, zd, z, stats, ndeg, st);
}

}  // namespace pcc
