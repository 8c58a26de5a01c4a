// Calibration probe, built as its own library (libpcc_probe.so), not part of
// the correlation ABI: a register-only loop of independent
// v_mfma_f32_32x32x16_bf16 chains with no memory traffic, which measures the
// MFMA rate the chip sustains under full load.  The tile kernels' roofline
// fraction is quoted against the nominal peak; this rate says how much of
// the gap is the clock the chip holds while every matrix core is busy.
#include <hip/hip_runtime.h>

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kChains = 8;  // independent accumulators per wave (covers MFMA latency)

__global__ __launch_bounds__(256) void mfma_loop(const bf16x8 *__restrict__ in,
                                                 float *__restrict__ out, int iters) {
  const bf16x8 a = in[threadIdx.x & 63];
  const bf16x8 b = in[(threadIdx.x + 7) & 63];
  f32x16 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[c][v] = 0.0f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int c = 0; c < kChains; ++c)
      acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c)
#pragma unroll
    for (int v = 0; v < 16; ++v) s += acc[c][v];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;  // keeps the loop live
}

}  // namespace

// in: 64 x 8 bf16 values (1 KiB, device); out: blocks * 256 floats (device).
// Each block is 4 waves; every wave issues iters * 8 MFMAs of 32 x 32 x 16,
// i.e. blocks * 4 * iters * 8 * 32768 flops in total.  Returns 0, or -1 if
// the launch failed.
extern "C" int pcc_probe_mfma_bf16(int blocks, int iters, const void *in, float *out,
                                   void *stream) {
  if (blocks <= 0 || iters <= 0 || !in || !out) return -1;
  hipLaunchKernelGGL(mfma_loop, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                     (const bf16x8 *)in, out, iters);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

extern "C" double pcc_probe_mfma_bf16_flops(int blocks, int iters) {
  return (double)blocks * 4.0 * iters * kChains * 32768.0;
}
