// Uneven batches: many independent datasets (different n and l) in one
// graph launch.  A plan uploads a descriptor table, then captures into one
// hipGraph:
//   1. a one-thread kernel zeroing the job counter (no memset node);
//   2. the batched transformation, Eq. (4), a grid-stride loop of waves
//      over the concatenated padded rows of every dataset;
//   3. one persistent all-pairs kernel whose workgroups draw tile jobs from
//      the shared counter (dynamic distribution through a shared integer
//      counter, which the all-pairs framework offers for jobs of varied
//      work) over the concatenated tile-id spaces; every dataset's ids are
//      mapped to its tile cells by Eq. (16)-(19) with its own m.
// Datasets are ordered by descending work per job so that the counter hands
// out the long jobs first.  Each tile is computed exactly as pcc_allpairs
// computes it with the same tile size, so batched and single results are
// bit-identical.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "norm_core.h"
#include "tile_core.h"

namespace pcc {
namespace {

struct BatchDesc {
  const void *x;
  int64_t ldx;
  int64_t n, l, l_pad, n_pad, row_bytes;
  unsigned char *z;
  float *r;
  int64_t m;     // tiles per side
  int64_t job0;  // first job id of this dataset in the concatenated space
  int64_t row0;  // first padded row of this dataset in the concatenated rows
  int32_t xt;
  int32_t tile;
  int32_t nchunks;
  float scale;
  double out_scale;  // normalisation multiplier (FP16 layout: sqrt(l))
};

constexpr size_t kCounterBytes = 256;

__device__ __forceinline__ int find_desc(const BatchDesc *d, int D, int64_t key, bool by_job) {
  int lo = 0, hi = D - 1;  // last dataset whose start <= key
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int64_t start = by_job ? d[mid].job0 : d[mid].row0;
    if (start <= key)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ void batch_zero_kernel(unsigned long long *counter) { *counter = 0ull; }

template <int MODE>
__global__ __launch_bounds__(256) void batch_norm_kernel(const BatchDesc *__restrict__ descs,
                                                         int D, int64_t total_rows) {
  const int64_t stride = (int64_t)gridDim.x * 4;
  for (int64_t R = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); R < total_rows; R += stride) {
    const BatchDesc &d = descs[find_desc(descs, D, R, false)];
    const int64_t row = R - d.row0;
    unsigned char *zr = d.z + row * d.row_bytes;
    if (row >= d.n) {
      zero_row(zr, d.row_bytes);
      continue;
    }
    if (d.xt == PCC_IN_F64) {
      const double *xr = (const double *)d.x + row * d.ldx;
      const bool vec = (d.ldx % 2 == 0) && ((reinterpret_cast<uintptr_t>(d.x) & 15) == 0);
      normalize_row<double, MODE, CacheOf<MODE>::C>(xr, d.l, d.l_pad, zr, nullptr, nullptr,
                                                    d.out_scale, vec);
    } else {
      const float *xr = (const float *)d.x + row * d.ldx;
      const bool vec = (d.ldx % 4 == 0) && ((reinterpret_cast<uintptr_t>(d.x) & 15) == 0);
      normalize_row<float, MODE, CacheOf<MODE>::C>(xr, d.l, d.l_pad, zr, nullptr, nullptr,
                                                   d.out_scale, vec);
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(kTileThreads, 1) void batch_tile_kernel(const BatchDesc *__restrict__ descs,
                                                            int D, int64_t total_jobs,
                                                            unsigned long long *counter) {
  __shared__ u32x4 smem[TileShape<256>::LDS_UNITS];
  __shared__ int64_t jslot;
  for (;;) {
    if (threadIdx.x == 0) jslot = (int64_t)atomicAdd(counter, 1ull);
    __syncthreads();
    const int64_t J = jslot;
    if (J >= total_jobs) break;  // uniform across the workgroup
    const BatchDesc &d = descs[find_desc(descs, D, J, true)];
    const Cell tc = tri_cell(d.m, J - d.job0);
    ZView zv{d.z, d.row_bytes, d.n, d.nchunks, d.scale, d.z, d.n};
    EpiArgs ea{};
    ea.r = d.r;
    // Consecutive jobs may use different tile sizes, whose stage copies give
    // a wave different LDS units: the previous job's last copies (possibly
    // still in flight) must land before any wave starts the next job's.
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    if (d.tile == 128)
      do_tile<MODE, 128, EPI_PACKED>(zv, ea, tc.y, tc.x, smem);
    else
      do_tile<MODE, 256, EPI_PACKED>(zv, ea, tc.y, tc.x, smem);
    // do_tile begins with a barrier, which every thread reaches after it has
    // read jslot, so thread 0 may overwrite jslot at the next iteration.
  }
}

template <int MODE>
hipError_t launch_batch(const BatchDesc *descs, int D, int64_t total_rows, int64_t total_jobs,
                        unsigned long long *counter, int cus, hipStream_t st) {
  hipLaunchKernelGGL(batch_zero_kernel, dim3(1), dim3(1), 0, st, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t nblocks = (total_rows + 3) / 4;
  if (nblocks > 65536) nblocks = 65536;
  hipLaunchKernelGGL((batch_norm_kernel<MODE>), dim3((unsigned)nblocks), dim3(256), 0, st, descs,
                     D, total_rows);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  int64_t grid = cus;
  if (grid > total_jobs) grid = total_jobs;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((batch_tile_kernel<MODE>), dim3((unsigned)grid), dim3(kTileThreads), 0, st, descs, D,
                     total_jobs, counter);
  return hipGetLastError();
}

}  // namespace
}  // namespace pcc

using namespace pcc;

struct pcc_batch_plan {
  int32_t D;
  int32_t mode;
  int64_t jobs;
  int64_t rows;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" {

size_t pcc_batch_workspace_size(int32_t D) {
  if (D < 0) return 0;
  return kCounterBytes + ((size_t)D * sizeof(BatchDesc) + 255) / 256 * 256;
}

pcc_status pcc_batch_plan_create(int32_t D, const pcc_batch_item *items, pcc_mode_t mode,
                                 void *workspace, size_t workspace_bytes, void *stream,
                                 pcc_batch_plan **plan) {
  if (!plan || D < 1 || !items) return PCC_E_ARG;
  *plan = nullptr;
  if (mode < PCC_FP32 || mode > PCC_FP16) return PCC_E_MODE;
  if (!workspace || workspace_bytes < pcc_batch_workspace_size(D)) return PCC_E_WORKSPACE;
  std::vector<BatchDesc> ds((size_t)D);
  for (int32_t k = 0; k < D; ++k) {
    const pcc_batch_item &it = items[k];
    if (!it.x || !it.z || !it.r) return PCC_E_ARG;
    if (it.xt != PCC_IN_F32 && it.xt != PCC_IN_F64) return PCC_E_ARG;
    pcc_zdesc zd;
    const pcc_status s = pcc_z_layout(it.n, it.l, mode, &zd);
    if (s != PCC_OK) return s;
    if (it.n < 2 || it.ldx < it.l) return PCC_E_SHAPE;
    int tile = it.tile;
    if (tile == 0) {
      pcc_tile_cfg c;
      pcc_default_cfg(&zd, &c);
      tile = c.tile;
    }
    if (tile != 128 && tile != 256) return PCC_E_ARG;
    BatchDesc &d = ds[(size_t)k];
    memset(&d, 0, sizeof(d));
    d.x = it.x;
    d.ldx = it.ldx;
    d.n = zd.n;
    d.l = zd.l;
    d.l_pad = zd.l_pad;
    d.n_pad = zd.n_pad;
    d.row_bytes = zd.row_bytes;
    d.z = (unsigned char *)it.z;
    d.r = it.r;
    d.m = (zd.n + tile - 1) / tile;
    d.xt = it.xt;
    d.tile = tile;
    d.nchunks = (int32_t)(zd.l_pad / zd.kchunk);
    d.scale = (mode == PCC_FP16) ? (float)(1.0 / (double)zd.l) : 1.0f;
    d.out_scale = (mode == PCC_FP16) ? sqrt((double)zd.l) : 1.0;
  }
  // Longest jobs first (work of one job ~ tile^2 * l_pad).
  std::stable_sort(ds.begin(), ds.end(), [](const BatchDesc &a, const BatchDesc &b) {
    return (double)a.tile * a.tile * a.l_pad > (double)b.tile * b.tile * b.l_pad;
  });
  int64_t jobs = 0, rows = 0;
  for (BatchDesc &d : ds) {
    d.job0 = jobs;
    d.row0 = rows;
    jobs += d.m * (d.m + 1) / 2;
    rows += d.n_pad;
  }
  hipStream_t st = (hipStream_t)stream;
  unsigned char *ws = (unsigned char *)workspace;
  BatchDesc *ddesc = (BatchDesc *)(ws + kCounterBytes);
  if (note_hip(hipMemcpyAsync(ddesc, ds.data(), ds.size() * sizeof(BatchDesc),
                              hipMemcpyHostToDevice, st)) != hipSuccess ||
      note_hip(hipStreamSynchronize(st)) != hipSuccess)
    return PCC_E_HIP;

  int dev = 0, cus = 0;
  if (note_hip(hipGetDevice(&dev)) != hipSuccess ||
      note_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return PCC_E_HIP;

  pcc_batch_plan *p = (pcc_batch_plan *)calloc(1, sizeof(pcc_batch_plan));
  if (!p) return PCC_E_ARG;
  p->D = D;
  p->mode = mode;
  p->jobs = jobs;
  p->rows = rows;
  hipStream_t cs = nullptr;
  if (note_hip(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) {
    free(p);
    return PCC_E_HIP;
  }
  pcc_status rs = PCC_OK;
  if (note_hip(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed)) != hipSuccess) {
    rs = PCC_E_HIP;
  } else {
    unsigned long long *counter = (unsigned long long *)ws;
    hipError_t e = hipErrorInvalidValue;
    switch (mode) {
      case PCC_FP32: e = launch_batch<PCC_FP32>(ddesc, D, rows, jobs, counter, cus, cs); break;
      case PCC_SPLIT_BF16X3:
        e = launch_batch<PCC_SPLIT_BF16X3>(ddesc, D, rows, jobs, counter, cus, cs);
        break;
      case PCC_BF16: e = launch_batch<PCC_BF16>(ddesc, D, rows, jobs, counter, cus, cs); break;
      case PCC_FP16: e = launch_batch<PCC_FP16>(ddesc, D, rows, jobs, counter, cus, cs); break;
    }
    hipGraph_t g = nullptr;
    note_hip(e);
    const hipError_t e2 = note_hip(hipStreamEndCapture(cs, &g));
    if (e != hipSuccess || e2 != hipSuccess || !g) {
      rs = PCC_E_HIP;
      if (g) hipGraphDestroy(g);
    } else {
      p->graph = g;
      if (note_hip(hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
        hipGraphDestroy(g);
        p->graph = nullptr;
        rs = PCC_E_HIP;
      }
    }
  }
  hipStreamDestroy(cs);
  if (rs != PCC_OK) {
    free(p);
    return rs;
  }
  *plan = p;
  return PCC_OK;
}

pcc_status pcc_batch_plan_launch(pcc_batch_plan *plan, void *stream) {
  if (!plan || !plan->exec) return PCC_E_ARG;
  return note_hip(hipGraphLaunch(plan->exec, (hipStream_t)stream)) == hipSuccess ? PCC_OK : PCC_E_HIP;
}

int64_t pcc_batch_plan_jobs(const pcc_batch_plan *plan) { return plan ? plan->jobs : -1; }

pcc_status pcc_batch_plan_destroy(pcc_batch_plan *plan) {
  if (!plan) return PCC_E_ARG;
  pcc_status s = PCC_OK;
  if (plan->exec && note_hip(hipGraphExecDestroy(plan->exec)) != hipSuccess) s = PCC_E_HIP;
  if (plan->graph && note_hip(hipGraphDestroy(plan->graph)) != hipSuccess) s = PCC_E_HIP;
  free(plan);
  return s;
}

}  // extern "C"
