// Uniform all-pairs kernels: Eq. (5) evaluated on the upper-triangle tiles
// only (Sec. III-C), every tile placed from its tile id by the bijection of
// Eq. (16)-(19) (or the banded order built on it).
//
// Persistent grid (the static stride of the multithreaded tile kernel over
// tile ids): workgroup b takes ids s(b), s(b) + G, s(b) + 2G, ..., where s()
// gives the workgroups of one XCD consecutive ids.  Every job has the same
// work, so the static stride balances without a counter.
#include "tile_core.h"

namespace pcc {
namespace {

struct UniformArgs {
  ZView zv;
  EpiArgs ea;
  int64_t m;      // tiles per side
  int64_t njobs;  // m(m+1)/2
  int32_t order;
  int32_t band;
};

template <int MODE, int TILE, int EPI>
__global__ __launch_bounds__(kTileThreads, 1) void tile_kernel(UniformArgs a) {
  __shared__ u32x4 smem[TileShape<TILE>::LDS_UNITS];
  const int64_t G = gridDim.x;
  for (int64_t J = xcd_slot(blockIdx.x, G); J < a.njobs; J += G) {
    const Cell tc = tile_of_job(a.m, a.order, a.band, J);
    do_tile<MODE, TILE, EPI>(a.zv, a.ea, tc.y, tc.x, smem);
  }
}

__global__ void zero_u64_kernel(unsigned long long *p) { *p = 0ull; }

template <int MODE, int EPI> const void *kernel_ptr_t(int tile) {
  return tile == 128 ? (const void *)tile_kernel<MODE, 128, EPI>
                     : (const void *)tile_kernel<MODE, 256, EPI>;
}

const void *kernel_for(int mode, int tile, int epi) {
  switch (mode) {
    case PCC_FP32:
      return epi ? kernel_ptr_t<PCC_FP32, 1>(tile) : kernel_ptr_t<PCC_FP32, 0>(tile);
    case PCC_SPLIT_BF16X3:
      return epi ? kernel_ptr_t<PCC_SPLIT_BF16X3, 1>(tile) : kernel_ptr_t<PCC_SPLIT_BF16X3, 0>(tile);
    case PCC_BF16:
      return epi ? kernel_ptr_t<PCC_BF16, 1>(tile) : kernel_ptr_t<PCC_BF16, 0>(tile);
    case PCC_FP16:
      return epi ? kernel_ptr_t<PCC_FP16, 1>(tile) : kernel_ptr_t<PCC_FP16, 0>(tile);
  }
  return nullptr;
}

__global__ void cells_kernel(int64_t m, int diag, int64_t J0, int64_t count, int64_t *y,
                             int64_t *x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const Cell c = diag ? tri_cell(m, J0 + t) : packed_cell(m, J0 + t);
  y[t] = c.y;
  x[t] = c.x;
}

UniformArgs make_args(const pcc_zdesc &zd, const void *z, const pcc_tile_cfg &cfg) {
  UniformArgs a{};
  a.zv.z = (const unsigned char *)z;
  a.zv.row_bytes = zd.row_bytes;
  a.zv.n = zd.n;
  a.zv.nchunks = (int32_t)(zd.l_pad / zd.kchunk);
  a.zv.scale = (zd.mode == PCC_FP16) ? (float)(1.0 / (double)zd.l) : 1.0f;
  a.m = (zd.n + cfg.tile - 1) / cfg.tile;
  a.njobs = a.m * (a.m + 1) / 2;
  a.order = cfg.order;
  a.band = cfg.band;
  return a;
}

hipError_t launch(const pcc_zdesc &zd, UniformArgs a, int tile, int epi, int grid,
                  hipStream_t st) {
  const void *k = kernel_for(zd.mode, tile, epi);
  if (!k) return hipErrorInvalidValue;
  void *args[] = {(void *)&a};
  return hipLaunchKernel(k, dim3(grid), dim3(kTileThreads), args, 0, st);
}

}  // namespace

int tile_occupancy(int mode, int tile, int epi) {
  static int cache[4][2][2] = {};
  if (mode < 0 || mode > 3) return 1;
  int &c = cache[mode][tile == 128 ? 0 : 1][epi ? 1 : 0];
  if (c == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel_for(mode, tile, epi), kTileThreads, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    c = nb;
  }
  return c;
}

hipError_t launch_allpairs(const pcc_zdesc &zd, const void *z, float *r, const pcc_tile_cfg &cfg,
                           int grid, hipStream_t st) {
  UniformArgs a = make_args(zd, z, cfg);
  a.ea.r = r;
  return launch(zd, a, cfg.tile, EPI_PACKED, grid, st);
}

hipError_t launch_edges(const pcc_zdesc &zd, const void *z, float thr, int32_t *ij, float *rv,
                        int64_t cap, int64_t *count, const pcc_tile_cfg &cfg, int grid,
                        hipStream_t st) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, st, (unsigned long long *)count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  UniformArgs a = make_args(zd, z, cfg);
  a.ea.thr = thr;
  a.ea.ij = ij;
  a.ea.rv = rv;
  a.ea.cap = cap;
  a.ea.count = (unsigned long long *)count;
  return launch(zd, a, cfg.tile, EPI_EDGES, grid, st);
}

hipError_t launch_cells(int64_t m, int diag, int64_t J0, int64_t count, int64_t *y, int64_t *x,
                        hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(cells_kernel, dim3((unsigned)blocks), dim3(256), 0, st, m, diag, J0, count,
                     y, x);
  return hipGetLastError();
}

}  // namespace pcc
