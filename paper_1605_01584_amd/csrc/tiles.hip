// Uniform all-pairs kernels.
//
// Symmetric job matrix: Eq. (5) evaluated on the upper-triangle tiles only
// (Sec. III-C), every tile placed from its tile id by the bijection of
// Eq. (16)-(19) (or the banded order built on it).
// Non-symmetric job matrix (two variable sets): every tile of the
// mr x mc tile rectangle is a job, placed by Eq. (7)-(8) (or bands of tile
// rows walked column by column).
//
// Persistent grid (the static stride of the multithreaded tile kernel over
// tile ids): workgroup b takes ids s(b), s(b) + G, s(b) + 2G, ..., where s()
// gives the workgroups of one XCD consecutive ids.  Every job has the same
// work, so the static stride balances without a counter.
#include <atomic>

#include "tile_core.h"

namespace pcc {
namespace {

struct UniformArgs {
  ZView zv;
  EpiArgs ea;
  int64_t mr;     // tile rows
  int64_t mc;     // tile columns (non-symmetric)
  int64_t j0;     // first tile id of this launch
  int64_t njobs;  // one past the last tile id: mr(mr+1)/2 or mr mc for a whole run
  int64_t split;  // work units from j0 on: tile ids j0 + u for u < split, then
  int64_t nunits; // quarters: unit split + 4 s + q is quarter q of tile j0 + split + s
  int32_t order;
  int32_t band;
};

template <int EPI> constexpr bool is_rect() { return EPI == EPI_RECT || EPI == EPI_RECT_EDGES; }

// Persistent workgroups take work units u = slot, slot + G, ...  A unit is
// a whole tile job, except that the symmetric 256-wide FP32 kernels may
// compute the jobs of a last, mostly empty round as four 128 x 128 quarters
// each (units from a.split on), so that every workgroup has a share of it.
// Both tile widths sum every pair's samples in the same order: r is the
// same.  The BF16 modes gain nothing from it: the chip is power-limited
// there, and the compute units busy in a sparse last round run at a higher
// clock.
template <int MODE, int TILE, int EPI>
__global__ __launch_bounds__(kTileThreads, 1) void tile_kernel(UniformArgs a) {
  __shared__ u32x4 smem[TileShape<TILE>::LDS_UNITS];
  const int64_t G = gridDim.x;
  int64_t u = xcd_slot(blockIdx.x, G);
  for (; u < a.split; u += G) {
    const int64_t J = a.j0 + u;
    Cell tc;
    if constexpr (is_rect<EPI>())
      tc = rect_cell(a.mr, a.mc, a.order, a.band, J);
    else
      tc = tile_of_job(a.mr, a.order, a.band, J);
    if constexpr (MODE == PCC_FP64)
      do_tile_f64<EPI>(a.zv, a.ea, tc.y, tc.x, smem);
    else
      do_tile<MODE, TILE, EPI>(a.zv, a.ea, tc.y, tc.x, smem);
  }
  // A loop of its own, so that what the 128-wide code keeps in registers is
  // not held through the whole-tile loop.
  if constexpr (TILE == 256 && !is_rect<EPI>() && MODE == PCC_FP32) {
    if (u < a.nunits) {
      // copies of the last 256-wide call may still be in flight into LDS
      // units that the 128-wide layout uses differently
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    }
    for (; u < a.nunits; u += G) {
      const int64_t s = u - a.split;
      const Cell tc = tile_of_job(a.mr, a.order, a.band, a.j0 + a.split + (s >> 2));
      const int64_t qy = 2 * tc.y + ((s >> 1) & 1), qx = 2 * tc.x + (s & 1);
      if (qy > qx) continue;  // the lower quarter of a diagonal tile
      do_tile<MODE, 128, EPI>(a.zv, a.ea, qy, qx, smem);
    }
  }
}

__global__ void zero_u64_kernel(unsigned long long *p) { *p = 0ull; }

// Permutation test on tiles: slot s of a launch holds one column-permuted
// copy of Z (at zp + s * zp_stride) and its own counts (cnt + s *
// cnt_stride).  A job is (slot, tile), the tiles of a slot numbered as the
// symmetric schedule numbers them; every job is the only writer of its
// slot's counts in its tile.
struct PermTileArgs {
  ZView zv;                  // zc is set per job
  EpiArgs ea;                // robs, cnt (slot 0)
  const unsigned char *zp;
  int64_t zp_stride;         // bytes
  int64_t cnt_stride;        // counts
  int64_t m;                 // tiles per side
  int64_t T;                 // tiles per slot: m(m+1)/2
  int64_t njobs;             // slots * T
  int32_t order;
  int32_t band;
};

template <int MODE, int TILE>
__global__ __launch_bounds__(kTileThreads, 1) void perm_tile_kernel(PermTileArgs a) {
  __shared__ u32x4 smem[TileShape<TILE>::LDS_UNITS];
  const int64_t G = gridDim.x;
  for (int64_t u = xcd_slot(blockIdx.x, G); u < a.njobs; u += G) {
    // several copies per launch only when a copy has few tiles (the pairs
    // of n profiles are then fewer than 2^26): a 32-bit division, its result
    // said to be wave-uniform, which keeps the job decode in scalar registers
    // (a 64-bit division here made the 256-wide kernel spill in its K loop)
    int64_t s = 0, t = u;
    if (a.njobs > a.T) {
      s = __builtin_amdgcn_readfirstlane((uint32_t)u / (uint32_t)a.T);
      t = u - s * a.T;
    }
    const Cell tc = tile_of_job(a.m, a.order, a.band, t);
    ZView zv = a.zv;
    zv.zc = a.zp + s * a.zp_stride;
    EpiArgs ea = a.ea;
    ea.cnt = a.ea.cnt + s * a.cnt_stride;
    do_tile<MODE, TILE, EPI_PERM>(zv, ea, tc.y, tc.x, smem);
  }
}

const void *perm_kernel_for(int mode, int tile) {
  if (mode == PCC_FP32)
    return tile == 128 ? (const void *)perm_tile_kernel<PCC_FP32, 128>
                       : (const void *)perm_tile_kernel<PCC_FP32, 256>;
  if (mode == PCC_SPLIT_BF16X3)
    return tile == 128 ? (const void *)perm_tile_kernel<PCC_SPLIT_BF16X3, 128>
                       : (const void *)perm_tile_kernel<PCC_SPLIT_BF16X3, 256>;
  return nullptr;
}

template <int MODE, int EPI> const void *kernel_ptr_t(int tile) {
  if constexpr (MODE == PCC_FP64)
    return tile == 128 ? (const void *)tile_kernel<MODE, 128, EPI> : nullptr;
  else
    return tile == 128 ? (const void *)tile_kernel<MODE, 128, EPI>
                       : (const void *)tile_kernel<MODE, 256, EPI>;
}

template <int EPI> const void *kernel_for_epi(int mode, int tile) {
  switch (mode) {
    case PCC_FP32: return kernel_ptr_t<PCC_FP32, EPI>(tile);
    case PCC_SPLIT_BF16X3: return kernel_ptr_t<PCC_SPLIT_BF16X3, EPI>(tile);
    case PCC_BF16: return kernel_ptr_t<PCC_BF16, EPI>(tile);
    case PCC_FP16: return kernel_ptr_t<PCC_FP16, EPI>(tile);
    case PCC_FP64: return kernel_ptr_t<PCC_FP64, EPI>(tile);
  }
  return nullptr;
}

const void *kernel_for(int mode, int tile, int epi) {
  switch (epi) {
    case EPI_PACKED: return kernel_for_epi<EPI_PACKED>(mode, tile);
    case EPI_EDGES: return kernel_for_epi<EPI_EDGES>(mode, tile);
    case EPI_RECT: return kernel_for_epi<EPI_RECT>(mode, tile);
    case EPI_RECT_EDGES: return kernel_for_epi<EPI_RECT_EDGES>(mode, tile);
    case EPI_PACKED_F64:
      return mode == PCC_FP64 ? kernel_ptr_t<PCC_FP64, EPI_PACKED_F64>(tile) : nullptr;
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
  a.zv.zc = a.zv.z;
  a.zv.nc = zd.n;
  a.mr = (zd.n + cfg.tile - 1) / cfg.tile;
  a.mc = a.mr;
  a.njobs = a.mr * (a.mr + 1) / 2;
  a.order = cfg.order;
  a.band = cfg.band;
  return a;
}

UniformArgs make_args_xy(const pcc_zdesc &zdx, const void *zx, const pcc_zdesc &zdy,
                         const void *zy, const pcc_tile_cfg &cfg) {
  UniformArgs a = make_args(zdx, zx, cfg);
  a.zv.zc = (const unsigned char *)zy;
  a.zv.nc = zdy.n;
  a.mc = (zdy.n + cfg.tile - 1) / cfg.tile;
  a.njobs = a.mr * a.mc;
  return a;
}

// Work units of a launch over tile ids [j0, njobs) on `grid` workgroups:
// whole tiles, and for the symmetric 256-wide FP32 kernels the quarters of
// the last round's tiles when that round would leave more than half of the
// workgroups idle (its quarters then take at most two 128-wide rounds).
void plan_units(int mode, int tile, int epi, int64_t grid, UniformArgs &a) {
  const int64_t N = a.njobs - a.j0;
  a.split = N;
  a.nunits = N;
  const bool quarters = tile == 256 && mode == PCC_FP32 && (epi == EPI_PACKED || epi == EPI_EDGES);
  if (!quarters || N <= 0 || grid < 2) return;
  const int64_t T = N - (N - 1) / grid * grid;  // tiles of the last round
  if (2 * T > grid) return;
  a.split = N - T;
  a.nunits = a.split + 4 * T;
}

hipError_t launch(int mode, UniformArgs a, int tile, int epi, int grid, hipStream_t st) {
  const void *k = kernel_for(mode, tile, epi);
  if (!k) return hipErrorInvalidValue;
  if (grid < 1) grid = 1;
  plan_units(mode, tile, epi, grid, a);
  if (a.nunits < grid) grid = (int)a.nunits;
  if (grid < 1) return hipSuccess;  // empty range
  void *args[] = {(void *)&a};
  return hipLaunchKernel(k, dim3(grid), dim3(kTileThreads), args, 0, st);
}

hipError_t zero_count(int64_t *count, hipStream_t st) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, st, (unsigned long long *)count);
  return hipGetLastError();
}

}  // namespace

// Workgroups of a tile kernel one compute unit holds, queried once per
// kernel (calls from several host threads may race to fill an entry; they
// store the same value, and the entries are atomic).
int tile_occupancy(int mode, int tile, int epi) {
  static std::atomic<int> cache[5][2][5] = {};
  if (mode < 0 || mode > 4 || epi < 0 || epi > 4) return 1;
  std::atomic<int> &c = cache[mode][tile == 128 ? 0 : 1][epi];
  int v = c.load(std::memory_order_relaxed);
  if (v == 0) {
    int nb = 0;
    const void *k = kernel_for(mode, tile, epi);
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kTileThreads, 0) != hipSuccess ||
        nb < 1)
      nb = 1;
    c.store(nb, std::memory_order_relaxed);
    v = nb;
  }
  return v;
}

hipError_t launch_allpairs(const pcc_zdesc &zd, const void *z, float *r, const pcc_tile_cfg &cfg,
                           int grid, hipStream_t st) {
  UniformArgs a = make_args(zd, z, cfg);
  a.ea.r = r;
  return launch(arith_mode(zd), a, cfg.tile, EPI_PACKED, grid, st);
}

// Tile ids [j0, j1) of the symmetric schedule, r holding the packed
// triangle from index roff on (a contiguous slice when [j0, j1) is a whole
// number of tile rows, or of bands in the banded order).
hipError_t launch_allpairs_range(const pcc_zdesc &zd, const void *z, float *r, int64_t roff,
                                 const pcc_tile_cfg &cfg, int64_t j0, int64_t j1, int grid,
                                 hipStream_t st) {
  UniformArgs a = make_args(zd, z, cfg);
  a.ea.r = r;
  a.ea.roff = roff;
  a.j0 = j0;
  a.njobs = j1;
  return launch(arith_mode(zd), a, cfg.tile, EPI_PACKED, grid, st);
}

hipError_t launch_allpairs_f64(const pcc_zdesc &zd, const void *z, double *r,
                               const pcc_tile_cfg &cfg, int grid, hipStream_t st) {
  UniformArgs a = make_args(zd, z, cfg);
  a.ea.r64 = r;
  return launch(arith_mode(zd), a, cfg.tile, EPI_PACKED_F64, grid, st);
}

hipError_t launch_edges(const pcc_zdesc &zd, const void *z, float thr, int32_t *ij, float *rv,
                        int64_t cap, int64_t *count, const pcc_tile_cfg &cfg, int grid,
                        hipStream_t st) {
  hipError_t e = zero_count(count, st);
  if (e != hipSuccess) return e;
  UniformArgs a = make_args(zd, z, cfg);
  a.ea.thr = thr;
  a.ea.ij = ij;
  a.ea.rv = rv;
  a.ea.cap = cap;
  a.ea.count = (unsigned long long *)count;
  return launch(arith_mode(zd), a, cfg.tile, EPI_EDGES, grid, st);
}

hipError_t launch_allpairs_xy(const pcc_zdesc &zdx, const void *zx, const pcc_zdesc &zdy,
                              const void *zy, float *r, int64_t ldr, const pcc_tile_cfg &cfg,
                              int grid, hipStream_t st) {
  UniformArgs a = make_args_xy(zdx, zx, zdy, zy, cfg);
  a.ea.r = r;
  a.ea.ldr = ldr;
  return launch(arith_mode(zdx), a, cfg.tile, EPI_RECT, grid, st);
}

hipError_t launch_edges_xy(const pcc_zdesc &zdx, const void *zx, const pcc_zdesc &zdy,
                           const void *zy, float thr, int32_t *ij, float *rv, int64_t cap,
                           int64_t *count, const pcc_tile_cfg &cfg, int grid, hipStream_t st) {
  hipError_t e = zero_count(count, st);
  if (e != hipSuccess) return e;
  UniformArgs a = make_args_xy(zdx, zx, zdy, zy, cfg);
  a.ea.thr = thr;
  a.ea.ij = ij;
  a.ea.rv = rv;
  a.ea.cap = cap;
  a.ea.count = (unsigned long long *)count;
  return launch(arith_mode(zdx), a, cfg.tile, EPI_RECT_EDGES, grid, st);
}

// One launch of the tiled permutation test: `slots` permuted copies of Z
// against Z over the symmetric tile schedule of cfg, counts added in place.
hipError_t launch_perm_tiles(const pcc_zdesc &zd, const void *z, const unsigned char *zp,
                             int64_t zp_stride, const float *robs, int32_t *cnt,
                             int64_t cnt_stride, int slots, const pcc_tile_cfg &cfg, int cus,
                             hipStream_t st) {
  const int mode = arith_mode(zd);
  const void *k = perm_kernel_for(mode, cfg.tile);
  if (!k) return hipErrorInvalidValue;
  UniformArgs u = make_args(zd, z, cfg);
  PermTileArgs a{};
  a.zv = u.zv;
  a.ea.robs = robs;
  a.ea.cnt = cnt;
  a.zp = zp;
  a.zp_stride = zp_stride;
  a.cnt_stride = cnt_stride;
  a.m = u.mr;
  a.T = u.njobs;
  a.njobs = (int64_t)slots * u.njobs;
  a.order = cfg.order;
  a.band = cfg.band;
  if (a.njobs <= 0) return hipSuccess;
  static std::atomic<int> occ_cache[2][2] = {};
  std::atomic<int> &oc = occ_cache[mode == PCC_FP32 ? 0 : 1][cfg.tile == 128 ? 0 : 1];
  int occ = oc.load(std::memory_order_relaxed);
  if (occ == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, kTileThreads, 0) != hipSuccess ||
        occ < 1)
      occ = 1;
    oc.store(occ, std::memory_order_relaxed);
  }
  int64_t grid = cfg.grid > 0 ? cfg.grid : (int64_t)(cus > 0 ? cus : 256) * occ;
  if (grid > a.njobs) grid = a.njobs;
  void *args[] = {(void *)&a};
  return hipLaunchKernel(k, dim3((unsigned)grid), dim3(kTileThreads), args, 0, st);
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
