// Uneven batches: many independent datasets (different n and l) in one
// persistent kernel.  A plan uploads a descriptor table, then captures into
// one hipGraph:
//   1. a one-thread kernel zeroing the job counters (no memset node);
//   2. one persistent kernel that first transforms every dataset's rows,
//      Eq. (4) (row groups drawn from a shared counter), then, once every
//      row is done, computes the tile jobs drawn from a second counter
//      (dynamic distribution through a shared integer counter, which the
//      all-pairs framework offers for jobs of varied work) over the
//      concatenated tile-id spaces; every dataset's ids are mapped to its
//      tile cells by Eq. (16)-(19) with its own m.
// Datasets are ordered by descending work per job so that the counter hands
// out the long jobs first.  Each tile is computed exactly as pcc_allpairs
// computes it with the same tile size, and each row exactly as
// pcc_normalize transforms it, so batched and single results are
// bit-identical.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
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
  int64_t grp0;  // first row group (64 / lanes rows, one wave) of this dataset
  int32_t xt;
  int32_t tile;
  int32_t nchunks;
  int32_t lanes;  // lanes per row in the transformation (4, 8, 16, 32 or 64)
  float scale;
  double out_scale;  // normalisation multiplier (FP16 layout: sqrt(l))
};

constexpr size_t kCounterBytes = 512;  // four counters, 128 bytes apart

// Workspace: [job counters | descriptor table | job0 of every dataset |
// first row group of every dataset], each part 256-byte aligned.  A
// workgroup copies the start keys it searches (first job or first row group
// of each dataset) into LDS when there are at most kKeysInLds datasets, so
// that finding the dataset of
// a job or a row is a binary search in LDS instead of a chain of dependent
// global loads; larger batches search the compact key array in place.
constexpr int kKeysInLds = 1024;

constexpr size_t round256(size_t b) { return (b + 255) / 256 * 256; }

constexpr size_t batch_ws_bytes(int32_t D) {
  return kCounterBytes + round256((size_t)D * sizeof(BatchDesc)) +
         2 * round256((size_t)D * sizeof(int64_t));
}

// Datasets of one pcc_batch_run_noalloc call, and the size of its static
// scratch (their workspace).
constexpr int32_t kStaticMaxD = PCC_BATCH_NOALLOC_MAX_D;
constexpr size_t kStaticScratchBytes = batch_ws_bytes(kStaticMaxD);

// Whole workgroup; returns the keys to search (LDS copy or global array).
__device__ __forceinline__ const int64_t *load_keys(const int64_t *__restrict__ gkeys, int D,
                                                    int64_t *skeys) {
  if (D > kKeysInLds) return gkeys;
  for (int i = threadIdx.x; i < D; i += blockDim.x) skeys[i] = gkeys[i];
  __syncthreads();
  return skeys;
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Last dataset whose start key <= key.
__device__ __forceinline__ int find_desc(const int64_t *keys, int D, int64_t key) {
  int lo = 0, hi = D - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (keys[mid] <= key)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ void batch_zero_kernel(unsigned long long *counters) {
  if (threadIdx.x < 4) counters[16 * threadIdx.x] = 0ull;
}

// Row normalisation of a batch.  One kernel serves every input variant of
// the batch (FP32/FP64, vector or scalar loads), with the single-matrix
// kernel's row code and register cache.  A row is owned by `lanes` lanes:
// short rows share a wave (4 to 32 lanes each), so a wave has several rows'
// loads in flight at once.  The part of a row longer than the registers hold
// (more than 2048 samples) is staged in the wave's share of the tile LDS,
// which the transformation phase does not use (16 KB per wave: rows of up to
// 6144 FP32 samples are read from memory once); what remains is read again.
constexpr int kStageBytesPerWave = 16384;
static_assert(kStageBytesPerWave * (kTileThreads / 64) <= TileShape<256>::LDS_UNITS * 16,
              "the waves' staging areas lie inside the tile LDS");

template <typename TIn, int MODE, bool VEC>
__device__ __forceinline__ void batch_row(const TIn *xr, int64_t l, int64_t l_pad,
                                          unsigned char *zr, double out_scale, int lanes,
                                          unsigned char *stage) {
  constexpr int E = UnitOf<MODE>::E, kc = CacheOf<TIn, MODE>::C;
  // only whole-wave rows have units past the registers' share
  int64_t tail = lanes == 64 ? l_pad / E - 64 * kc : 0;
  if (tail < 0) tail = 0;
  constexpr int64_t cap = kStageBytesPerWave / (E * (int64_t)sizeof(TIn));
  normalize_row<TIn, MODE, kc, VEC>(xr, l, l_pad, zr, nullptr, nullptr, out_scale, lanes,
                                    reinterpret_cast<TIn *>(stage), (int)(tail < cap ? tail : cap));
}

// Row `row` (< n) of dataset d, by input type and alignment.
template <int MODE>
__device__ __forceinline__ void batch_dataset_row(const BatchDesc &d, int64_t row,
                                                  unsigned char *zr, int lanes,
                                                  unsigned char *stage) {
  if (d.xt == PCC_IN_F64) {
    const double *xr = (const double *)d.x + row * d.ldx;
    const bool vec = (d.ldx % 2 == 0) && ((reinterpret_cast<uintptr_t>(d.x) & 15) == 0);
    if (vec)
      batch_row<double, MODE, true>(xr, d.l, d.l_pad, zr, d.out_scale, lanes, stage);
    else
      batch_row<double, MODE, false>(xr, d.l, d.l_pad, zr, d.out_scale, lanes, stage);
  } else {
    const float *xr = (const float *)d.x + row * d.ldx;
    const bool vec = (d.ldx % 4 == 0) && ((reinterpret_cast<uintptr_t>(d.x) & 15) == 0);
    if (vec)
      batch_row<float, MODE, true>(xr, d.l, d.l_pad, zr, d.out_scale, lanes, stage);
    else
      batch_row<float, MODE, false>(xr, d.l, d.l_pad, zr, d.out_scale, lanes, stage);
  }
}

// kRowsAtOnce row groups of one FP32 dataset (all rows real, each fitting
// its lanes' registers: 32 floats per lane and row, 128 registers for the
// four), transformed together: every row's loads first.
constexpr int kRowsAtOnce = 4;

template <int MODE, typename TIn, bool VEC>
__device__ __forceinline__ void batch_rows_together(const BatchDesc &d, int64_t row0,
                                                    int64_t rows_per_group, int lanes) {
  const TIn *xr[kRowsAtOnce];
  unsigned char *zr[kRowsAtOnce];
#pragma unroll
  for (int r = 0; r < kRowsAtOnce; ++r) {
    const int64_t row = row0 + r * rows_per_group;
    xr[r] = (const TIn *)d.x + row * d.ldx;
    zr[r] = d.z + row * d.row_bytes;
  }
  normalize_rows_cached<TIn, MODE, CacheOf<TIn, MODE>::C, VEC, kRowsAtOnce>(
      xr, d.l, d.l_pad, zr, d.out_scale, lanes);
}

template <int MODE>
__device__ __forceinline__ void batch_dataset_rows_together(const BatchDesc &d, int64_t row0,
                                                            int64_t rows_per_group, int lanes) {
  if ((d.ldx % 4 == 0) && ((reinterpret_cast<uintptr_t>(d.x) & 15) == 0))
    batch_rows_together<MODE, float, true>(d, row0, rows_per_group, lanes);
  else
    batch_rows_together<MODE, float, false>(d, row0, rows_per_group, lanes);
}

// Row groups [W, W + kRowsAtOnce) together when they are of one dataset,
// all their rows are real and fit the lanes' registers; returns false (and
// does nothing) otherwise.  Whole wave, W wave-uniform.
template <int MODE>
__device__ __forceinline__ bool norm_row_groups_together(const BatchDesc *__restrict__ descs,
                                                         const int64_t *keys, int D, int64_t W) {
  const BatchDesc &d = descs[__builtin_amdgcn_readfirstlane(find_desc(keys, D, W))];
  const int lanes = d.lanes;
  const int64_t rpg = 64 / lanes;  // rows per group
  const int64_t last_row = (W + kRowsAtOnce - 1 - d.grp0) * rpg + rpg - 1;
  const bool f32 = MODE == PCC_SPLIT_BF16X3 && d.l_pad <= kSplitFp32MaxLPad;
  // padded units of a row against what the lanes' registers hold (32
  // samples per lane for every mode)
  if (d.xt != PCC_IN_F32 || last_row >= d.n || d.l_pad > (int64_t)32 * lanes) return false;
  const int64_t row0 = (W - d.grp0) * rpg + (int64_t)((threadIdx.x & 63) / lanes);
  if (f32)
    batch_dataset_rows_together<PCC_FP32>(d, row0, rpg, lanes);
  else
    batch_dataset_rows_together<MODE>(d, row0, rpg, lanes);
  return true;
}

// Row group W (one wave's rows) of the concatenated padded rows: its
// dataset by binary search in keys, then the rows of the group, `lanes`
// lanes each.  Whole wave; W and the dataset are wave-uniform, which keeps
// the descriptor in scalar registers.
template <int MODE>
__device__ __forceinline__ void norm_row_group(const BatchDesc *__restrict__ descs,
                                               const int64_t *keys, int D, int64_t W,
                                               unsigned char *stage) {
  const BatchDesc &d = descs[__builtin_amdgcn_readfirstlane(find_desc(keys, D, W))];
  const int lanes = d.lanes;
  const int64_t row = (W - d.grp0) * (64 / lanes) + (int64_t)((threadIdx.x & 63) / lanes);
  unsigned char *zr = d.z + row * d.row_bytes;
  if (row >= d.n) {
    zero_row(zr, d.row_bytes, lanes);
    return;
  }
  // a split dataset of short rows holds FP32 z, as the single-matrix
  // transformation writes it
  if (MODE == PCC_SPLIT_BF16X3 && d.l_pad <= kSplitFp32MaxLPad)
    batch_dataset_row<PCC_FP32>(d, row, zr, lanes, stage);
  else
    batch_dataset_row<MODE>(d, row, zr, lanes, stage);
}

// The batch in one persistent kernel: first every workgroup transforms row
// groups drawn from a counter (Eq. (4); runs of row groups, one per wave),
// then, once every row group is done, tile jobs drawn from a second counter
// (both tile sizes; LDS sized for the 256-wide tiles, a 128-wide job uses
// the first half of it).
//
// The switch between the phases is a wait on a count of finished row groups.
// Only running workgroups claim row groups, and a claimed group is finished
// without waiting for anything, so the count always reaches the total: the
// wait needs no guarantee that every workgroup of the grid is resident.  A
// workgroup publishes its groups with one agent-scope release (the rows it
// wrote leave its XCD's L2) before adding them to the count, and a workgroup
// that has seen the full count does one agent-scope acquire before reading
// any Z; that is one write-back and one invalidation of an XCD's L2 per
// workgroup, all at the switch.  The wait is bounded (2 s of the real-time
// counter): should it ever expire, the kernel goes on and counts the event
// in counters[kTimeoutSlot] instead of hanging.
constexpr int kClaimSlot = 0, kDoneSlot = 16, kTileSlot = 32, kTimeoutSlot = 48;
constexpr int kClaimGroups = 16;  // row groups per claim
constexpr uint64_t kWaitTicks = 200000000ull;  // 2 s of the 100 MHz real-time counter

template <int MODE>
__global__ __launch_bounds__(kTileThreads, 1) void batch_kernel(const BatchDesc *__restrict__ descs,
                                                       const int64_t *__restrict__ job0s,
                                                       const int64_t *__restrict__ grp0s, int D,
                                                       int64_t total_groups, int64_t total_jobs,
                                                       unsigned long long *counters) {
  __shared__ u32x4 smem[TileShape<256>::LDS_UNITS];
  __shared__ int64_t jslot;
  __shared__ unsigned int wg_groups;
  __shared__ int64_t skeys[kKeysInLds];
  if (threadIdx.x == 0) wg_groups = 0u;
  __syncthreads();
  const int64_t *gkeys = load_keys(grp0s, D, skeys);
  // the wave's share of the tile LDS, for the long rows of phase 1
  unsigned char *stage = reinterpret_cast<unsigned char *>(smem) + (threadIdx.x >> 6) * kStageBytesPerWave;
  // phase 1: runs of kClaimGroups consecutive row groups, one run per wave
  // at a time (one claim per run keeps the shared counter off the path)
  unsigned int mine = 0u;
  for (;;) {
    unsigned long long w = 0ull;
    if ((threadIdx.x & 63) == 0) w = atomicAdd(counters + kClaimSlot, (unsigned long long)kClaimGroups);
    const int64_t W0 = uniform64((int64_t)w);
    if (W0 >= total_groups) break;
    const int64_t W1 = W0 + kClaimGroups < total_groups ? W0 + kClaimGroups : total_groups;
    for (int64_t W = W0; W < W1;) {
      if (W + kRowsAtOnce <= W1 && norm_row_groups_together<MODE>(descs, gkeys, D, W)) {
        W += kRowsAtOnce;
      } else {
        norm_row_group<MODE>(descs, gkeys, D, W, stage);
        ++W;
      }
    }
    mine += (unsigned int)(W1 - W0);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's rows are in L2
  if ((threadIdx.x & 63) == 0 && mine) atomicAdd(&wg_groups, mine);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (wg_groups) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(counters + kDoneSlot, (unsigned long long)wg_groups, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    bool late = false;
    while (__hip_atomic_load(counters + kDoneSlot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
           (unsigned long long)total_groups) {
      if (__builtin_amdgcn_s_memrealtime() - t0 > kWaitTicks) {
        late = true;
        break;
      }
      __builtin_amdgcn_s_sleep(4);
    }
    if (late) atomicAdd(counters + kTimeoutSlot, 1ull);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  // phase 2: tile jobs
  const int64_t *keys = load_keys(job0s, D, skeys);
  int prev = 0;  // tile size of the previous job
  for (;;) {
    if (threadIdx.x == 0) jslot = (int64_t)atomicAdd(counters + kTileSlot, 1ull);
    __syncthreads();
    // J and the dataset index are uniform across the workgroup; saying so
    // keeps the descriptor in scalar registers
    const int64_t J = uniform64(jslot);
    if (J >= total_jobs) break;
    const BatchDesc &d = descs[__builtin_amdgcn_readfirstlane(find_desc(keys, D, J))];
    const Cell tc = tri_cell(d.m, J - d.job0);
    ZView zv{d.z, d.row_bytes, d.n, d.nchunks, d.scale, d.z, d.n};
    EpiArgs ea{};
    ea.r = d.r;
    // short split rows hold FP32 z (same LDS layout as the split rows)
    const bool f32 = MODE == PCC_SPLIT_BF16X3 && d.nchunks * 32 <= kSplitFp32MaxLPad;
    const int kind = d.tile;
    // the last stage copy of a call may still be in flight into LDS units
    // that a job of the other tile size lays out differently
    if (prev != 0 && prev != kind) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    prev = kind;
    if (kind == 256) {
      if (f32)
        do_tile<PCC_FP32, 256, EPI_PACKED>(zv, ea, tc.y, tc.x, smem);
      else
        do_tile<MODE, 256, EPI_PACKED>(zv, ea, tc.y, tc.x, smem);
    } else {
      if (f32)
        do_tile<PCC_FP32, 128, EPI_PACKED>(zv, ea, tc.y, tc.x, smem);
      else
        do_tile<MODE, 128, EPI_PACKED>(zv, ea, tc.y, tc.x, smem);
    }
    // do_tile begins with a barrier, which every thread reaches after it has
    // read jslot, so thread 0 may overwrite jslot at the next iteration.
  }
}

template <int MODE>
hipError_t launch_batch(const BatchDesc *descs, const int64_t *job0s, const int64_t *grp0s, int D,
                        int64_t total_groups, int64_t jobs, unsigned long long *counters, int cus,
                        hipStream_t st) {
  hipLaunchKernelGGL(batch_zero_kernel, dim3(1), dim3(64), 0, st, counters);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || D <= 0) return e;
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_kernel<MODE>, kTileThreads, 0) !=
          hipSuccess ||
      occ < 1)
    occ = 1;
  const int64_t grid = (int64_t)cus * occ;
  hipLaunchKernelGGL((batch_kernel<MODE>), dim3((unsigned)grid), dim3(kTileThreads), 0, st, descs,
                     job0s, grp0s, D, total_groups, jobs, counters);
  return hipGetLastError();
}

}  // namespace
}  // namespace pcc

using namespace pcc;

namespace pcc {
namespace {

// Totals of a batch after build_batch.
struct BatchSums {
  int64_t jobs, groups, rows;
};

// Host work of a batch: validate the items, fill one descriptor per dataset,
// order them by decreasing work per job (l_pad * tile^2: the job counter
// hands out the long jobs first) and give each its first job, row and row
// group.  ds holds D descriptors.
// Stable ordering, by insertion for the few datasets of a call that may not
// allocate and by std::stable_sort otherwise: either way the order is the
// one the comparison fixes, so both entry points build the same table.
pcc_status build_batch(int32_t D, const pcc_batch_item *items, pcc_mode_t mode, BatchDesc *ds,
                       BatchSums *sums) {
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
    BatchDesc &d = ds[k];
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
    d.lanes = norm_lanes(zd.l_pad);
    d.scale = (mode == PCC_FP16) ? (float)(1.0 / (double)zd.l) : 1.0f;
    d.out_scale = (mode == PCC_FP16) ? sqrt((double)zd.l) : 1.0;
  }
  const auto before = [](const BatchDesc &a, const BatchDesc &b) {
    return a.l_pad * a.tile * a.tile > b.l_pad * b.tile * b.tile;
  };
  if (D <= kStaticMaxD) {
    for (int32_t k = 1; k < D; ++k) {
      const BatchDesc v = ds[k];
      int32_t j = k;
      for (; j > 0 && before(v, ds[j - 1]); --j) ds[j] = ds[j - 1];
      ds[j] = v;
    }
  } else {
    std::stable_sort(ds, ds + D, before);
  }
  BatchSums t{0, 0, 0};
  for (int32_t k = 0; k < D; ++k) {
    BatchDesc &d = ds[k];
    d.job0 = t.jobs;
    d.row0 = t.rows;
    d.grp0 = t.groups;
    t.jobs += d.m * (d.m + 1) / 2;
    t.rows += d.n_pad;
    t.groups += d.n_pad / (64 / d.lanes);  // n_pad is a multiple of 256
  }
  *sums = t;
  return PCC_OK;
}

// Descriptor table of a call that may not allocate: written into the
// static scratch by kernels that take the descriptors as arguments, so the
// call records no copy or fill node under stream capture.
constexpr int kDescsPerUpload = 8;
struct DescUpload {
  BatchDesc d[kDescsPerUpload];
};

__global__ void batch_upload_kernel(DescUpload u, int first, int count, BatchDesc *descs,
                                    int64_t *job0s, int64_t *grp0s) {
  const int k = threadIdx.x;
  if (k < count) {
    descs[first + k] = u.d[k];
    job0s[first + k] = u.d[k].job0;
    grp0s[first + k] = u.d[k].grp0;
  }
}

template <int MODE>
hipError_t launch_batch_mode(const BatchDesc *descs, const int64_t *job0s, const int64_t *grp0s,
                             int D, const BatchSums &t, unsigned long long *counters, int cus,
                             hipStream_t st) {
  return launch_batch<MODE>(descs, job0s, grp0s, D, t.groups, t.jobs, counters, cus, st);
}

hipError_t launch_batch_any(int mode, const BatchDesc *descs, const int64_t *job0s,
                            const int64_t *grp0s, int D, const BatchSums &t,
                            unsigned long long *counters, int cus, hipStream_t st) {
  switch (mode) {
    case PCC_FP32: return launch_batch_mode<PCC_FP32>(descs, job0s, grp0s, D, t, counters, cus, st);
    case PCC_SPLIT_BF16X3:
      return launch_batch_mode<PCC_SPLIT_BF16X3>(descs, job0s, grp0s, D, t, counters, cus, st);
    case PCC_BF16: return launch_batch_mode<PCC_BF16>(descs, job0s, grp0s, D, t, counters, cus, st);
    case PCC_FP16: return launch_batch_mode<PCC_FP16>(descs, job0s, grp0s, D, t, counters, cus, st);
  }
  return hipErrorInvalidValue;
}

// Workspace layout: [job counters | descriptor table | job0 keys | grp0 keys].
struct WsParts {
  unsigned long long *counters;
  BatchDesc *descs;
  int64_t *job0s, *grp0s;
};

WsParts ws_parts(void *ws, int32_t D) {
  unsigned char *b = (unsigned char *)ws;
  WsParts p;
  p.counters = (unsigned long long *)b;
  p.descs = (BatchDesc *)(b + kCounterBytes);
  p.job0s = (int64_t *)(b + kCounterBytes + round256((size_t)D * sizeof(BatchDesc)));
  p.grp0s = (int64_t *)((unsigned char *)p.job0s + round256((size_t)D * sizeof(int64_t)));
  return p;
}

// Scratch of pcc_batch_run_noalloc: the workspace of kStaticMaxD datasets in
// a file-scope device array.  Host code never passes this name to a kernel
// (on the host it is only a stand-in for the symbol): the device address
// comes from hipGetSymbolAddress, once per device, and is kept per device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::atomic<void *> g_scratch_addr[kMaxDevices];

// Device address of `scratch` on the current device.  Two threads may both
// look it up on a first call; they store the same address.
hipError_t scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  void *p = g_scratch_addr[dev].load(std::memory_order_acquire);
  if (!p) {
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[dev].store(p, std::memory_order_release);
  }
  *out = p;
  return hipSuccess;
}

int device_cus_or(int fallback) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    return fallback;
  return cus;
}

}  // namespace
}  // namespace pcc

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
  return batch_ws_bytes(D);
}

pcc_status pcc_batch_plan_create(int32_t D, const pcc_batch_item *items, pcc_mode_t mode,
                                 void *workspace, size_t workspace_bytes, void *stream,
                                 pcc_batch_plan **plan) {
  if (!plan || D < 1 || !items) return PCC_E_ARG;
  *plan = nullptr;
  if (mode < PCC_FP32 || mode > PCC_FP16) return PCC_E_MODE;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) ||
      workspace_bytes < pcc_batch_workspace_size(D))
    return PCC_E_WORKSPACE;
  std::vector<BatchDesc> ds((size_t)D);
  BatchSums t;
  const pcc_status bs = build_batch(D, items, mode, ds.data(), &t);
  if (bs != PCC_OK) return bs;
  const int64_t jobs = t.jobs;
  hipStream_t st = (hipStream_t)stream;
  const WsParts wp = ws_parts(workspace, D);
  std::vector<int64_t> keys(2 * (size_t)D);
  for (int32_t k = 0; k < D; ++k) {
    keys[(size_t)k] = ds[(size_t)k].job0;
    keys[(size_t)D + k] = ds[(size_t)k].grp0;
  }
  if (note_hip(hipMemcpyAsync(wp.descs, ds.data(), ds.size() * sizeof(BatchDesc),
                              hipMemcpyHostToDevice, st)) != hipSuccess ||
      note_hip(hipMemcpyAsync(wp.job0s, keys.data(), (size_t)D * sizeof(int64_t),
                              hipMemcpyHostToDevice, st)) != hipSuccess ||
      note_hip(hipMemcpyAsync(wp.grp0s, keys.data() + D, (size_t)D * sizeof(int64_t),
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
  p->rows = t.rows;
  hipStream_t cs = nullptr;
  if (note_hip(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) {
    free(p);
    return PCC_E_HIP;
  }
  pcc_status rs = PCC_OK;
  if (note_hip(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed)) != hipSuccess) {
    rs = PCC_E_HIP;
  } else {
    const hipError_t e =
        launch_batch_any(mode, wp.descs, wp.job0s, wp.grp0s, D, t, wp.counters, cus, cs);
    hipGraph_t g = nullptr;
    (void)note_hip(e);
    const hipError_t e2 = note_hip(hipStreamEndCapture(cs, &g));
    if (e != hipSuccess || e2 != hipSuccess || !g) {
      rs = PCC_E_HIP;
      if (g) (void)hipGraphDestroy(g);
    } else {
      p->graph = g;
      if (note_hip(hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(g);
        p->graph = nullptr;
        rs = PCC_E_HIP;
      }
    }
  }
  if (note_hip(hipStreamDestroy(cs)) != hipSuccess && rs == PCC_OK) rs = PCC_E_HIP;
  if (rs != PCC_OK) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    free(p);
    return rs;
  }
  *plan = p;
  return PCC_OK;
}

pcc_status pcc_batch_run_noalloc(int32_t D, const pcc_batch_item *items, pcc_mode_t mode,
                                 void *stream) {
  if (D < 1 || !items) return PCC_E_ARG;
  if (mode < PCC_FP32 || mode > PCC_FP16) return PCC_E_MODE;
  if (D > kStaticMaxD) return PCC_E_SHAPE;
  BatchDesc ds[kStaticMaxD];  // host stack, about 35 KB
  BatchSums t;
  const pcc_status bs = build_batch(D, items, mode, ds, &t);
  if (bs != PCC_OK) return bs;
  void *sp = nullptr;
  if (note_hip(scratch_address(&sp)) != hipSuccess) return PCC_E_HIP;
  const WsParts wp = ws_parts(sp, D);
  hipStream_t st = (hipStream_t)stream;
  for (int32_t k0 = 0; k0 < D; k0 += kDescsPerUpload) {
    DescUpload u;
    memset(&u, 0, sizeof(u));
    const int cnt = std::min<int32_t>(kDescsPerUpload, D - k0);
    for (int k = 0; k < cnt; ++k) u.d[k] = ds[k0 + k];
    hipLaunchKernelGGL(batch_upload_kernel, dim3(1), dim3(64), 0, st, u, (int)k0, cnt, wp.descs,
                       wp.job0s, wp.grp0s);
    if (note_hip(hipGetLastError()) != hipSuccess) return PCC_E_HIP;
  }
  // the job counters are zeroed by the batch's first kernel
  return note_hip(launch_batch_any(mode, wp.descs, wp.job0s, wp.grp0s, D, t, wp.counters,
                                   device_cus_or(256), st)) == hipSuccess
             ? PCC_OK
             : PCC_E_HIP;
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
