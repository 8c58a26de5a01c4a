// Host side of the C ABI declared in include/pcc.h: argument validation,
// the Z layout, schedule defaults, launches, host job maps and autotuning.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "pcc_internal.h"

namespace pcc {
hipError_t launch_normalize(const void *x, int xt, int64_t ldx, const pcc_zdesc &zd, void *z,
                            double *stats, int32_t *ndeg, hipStream_t st);
hipError_t launch_allpairs(const pcc_zdesc &zd, const void *z, float *r, const pcc_tile_cfg &cfg,
                           int grid, hipStream_t st);
hipError_t launch_allpairs_f64(const pcc_zdesc &zd, const void *z, double *r,
                               const pcc_tile_cfg &cfg, int grid, hipStream_t st);
hipError_t launch_allpairs_range(const pcc_zdesc &zd, const void *z, float *r, int64_t roff,
                                 const pcc_tile_cfg &cfg, int64_t j0, int64_t j1, int grid,
                                 hipStream_t st);
hipError_t launch_edges(const pcc_zdesc &zd, const void *z, float thr, int32_t *ij, float *rv,
                        int64_t cap, int64_t *count, const pcc_tile_cfg &cfg, int grid,
                        hipStream_t st);
hipError_t launch_allpairs_xy(const pcc_zdesc &zdx, const void *zx, const pcc_zdesc &zdy,
                              const void *zy, float *r, int64_t ldr, const pcc_tile_cfg &cfg,
                              int grid, hipStream_t st);
hipError_t launch_edges_xy(const pcc_zdesc &zdx, const void *zx, const pcc_zdesc &zdy,
                           const void *zy, float thr, int32_t *ij, float *rv, int64_t cap,
                           int64_t *count, const pcc_tile_cfg &cfg, int grid, hipStream_t st);
hipError_t launch_cells(int64_t m, int diag, int64_t J0, int64_t count, int64_t *y, int64_t *x,
                        hipStream_t st);
int tile_occupancy(int mode, int tile, int epi);
hipError_t launch_permtest(const pcc_zdesc &zd, const void *z, const int32_t *perms, int32_t P,
                           int32_t *counts, int cus, hipStream_t st);
int64_t permtest_max_l(int mode);
size_t permtest_tiles_workspace(const pcc_zdesc &zd);
int permtest_slots(int64_t npairs);
hipError_t launch_permtest_tiles(const pcc_zdesc &zd, const void *z, const int32_t *perms,
                                 int32_t P, int32_t *counts, void *ws, const pcc_tile_cfg &cfg,
                                 int cus, hipStream_t st);

namespace {

constexpr int64_t kMaxN = 2147483647LL;  // (i, j) of an edge are int32
constexpr int64_t kMaxL = 1LL << 21;  // a 256-row panel of Z stays within 2 GiB (32-bit offsets)

bool valid_mode(int m) { return m >= PCC_FP32 && m <= PCC_FP64; }

// Epilogue kinds of the tile kernels (as in the device core).
enum { kEpiPacked = 0, kEpiEdges = 1, kEpiRect = 2, kEpiRectEdges = 3, kEpiPackedF64 = 4 };

pcc_status check_zdesc(const pcc_zdesc *zd) {
  if (!zd) return PCC_E_ARG;
  if (!valid_mode(zd->mode)) return PCC_E_MODE;
  pcc_zdesc ref;
  const pcc_status s = pcc_z_layout(zd->n, zd->l, (pcc_mode_t)zd->mode, &ref);
  if (s != PCC_OK) return s;
  if (ref.n_pad != zd->n_pad || ref.l_pad != zd->l_pad || ref.row_bytes != zd->row_bytes ||
      ref.bytes != zd->bytes || ref.kchunk != zd->kchunk)
    return PCC_E_SHAPE;
  return PCC_OK;
}

pcc_status check_cfg(const pcc_zdesc &zd, const pcc_tile_cfg *in, pcc_tile_cfg &out) {
  if (in) {
    out = *in;
  } else {
    pcc_default_cfg(&zd, &out);
  }
  if (out.tile != 128 && out.tile != 256) return PCC_E_ARG;
  if (zd.mode == PCC_FP64 && out.tile != 128) return PCC_E_ARG;
  if (out.order != 0 && out.order != 1) return PCC_E_ARG;
  if (out.order == 1 && out.band < 1) return PCC_E_ARG;
  if (out.grid < 0) return PCC_E_ARG;
  return PCC_OK;
}

int device_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  return cus;
}

// Persistent grid: cfg.grid, or compute units x occupancy; never more
// workgroups than jobs.  ny > 0: the non-symmetric job matrix n x ny.
int grid_for(const pcc_zdesc &zd, const pcc_tile_cfg &cfg, int epi, int64_t ny = 0) {
  const int64_t m = (zd.n + cfg.tile - 1) / cfg.tile;
  const int64_t jobs = ny > 0 ? m * ((ny + cfg.tile - 1) / cfg.tile) : m * (m + 1) / 2;
  int64_t g = cfg.grid;
  if (g == 0) {
    const int cus = device_cus();
    int occ = tile_occupancy(arith_mode(zd), cfg.tile, epi);
    if (occ < 1) occ = 1;
    g = (int64_t)(cus > 0 ? cus : 256) * occ;
  }
  if (g > jobs) g = jobs;
  if (g < 1) g = 1;
  return (int)g;
}

pcc_status hip_status(hipError_t e) { return note_hip(e) == hipSuccess ? PCC_OK : PCC_E_HIP; }

// pcc_autotune's built-in candidates: both tile sizes, each in the paper's
// row order and in bands of 2, 4, 8 and 16 tile rows.
std::vector<pcc_tile_cfg> default_candidates() {
  std::vector<pcc_tile_cfg> list;
  for (int tile : {256, 128}) {
    list.push_back(pcc_tile_cfg{tile, 0, 1, 0});
    for (int b : {2, 4, 8, 16}) list.push_back(pcc_tile_cfg{tile, 1, b, 0});
  }
  return list;
}

thread_local hipError_t g_last_hip = hipSuccess;

}  // namespace

hipError_t note_hip(hipError_t e) {
  if (e != hipSuccess) g_last_hip = e;
  return e;
}

}  // namespace pcc

using namespace pcc;

extern "C" {

const char *pcc_status_string(pcc_status s) {
  switch (s) {
    case PCC_OK: return "PCC_OK";
    case PCC_E_ARG: return "PCC_E_ARG: null pointer or invalid argument";
    case PCC_E_SHAPE: return "PCC_E_SHAPE: size outside the supported range";
    case PCC_E_MODE: return "PCC_E_MODE: unknown or unsupported precision mode";
    case PCC_E_CAPACITY: return "PCC_E_CAPACITY: edge list capacity exceeded";
    case PCC_E_HIP: return "PCC_E_HIP: HIP runtime error";
    case PCC_E_WORKSPACE: return "PCC_E_WORKSPACE: workspace missing or too small";
    case PCC_E_DEVICE: return "PCC_E_DEVICE: no usable device";
  }
  return "unknown pcc_status";
}

int32_t pcc_version(void) { return 10000; }

int32_t pcc_last_hip_error(void) { return (int32_t)g_last_hip; }

const char *pcc_last_hip_error_string(void) { return hipGetErrorName(g_last_hip); }

pcc_status pcc_z_layout(int64_t n, int64_t l, pcc_mode_t mode, pcc_zdesc *out) {
  if (!out) return PCC_E_ARG;
  if (!valid_mode(mode)) return PCC_E_MODE;
  if (n < 1 || n > kMaxN || l < 2 || l > kMaxL) return PCC_E_SHAPE;
  pcc_zdesc d;
  memset(&d, 0, sizeof(d));
  d.n = n;
  d.l = l;
  d.mode = mode;
  d.kchunk = kchunk_of(mode);
  d.n_pad = (n + kRowPadMultiple - 1) / kRowPadMultiple * kRowPadMultiple;
  d.l_pad = (l + d.kchunk - 1) / d.kchunk * d.kchunk;
  d.row_bytes = d.l_pad / d.kchunk * kChunkBytes;
  d.bytes = d.n_pad * d.row_bytes;
  *out = d;
  return PCC_OK;
}

pcc_status pcc_default_cfg(const pcc_zdesc *zd, pcc_tile_cfg *out) {
  if (!zd || !out) return PCC_E_ARG;
  pcc_tile_cfg c;
  // Large triangles: 256-wide tiles (twice the arithmetic per staged byte)
  // in the banded order.  Small ones: 128-wide tiles so that every compute
  // unit gets work.
  const int64_t m256 = (zd->n + 255) / 256;
  if (zd->mode == PCC_FP64) {
    // FP64 tiles are 128 wide; FP64 MFMA is slow enough that 128-wide tiles
    // already do many flops per staged byte.
    const int64_t m128 = (zd->n + 127) / 128;
    c.tile = 128;
    c.order = 1;
    c.band = (m128 * (m128 + 1) / 2 >= 4 * 256) ? 8 : 4;
  } else if (m256 * (m256 + 1) / 2 >= 4 * 256) {
    c.tile = 256;
    c.order = 1;
    c.band = 8;
  } else {
    c.tile = 128;
    c.order = 1;
    c.band = 4;
  }
  c.grid = 0;
  *out = c;
  return PCC_OK;
}

pcc_status pcc_normalize(const void *x, pcc_in_t xt, int64_t ldx, const pcc_zdesc *zd, void *z,
                         double *stats, int32_t *n_degenerate, void *stream) {
  pcc_status s = check_zdesc(zd);
  if (s != PCC_OK) return s;
  if (!x || !z) return PCC_E_ARG;
  if (xt != PCC_IN_F32 && xt != PCC_IN_F64) return PCC_E_ARG;
  if (ldx < zd->l) return PCC_E_SHAPE;
  return hip_status(launch_normalize(x, xt, ldx, *zd, z, stats, n_degenerate, (hipStream_t)stream));
}

size_t pcc_workspace_size(const pcc_zdesc *zd, int32_t op) {
  if (check_zdesc(zd) != PCC_OK || zd->n < 2) return 0;
  const bool perm_mode = zd->mode == PCC_FP32 || zd->mode == PCC_SPLIT_BF16X3;
  if (op == 2 && perm_mode && zd->l_pad > permtest_max_l(zd->mode))
    return permtest_tiles_workspace(*zd);
  if (op == 3 && perm_mode) return permtest_tiles_workspace(*zd);
  return 0;
}

pcc_status pcc_allpairs(const pcc_zdesc *zd, const void *z, float *r, const pcc_tile_cfg *cfg,
                        void *workspace, void *stream) {
  (void)workspace;
  pcc_status s = check_zdesc(zd);
  if (s != PCC_OK) return s;
  if (zd->n < 2) return PCC_E_SHAPE;  // no pair
  if (!z || !r) return PCC_E_ARG;
  pcc_tile_cfg c;
  s = check_cfg(*zd, cfg, c);
  if (s != PCC_OK) return s;
  return hip_status(
      launch_allpairs(*zd, z, r, c, grid_for(*zd, c, kEpiPacked), (hipStream_t)stream));
}

pcc_status pcc_allpairs_f64(const pcc_zdesc *zd, const void *z, double *r,
                            const pcc_tile_cfg *cfg, void *workspace, void *stream) {
  (void)workspace;
  pcc_status s = check_zdesc(zd);
  if (s != PCC_OK) return s;
  if (zd->n < 2) return PCC_E_SHAPE;  // no pair
  if (zd->mode != PCC_FP64) return PCC_E_MODE;
  if (!z || !r) return PCC_E_ARG;
  pcc_tile_cfg c;
  s = check_cfg(*zd, cfg, c);
  if (s != PCC_OK) return s;
  return hip_status(launch_allpairs_f64(*zd, z, r, c, grid_for(*zd, c, kEpiPackedF64),
                                        (hipStream_t)stream));
}

// Packed-triangle slice of the tile rows [ya, yb) (clamped to the rows
// that hold pairs): [tri_F(n-1, ya T), tri_F(n-1, yb T)).
static void pass_slice(int64_t n, int64_t T, int64_t ya, int64_t yb, int64_t *first,
                       int64_t *count) {
  const int64_t a = std::min(n - 1, ya * T), b = std::min(n - 1, yb * T);
  *first = tri_F(n - 1, a);
  *count = tri_F(n - 1, b) - *first;
}

size_t pcc_stream_buffer_bytes(const pcc_zdesc *zd, const pcc_tile_cfg *cfg,
                               int64_t rows_per_pass) {
  pcc_tile_cfg c;
  if (check_zdesc(zd) != PCC_OK || zd->n < 2 || rows_per_pass < 1 ||
      check_cfg(*zd, cfg, c) != PCC_OK)
    return 0;
  // the first pass is the largest (the rows nearest the top are the longest)
  int64_t first = 0, count = 0;
  pass_slice(zd->n, c.tile, 0, rows_per_pass, &first, &count);
  return 2 * (size_t)count * sizeof(float);
}

pcc_status pcc_allpairs_to_host(const pcc_zdesc *zd, const void *z, float *r_host,
                                int64_t rows_per_pass, void *dev_buf, size_t dev_buf_bytes,
                                const pcc_tile_cfg *cfg, pcc_pass_fn on_pass, void *user,
                                void *compute_stream, void *copy_stream) {
  pcc_status s = check_zdesc(zd);
  if (s != PCC_OK) return s;
  if (zd->n < 2) return PCC_E_SHAPE;
  if (!z || !r_host || rows_per_pass < 1) return PCC_E_ARG;
  pcc_tile_cfg c;
  s = check_cfg(*zd, cfg, c);
  if (s != PCC_OK) return s;
  // a pass must be a whole number of bands to be a contiguous id range
  if (c.order == 1 && c.band > 1 && rows_per_pass % c.band != 0) return PCC_E_ARG;
  const size_t need = pcc_stream_buffer_bytes(zd, &c, rows_per_pass);
  if (!dev_buf || (reinterpret_cast<uintptr_t>(dev_buf) & 15) || dev_buf_bytes < need)
    return PCC_E_WORKSPACE;
  const int64_t n = zd->n, T = c.tile, m = (n + T - 1) / T;
  float *buf[2] = {(float *)dev_buf, (float *)dev_buf + need / 2 / sizeof(float)};
  hipStream_t cs = (hipStream_t)compute_stream, xs = (hipStream_t)copy_stream;
  const int grid = grid_for(*zd, c, kEpiPacked);

  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};  // K0 K1 C0 C1
  for (int k = 0; k < 4; ++k)
    if (note_hip(hipEventCreateWithFlags(&ev[k], hipEventDisableTiming)) != hipSuccess) {
      for (int q = 0; q < k; ++q) (void)hipEventDestroy(ev[q]);
      return PCC_E_HIP;
    }
  hipEvent_t *K = ev, *C = ev + 2;
  pcc_status rs = PCC_OK;
  int64_t prev_first = 0, prev_count = 0;
  bool have_prev = false;
  for (int64_t ya = 0, p = 0; ya < m && rs == PCC_OK; ya += rows_per_pass, ++p) {
    const int64_t yb = std::min(m, ya + rows_per_pass);
    const int b = (int)(p & 1);
    int64_t first = 0, count = 0;
    pass_slice(n, T, ya, yb, &first, &count);
    // buffer b is free once the copy of pass p - 2 has landed
    if (p >= 2 && note_hip(hipStreamWaitEvent(cs, C[b], 0)) != hipSuccess) rs = PCC_E_HIP;
    if (rs == PCC_OK &&
        (note_hip(launch_allpairs_range(*zd, z, buf[b], first, c, tri_F(m, ya), tri_F(m, yb), grid,
                                        cs)) != hipSuccess ||
         note_hip(hipEventRecord(K[b], cs)) != hipSuccess ||
         note_hip(hipStreamWaitEvent(xs, K[b], 0)) != hipSuccess ||
         (count > 0 && note_hip(hipMemcpyAsync(r_host + first, buf[b], (size_t)count * sizeof(float),
                                               hipMemcpyDeviceToHost, xs)) != hipSuccess) ||
         note_hip(hipEventRecord(C[b], xs)) != hipSuccess))
      rs = PCC_E_HIP;
    // host side of the previous pass, overlapped with this pass's kernel
    if (rs == PCC_OK && have_prev) {
      if (note_hip(hipEventSynchronize(C[1 - b])) != hipSuccess)
        rs = PCC_E_HIP;
      else if (on_pass && prev_count > 0)
        on_pass(prev_first, prev_count, user);
    }
    prev_first = first;
    prev_count = count;
    have_prev = true;
  }
  if (have_prev) {
    // the last pass (its buffer is the one recorded last)
    const int64_t passes = (m + rows_per_pass - 1) / rows_per_pass;
    const int b = (int)((passes - 1) & 1);
    if (note_hip(hipEventSynchronize(C[b])) != hipSuccess) {
      rs = PCC_E_HIP;
    } else if (rs == PCC_OK && on_pass && prev_count > 0) {
      on_pass(prev_first, prev_count, user);
    }
  }
  // drain both streams before the events go, also after an error
  if (note_hip(hipStreamSynchronize(xs)) != hipSuccess && rs == PCC_OK) rs = PCC_E_HIP;
  if (note_hip(hipStreamSynchronize(cs)) != hipSuccess && rs == PCC_OK) rs = PCC_E_HIP;
  for (int k = 0; k < 4; ++k) (void)hipEventDestroy(ev[k]);
  return rs;
}

pcc_status pcc_threshold_edges(const pcc_zdesc *zd, const void *z, float thr, int32_t *ij,
                               float *rv, int64_t cap, int64_t *count, const pcc_tile_cfg *cfg,
                               void *workspace, void *stream) {
  (void)workspace;
  pcc_status s = check_zdesc(zd);
  if (s != PCC_OK) return s;
  if (zd->n < 2) return PCC_E_SHAPE;  // no pair
  if (!z || !count || cap < 0 || (cap > 0 && (!ij || !rv))) return PCC_E_ARG;
  if (!(thr == thr)) return PCC_E_ARG;  // NaN threshold
  pcc_tile_cfg c;
  s = check_cfg(*zd, cfg, c);
  if (s != PCC_OK) return s;
  return hip_status(launch_edges(*zd, z, thr, ij, rv, cap, count, c, grid_for(*zd, c, kEpiEdges),
                                  (hipStream_t)stream));
}

// Both operands of a non-symmetric call: valid layouts, same mode and the
// same samples (so the same row layout).
static pcc_status check_xy(const pcc_zdesc *zdx, const void *zx, const pcc_zdesc *zdy,
                           const void *zy) {
  pcc_status s = check_zdesc(zdx);
  if (s != PCC_OK) return s;
  s = check_zdesc(zdy);
  if (s != PCC_OK) return s;
  if (zdx->mode != zdy->mode) return PCC_E_MODE;
  if (zdx->l != zdy->l) return PCC_E_SHAPE;
  if (!zx || !zy) return PCC_E_ARG;
  return PCC_OK;
}

pcc_status pcc_allpairs_xy(const pcc_zdesc *zdx, const void *zx, const pcc_zdesc *zdy,
                           const void *zy, float *r, int64_t ldr, const pcc_tile_cfg *cfg,
                           void *workspace, void *stream) {
  (void)workspace;
  pcc_status s = check_xy(zdx, zx, zdy, zy);
  if (s != PCC_OK) return s;
  if (!r) return PCC_E_ARG;
  if (ldr < zdy->n) return PCC_E_SHAPE;
  pcc_tile_cfg c;
  s = check_cfg(*zdx, cfg, c);
  if (s != PCC_OK) return s;
  return hip_status(launch_allpairs_xy(*zdx, zx, *zdy, zy, r, ldr, c,
                                       grid_for(*zdx, c, kEpiRect, zdy->n), (hipStream_t)stream));
}

pcc_status pcc_threshold_edges_xy(const pcc_zdesc *zdx, const void *zx, const pcc_zdesc *zdy,
                                  const void *zy, float thr, int32_t *ij, float *rv, int64_t cap,
                                  int64_t *count, const pcc_tile_cfg *cfg, void *workspace,
                                  void *stream) {
  (void)workspace;
  pcc_status s = check_xy(zdx, zx, zdy, zy);
  if (s != PCC_OK) return s;
  if (!count || cap < 0 || (cap > 0 && (!ij || !rv))) return PCC_E_ARG;
  if (!(thr == thr)) return PCC_E_ARG;
  pcc_tile_cfg c;
  s = check_cfg(*zdx, cfg, c);
  if (s != PCC_OK) return s;
  return hip_status(launch_edges_xy(*zdx, zx, *zdy, zy, thr, ij, rv, cap, count, c,
                                    grid_for(*zdx, c, kEpiRectEdges, zdy->n),
                                    (hipStream_t)stream));
}

pcc_status pcc_edges_status(int64_t count_host, int64_t cap) {
  if (count_host < 0 || cap < 0) return PCC_E_ARG;
  return count_host > cap ? PCC_E_CAPACITY : PCC_OK;
}

int64_t pcc_permtest_max_l(pcc_mode_t mode) { return permtest_max_l(mode); }

// Default schedule of the tiled permutation test: the all-pairs default,
// with 256-wide tiles whenever the copies of one launch give the grid a few
// rounds of them (one launch holds S copies' tiles).
static pcc_tile_cfg perm_default_cfg(const pcc_zdesc &zd) {
  pcc_tile_cfg c;
  pcc_default_cfg(&zd, &c);
  const int64_t S = permtest_slots(zd.n * (zd.n - 1) / 2);
  const int64_t m = (zd.n + 255) / 256;
  if (c.tile == 128 && S * (m * (m + 1) / 2) >= 4 * 256) {
    c.tile = 256;
    c.order = 1;
    c.band = 8;
  }
  return c;
}

pcc_status pcc_permtest(const pcc_zdesc *zd, const void *z, const int32_t *perms, int32_t P,
                        int32_t *counts, void *workspace, void *stream) {
  pcc_status s = check_zdesc(zd);
  if (s != PCC_OK) return s;
  if (zd->n < 2) return PCC_E_SHAPE;  // no pair
  if (!z || !counts || P < 0 || (P > 0 && !perms)) return PCC_E_ARG;
  if (permtest_max_l(zd->mode) <= 0) return PCC_E_MODE;
  const int cus = device_cus();
  if (zd->l_pad > permtest_max_l(zd->mode)) {
    // rows too long for the LDS kernel: the tiled form
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255)) return PCC_E_WORKSPACE;
    const pcc_tile_cfg c = perm_default_cfg(*zd);
    return hip_status(launch_permtest_tiles(*zd, z, perms, P, counts, workspace, c, cus,
                                            (hipStream_t)stream));
  }
  return hip_status(
      launch_permtest(*zd, z, perms, P, counts, cus > 0 ? cus : 256, (hipStream_t)stream));
}

pcc_status pcc_permtest_tiles(const pcc_zdesc *zd, const void *z, const int32_t *perms, int32_t P,
                              int32_t *counts, const pcc_tile_cfg *cfg, void *workspace,
                              size_t workspace_bytes, void *stream) {
  pcc_status s = check_zdesc(zd);
  if (s != PCC_OK) return s;
  if (zd->n < 2) return PCC_E_SHAPE;
  if (!z || !counts || P < 0 || (P > 0 && !perms)) return PCC_E_ARG;
  if (zd->mode != PCC_FP32 && zd->mode != PCC_SPLIT_BF16X3) return PCC_E_MODE;
  pcc_tile_cfg c = perm_default_cfg(*zd);
  if (cfg) {
    s = check_cfg(*zd, cfg, c);
    if (s != PCC_OK) return s;
  }
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255) ||
      workspace_bytes < permtest_tiles_workspace(*zd))
    return PCC_E_WORKSPACE;
  return hip_status(launch_permtest_tiles(*zd, z, perms, P, counts, workspace, c, device_cus(),
                                          (hipStream_t)stream));
}

int64_t pcc_job_of_cell(int64_t m, int64_t y, int64_t x) { return tri_F(m, y) + x - y; }

void pcc_cell_of_job(int64_t m, int64_t J, int64_t *y, int64_t *x) {
  const Cell c = tri_cell(m, J);
  if (y) *y = c.y;
  if (x) *x = c.x;
}

int64_t pcc_packed_index(int64_t n, int64_t y, int64_t x) { return packed_index(n, y, x); }

void pcc_packed_cell(int64_t n, int64_t Jp, int64_t *y, int64_t *x) {
  const Cell c = packed_cell(n, Jp);
  if (y) *y = c.y;
  if (x) *x = c.x;
}

pcc_status pcc_cells_host(int64_t m, int32_t diag, int64_t J0, int64_t count, int64_t *y,
                          int64_t *x) {
  if (count < 0 || (count > 0 && (!y || !x)) || m < 1 || J0 < 0) return PCC_E_ARG;
  const int64_t total = diag ? m * (m + 1) / 2 : m * (m - 1) / 2;
  if (J0 + count > total) return PCC_E_SHAPE;
  for (int64_t t = 0; t < count; ++t) {
    const Cell c = diag ? tri_cell(m, J0 + t) : packed_cell(m, J0 + t);
    y[t] = c.y;
    x[t] = c.x;
  }
  return PCC_OK;
}

pcc_status pcc_tile_order_host(int64_t m, const pcc_tile_cfg *cfg, int64_t J0, int64_t count,
                               int64_t *yt, int64_t *xt) {
  if (!cfg || count < 0 || (count > 0 && (!yt || !xt)) || m < 1 || J0 < 0) return PCC_E_ARG;
  if (cfg->order != 0 && cfg->order != 1) return PCC_E_ARG;
  if (cfg->order == 1 && cfg->band < 1) return PCC_E_ARG;
  if (J0 + count > m * (m + 1) / 2) return PCC_E_SHAPE;
  for (int64_t t = 0; t < count; ++t) {
    const Cell c = tile_of_job(m, cfg->order, cfg->band, J0 + t);
    yt[t] = c.y;
    xt[t] = c.x;
  }
  return PCC_OK;
}

pcc_status pcc_rect_tile_order_host(int64_t mr, int64_t mc, const pcc_tile_cfg *cfg, int64_t J0,
                                    int64_t count, int64_t *yt, int64_t *xt) {
  if (!cfg || count < 0 || (count > 0 && (!yt || !xt)) || mr < 1 || mc < 1 || J0 < 0)
    return PCC_E_ARG;
  if (cfg->order != 0 && cfg->order != 1) return PCC_E_ARG;
  if (cfg->order == 1 && cfg->band < 1) return PCC_E_ARG;
  if (J0 + count > mr * mc) return PCC_E_SHAPE;
  for (int64_t t = 0; t < count; ++t) {
    const Cell c = rect_cell(mr, mc, cfg->order, cfg->band, J0 + t);
    yt[t] = c.y;
    xt[t] = c.x;
  }
  return PCC_OK;
}

pcc_status pcc_cells_device(int64_t m, int32_t diag, int64_t J0, int64_t count, int64_t *y,
                            int64_t *x, void *stream) {
  if (count < 0 || (count > 0 && (!y || !x)) || m < 1 || J0 < 0) return PCC_E_ARG;
  const int64_t total = diag ? m * (m + 1) / 2 : m * (m - 1) / 2;
  if (J0 + count > total) return PCC_E_SHAPE;
  return hip_status(launch_cells(m, diag ? 1 : 0, J0, count, y, x, (hipStream_t)stream));
}

int32_t pcc_device_cus(void) { return device_cus(); }

int32_t pcc_autotune_default_count(void) { return (int32_t)default_candidates().size(); }

int32_t pcc_tile_arith(const pcc_zdesc *zd) {
  if (check_zdesc(zd) != PCC_OK) return -1;
  return arith_mode(*zd);
}

pcc_status pcc_autotune(const pcc_zdesc *zd, const void *z, float *r, const pcc_tile_cfg *cands,
                        int32_t ncands, int32_t reps, pcc_tile_cfg *best, float *times_ms,
                        void *stream) {
  pcc_status s = check_zdesc(zd);
  if (s != PCC_OK) return s;
  if (!z || !r || !best || reps < 1 || ncands < 0 || (ncands > 0 && !cands)) return PCC_E_ARG;
  std::vector<pcc_tile_cfg> list;
  if (ncands > 0)
    list.assign(cands, cands + ncands);
  else
    list = default_candidates();
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (note_hip(hipEventCreate(&e0)) != hipSuccess) return PCC_E_HIP;
  if (note_hip(hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return PCC_E_HIP;
  }
  float best_t = INFINITY;
  int best_i = -1;
  pcc_status rs = PCC_OK;
  for (size_t k = 0; k < list.size() && rs == PCC_OK; ++k) {
    pcc_tile_cfg c;
    if (check_cfg(*zd, &list[k], c) != PCC_OK) {
      if (times_ms) times_ms[k] = INFINITY;
      continue;
    }
    const int grid = grid_for(*zd, c, kEpiPacked);
    std::vector<float> ts;
    for (int rep = 0; rep <= reps && rs == PCC_OK; ++rep) {  // rep 0 warms up
      if (note_hip(hipEventRecord(e0, st)) != hipSuccess ||
          note_hip(launch_allpairs(*zd, z, r, c, grid, st)) != hipSuccess ||
          note_hip(hipEventRecord(e1, st)) != hipSuccess ||
          note_hip(hipEventSynchronize(e1)) != hipSuccess) {
        rs = PCC_E_HIP;
        break;
      }
      float ms = 0.f;
      if (note_hip(hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
        rs = PCC_E_HIP;
        break;
      }
      if (rep > 0) ts.push_back(ms);
    }
    if (rs != PCC_OK) break;
    std::sort(ts.begin(), ts.end());
    const float med = ts[ts.size() / 2];
    if (times_ms) times_ms[k] = med;
    if (med < best_t) {
      best_t = med;
      best_i = (int)k;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rs != PCC_OK) return rs;
  if (best_i < 0) return PCC_E_ARG;
  *best = list[best_i];
  return PCC_OK;
}

}  // extern "C"
