/*
 * pcc.h - all-pairs Pearson correlation on AMD Instinct MI355X (gfx950).
 *
 * The C ABI of libpcc.so.  Every argument is a plain pointer or integer;
 * device buffers are passed as device pointers, streams as hipStream_t cast
 * to void* (NULL means the default stream).  The caller owns every buffer.
 * No entry point allocates device memory while computing; the only device
 * allocations the library ever makes are the hipGraph objects of a batch
 * plan (pcc_batch_plan_create).  pcc_batch_run_noalloc uses a file-scope
 * device array of the library as its scratch.
 *
 * Method (Liu, Pan and Aluru, "Parallel pairwise correlation computation on
 * Intel Xeon Phi clusters"):
 *   Eq. (1)   r(u,v) = sum (u-ub)(v-vb) / sqrt(sum (u-ub)^2 * sum (v-vb)^2)
 *   Eq. (4)   U_i = (X_i - mean_i) / sqrt(sum_k (X_i[k] - mean_i)^2)
 *             (the square in the denominator restored as the variable
 *             transformation algorithm computes it)
 *   Eq. (5)   r(X_i, X_j) = U_i . U_j, so all pairs are A A^T with A = U,
 *             of which only the upper triangle is needed.
 *   Eq. (7)-(8)   non-symmetric all-pairs: job id J = y n + x over the whole
 *             job matrix (two different variable sets).
 *   Eq. (9)-(19)  direct bijective mapping between a job id and its
 *             upper-triangle cell, applied to t x t tiles (Sec. III-C).
 *
 * Conventions common to every entry point:
 *   - Calls are asynchronous on `stream`; results are valid after the
 *     stream has been synchronised.
 *   - Every argument error is detected on the host before anything is
 *     launched and returned as a pcc_status; nothing is launched then.
 *   - A HIP launch error is returned as PCC_E_HIP.  No C++ exception crosses
 *     this interface.
 *   - Calls on distinct streams are thread-safe.  Calls that share an output
 *     buffer race.
 *   - Degenerate profiles (zero sum of squared deviations, or a NaN/Inf
 *     sample) give r = NaN for every pair they are in.
 */
#ifndef PCC_H
#define PCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PCC_OK = 0,
  PCC_E_ARG = -1,        /* null pointer or bad scalar argument */
  PCC_E_SHAPE = -2,      /* n, l, ld or a size out of the supported range */
  PCC_E_MODE = -3,       /* unknown or unsupported precision mode */
  PCC_E_CAPACITY = -4,   /* reported by pcc_edges_status: edge list overflow */
  PCC_E_HIP = -5,        /* a HIP runtime call failed */
  PCC_E_WORKSPACE = -6,  /* workspace missing or too small */
  PCC_E_DEVICE = -7      /* no usable gfx950 device */
} pcc_status;

/* Element type of the input matrix X. */
typedef enum { PCC_IN_F32 = 0, PCC_IN_F64 = 1 } pcc_in_t;

/* Arithmetic of the tile contraction (FP32 accumulators on MFMA, except
 * PCC_FP64):
 *   PCC_FP32          z in FP32, v_mfma_f32_32x32x2_f32.
 *   PCC_SPLIT_BF16X3  z = hi + lo with hi = bf16(z), lo = bf16(z - hi);
 *                     r = hi.hi + hi.lo + lo.hi, v_mfma_f32_32x32x16_bf16.
 *                     Each product z_i[k] z_j[k] is then off by at most
 *                     3 * 2^-16 |z_i[k] z_j[k]|, so |dr| <= 3 * 2^-16 (about
 *                     4.6e-5) by Cauchy-Schwarz for any data.  On profiles of
 *                     continuous values the errors have random signs and
 *                     |dr| stays below 1e-5 once l > 64; rows of at most 64
 *                     samples are therefore computed in FP32 (pcc_tile_arith).
 *                     Profiles of a few repeated levels (binary data, say) make
 *                     the errors systematic: |dr| can reach about 1.1e-5 at any
 *                     l; use PCC_FP32 or PCC_FP64 for such data.
 *   PCC_BF16          z in BF16.
 *   PCC_FP16          z*sqrt(l) in FP16 (unit RMS entries), r = acc / l.
 *   PCC_FP64          z in FP64, FP64 accumulators, v_mfma_f64_16x16x4_f64:
 *                     the precision the paper computes in (its evaluation
 *                     uses double throughout).  128-wide tiles only. */
typedef enum {
  PCC_FP32 = 0,
  PCC_SPLIT_BF16X3 = 1,
  PCC_BF16 = 2,
  PCC_FP16 = 3,
  PCC_FP64 = 4
} pcc_mode_t;

/* Layout of the transformed matrix Z in device memory (written by
 * pcc_normalize, read by every other entry point).  Z is n_pad rows of
 * row_bytes bytes.  A row is a sequence of 128-byte chunks, each holding
 * kchunk consecutive samples:
 *   FP32:  32 floats;             BF16 / FP16: 64 halves;
 *   SPLIT: 32 bf16 hi values followed by the 32 matching bf16 lo values;
 *   FP64:  16 doubles.
 * Samples l..l_pad-1 and rows n..n_pad-1 are zero.  n_pad is a multiple of
 * 256 and l_pad a multiple of kchunk.
 * Exception: a SPLIT layout with l_pad <= 64 (rows of one or two chunks)
 * holds 32 FP32 values per chunk, exactly as the FP32 layout does, and its
 * tiles compute in FP32 (see pcc_tile_arith). */
typedef struct {
  int64_t n, l;          /* profiles and samples per profile */
  int64_t n_pad, l_pad;  /* padded sizes */
  int64_t row_bytes;     /* bytes of one Z row (l_pad / kchunk * 128) */
  int64_t bytes;         /* n_pad * row_bytes */
  int32_t mode;          /* pcc_mode_t */
  int32_t kchunk;        /* samples per 128-byte chunk */
} pcc_zdesc;

/* Tile schedule of the all-pairs kernels.
 *   tile:  256 or 128, the side t of one tile job (Sec. III-C); PCC_FP64
 *          supports 128 only.
 *   order: 0 = tile ids in the paper's order (row by row, Eq. (16)-(19));
 *          1 = banded order: the tile triangle is cut into bands of `band`
 *              tile rows; a band is walked column by column, so consecutive
 *              ids share row and column panels.  Both are bijections.
 *   grid:  persistent workgroups, 0 = one per compute unit times occupancy.
 * Identical results for every schedule (no split-K, no atomics on r): with
 * 256-wide FP32 tiles, a last round of the persistent grid that would leave
 * more than half of the workgroups idle is computed as 128-wide quarters,
 * which sum every pair's samples in the same order. */
typedef struct {
  int32_t tile;
  int32_t order;
  int32_t band;
  int32_t grid;
} pcc_tile_cfg;

/* Human-readable name of a status code (static string). */
const char *pcc_status_string(pcc_status s);

/* Library version as major*10000 + minor*100 + patch. */
int32_t pcc_version(void);

/* The hipError_t of the last HIP call that failed inside a pcc_* call on
 * the calling thread (0 if none has), and its name (static string).  It is
 * what a PCC_E_HIP result stands for; it is not reset by later successes. */
int32_t pcc_last_hip_error(void);
const char *pcc_last_hip_error_string(void);

/* Fill *out with the Z layout for n profiles of l samples in `mode`.
 * Host only, pure.  Requires 1 <= n <= 2^31-1 and 2 <= l <= 2^21 (a
 * 256-row panel of Z stays within 2 GiB, so tile loads use 32-bit offsets).
 * The symmetric entry points (all pairs of one set) need n >= 2 and return
 * PCC_E_SHAPE otherwise; one profile against a set is pcc_allpairs_xy. */
pcc_status pcc_z_layout(int64_t n, int64_t l, pcc_mode_t mode, pcc_zdesc *out);

/* Default tile schedule for a layout (host only, pure). */
pcc_status pcc_default_cfg(const pcc_zdesc *zd, pcc_tile_cfg *out);

/* Arithmetic the tile kernels use for a layout (host only, pure): zd->mode,
 * except PCC_FP32 for a PCC_SPLIT_BF16X3 layout with l_pad <= 64, whose rows
 * pcc_normalize writes in FP32 (over so few samples the split's per-product
 * errors do not average below 1e-5; Eq. (5) is then evaluated in FP32).
 * -1 for an invalid layout. */
int32_t pcc_tile_arith(const pcc_zdesc *zd);

/* Variable transformation, Eq. (4) and the variable transformation
 * algorithm (Sec. III-E).
 *   x      device, n rows of l samples, row pitch ldx elements (ldx >= l),
 *          element type xt.
 *   z      device, zd->bytes bytes, written in the layout of *zd, padding
 *          included.  Must not overlap x.
 *   stats  device, nullable: 2*n doubles, stats[2i] = mean of row i,
 *          stats[2i+1] = sum of squared deviations M2 (both FP64).
 *   n_degenerate  device int32, nullable: set to the number of rows with
 *          M2 == 0 or a non-finite M2; those rows of z are NaN.
 * Statistics are FP64 (two passes over the row, mean then M2); z is
 * (x - mean) / sqrt(M2) in FP64, then rounded to the mode's format. */
pcc_status pcc_normalize(const void *x, pcc_in_t xt, int64_t ldx,
                         const pcc_zdesc *zd, void *z, double *stats,
                         int32_t *n_degenerate, void *stream);

/* Bytes of device workspace an operation needs (0 for an invalid layout).
 * op 0 (pcc_allpairs), 1 (pcc_threshold_edges): 0 for every layout; the
 *   tile kernels keep their staging in LDS and registers and the edge
 *   counter is the caller's `count`, so their `workspace` arguments are
 *   unused and may be NULL (kept so that a future kernel needing scratch
 *   does not change the ABI).
 * op 2 (pcc_permtest): 0 while l_pad <= pcc_permtest_max_l(mode) (the LDS
 *   kernel, counts accumulate in LDS); for longer rows the size op 3 gives,
 *   since the call then runs the tiled form.
 * op 3 (pcc_permtest_tiles, FP32 and split layouts): the observed r
 *   (n(n-1)/2 floats), S column-permuted copies of Z (S * zd->bytes) and,
 *   when S > 1, S slots of int32 counts, S = min(32, max(1, 2^27 /
 *   (n(n-1)/2))); each part 256-byte aligned.  Independent of P and of the
 *   tile schedule.
 * (The uneven batch sizes its workspace with pcc_batch_workspace_size, the
 * multi-pass call its buffers with pcc_stream_buffer_bytes.) */
size_t pcc_workspace_size(const pcc_zdesc *zd, int32_t op);

/* All pairs (Sec. III-C, the tiled multithreaded kernel): tile jobs placed
 * by the bijection of Eq. (16)-(19), each tile of Z Z^T contracted on MFMA, and
 *   r[J'] = clamp(Z_y . Z_x, -1, 1)   for every 0 <= y < x < n,
 * with J' = F_{n-1}(y) + (x - 1) - y the strict-upper-triangle index (the
 * diagonal-free adaptation of Eq. (9)-(10)): row y of the triangle is
 * contiguous.  r: device, n(n-1)/2 floats.  cfg may be NULL (default). */
pcc_status pcc_allpairs(const pcc_zdesc *zd, const void *z, float *r,
                        const pcc_tile_cfg *cfg, void *workspace, void *stream);

/* As pcc_allpairs, for zd->mode == PCC_FP64 only, with r written in FP64:
 * r[J'] = clamp(Z_y . Z_x, -1, 1) as doubles (the paper's output
 * precision).  r: device, n(n-1)/2 doubles. */
pcc_status pcc_allpairs_f64(const pcc_zdesc *zd, const void *z, double *r,
                            const pcc_tile_cfg *cfg, void *workspace, void *stream);

/* ---- Multi-pass all pairs into host memory ------------------------------
 * For triangles larger than device memory, or results wanted on the host:
 * the multi-pass execution of Sec. III-C with the double buffering of the
 * asynchronous execution algorithm.  The tile-id range [0, m(m+1)/2) is cut
 * into passes of `rows_per_pass` whole tile rows (a multiple of cfg->band in
 * the banded order), so a pass covers the contiguous id range
 * [F_m(y_a), F_m(y_b)) (Eq. (17)) and its pairs are one contiguous slice of
 * the packed triangle.  Pass p is computed into device buffer p % 2 on
 * compute_stream, then copied by one asynchronous device-to-host copy on
 * copy_stream straight to its final place in r_host, while pass p + 1
 * computes into the other buffer.  After pass p's copy has landed,
 * on_pass(first, count, user) (nullable) is called on the calling thread
 * with the slice [first, first + count) of the packed triangle; meanwhile
 * the next pass computes (the host-side processing of the paper's loop).
 *
 *   r_host   host, n(n-1)/2 floats, the packed triangle as pcc_allpairs
 *            writes it.  Should be pinned (hipHostMalloc) for asynchronous
 *            copies.
 *   dev_buf  device, 16-byte aligned, at least pcc_stream_buffer_bytes(zd,
 *            cfg, rows_per_pass) bytes (two pass buffers); else
 *            PCC_E_WORKSPACE.
 * Blocking: returns after every pass has landed in r_host.  compute_stream
 * and copy_stream may be equal (no overlap then).  Creates and destroys
 * four HIP events per call; allocates no memory. */
typedef void (*pcc_pass_fn)(int64_t first, int64_t count, void *user);

size_t pcc_stream_buffer_bytes(const pcc_zdesc *zd, const pcc_tile_cfg *cfg,
                               int64_t rows_per_pass);

pcc_status pcc_allpairs_to_host(const pcc_zdesc *zd, const void *z, float *r_host,
                                int64_t rows_per_pass, void *dev_buf,
                                size_t dev_buf_bytes, const pcc_tile_cfg *cfg,
                                pcc_pass_fn on_pass, void *user,
                                void *compute_stream, void *copy_stream);

/* Thresholded edge list: the co-expression network construction that
 * motivates all-pairs correlation (Sec. I) keeps the pairs whose |r|
 * reaches a threshold.  Every pair y < x with |r| >= thr (r = Z_y . Z_x by
 * Eq. (5), clamped to the [-1, 1] that Eq. (1) bounds r to; NaN never
 * qualifies) is appended as ij[2s] = y,
 * ij[2s+1] = x, rv[s] = r for a slot s < cap.  *count (device int64) is
 * zeroed by the call and receives the true number of such pairs, which may
 * exceed cap (then only cap are stored: call again with a larger list).
 * The list is unordered.  ij, rv: device; cap >= 0. */
pcc_status pcc_threshold_edges(const pcc_zdesc *zd, const void *z, float thr,
                               int32_t *ij, float *rv, int64_t cap,
                               int64_t *count, const pcc_tile_cfg *cfg,
                               void *workspace, void *stream);

/* Host helper after pcc_threshold_edges has completed: PCC_OK if
 * count <= cap, PCC_E_CAPACITY otherwise (count read from host memory). */
pcc_status pcc_edges_status(int64_t count_host, int64_t cap);

/* Non-symmetric all pairs, Eq. (7)-(8): two variable sets X (nx profiles)
 * and Y (ny profiles) with the same number of samples, each transformed by
 * pcc_normalize in the same mode (zdx->l == zdy->l, zdx->mode == zdy->mode).
 * Every cell of the nx x ny job matrix is a job; tile jobs are numbered
 * J = yt mc + xt over the mx x mc tile rectangle (cfg->order 0) or in bands
 * of cfg->band tile rows walked column by column (order 1).
 *   r[y * ldr + x] = clamp(ZX_y . ZY_x, -1, 1)  for 0 <= y < nx, 0 <= x < ny
 * r: device, nx rows of pitch ldr >= ny floats (entries x >= ny untouched).
 * zx and zy may be the same buffer (then r is the full symmetric matrix,
 * diagonal included). */
pcc_status pcc_allpairs_xy(const pcc_zdesc *zdx, const void *zx, const pcc_zdesc *zdy,
                           const void *zy, float *r, int64_t ldr,
                           const pcc_tile_cfg *cfg, void *workspace, void *stream);

/* Thresholded edges of the non-symmetric job matrix: every (y, x) with
 * |r| >= thr, y indexing X and x indexing Y; otherwise as
 * pcc_threshold_edges (unordered, *count is the true total). */
pcc_status pcc_threshold_edges_xy(const pcc_zdesc *zdx, const void *zx,
                                  const pcc_zdesc *zdy, const void *zy, float thr,
                                  int32_t *ij, float *rv, int64_t cap, int64_t *count,
                                  const pcc_tile_cfg *cfg, void *workspace, void *stream);

/* Permutation test: the significance test by random permutations that the
 * evaluation (Sec. IV-A) motivates, at least 1,000 iterations of all-pairs
 * r on permuted data.
 * For every pair y < x (r by Eq. (5)):
 *   r_obs = Z_y . Z_x,  r_p = sum_k Z_y[k] Z_x[perm_p[k]],
 *   counts[J'] = #{p : |r_p| >= |r_obs|}  (ties counted; -1 if r_obs is NaN)
 * The second operand (column x) is permuted; Z's mean and norm are
 * invariant under a permutation, so Z is not renormalised.
 * Rows of l_pad <= pcc_permtest_max_l(mode): one persistent launch for all
 * P permutations, with the permuted profiles of a job in LDS for every
 * sample; `workspace` is unused (may be NULL).  FP32 jobs are 32 x 32 pair
 * blocks with both profile panels in LDS (l_pad <= 608 on gfx950's 160 KiB);
 * split jobs are 64 x 32 blocks whose 64 unpermuted profiles are streamed
 * through LDS (l_pad <= 992).
 * Longer rows: the tiled form of pcc_permtest_tiles with the default
 * schedule; `workspace` must hold pcc_workspace_size(zd, 2) bytes and be
 * 256-byte aligned (NULL or misaligned gives PCC_E_WORKSPACE).
 *   perms  device int32, P rows of l entries, each a permutation of 0..l-1.
 *          Not checked on the device: an entry outside [0, l) reads other
 *          data of the job (LDS of the workgroup, or the row of Z in the
 *          tiled form), so its counts are meaningless.  The Python binding
 *          checks them.
 *   counts device int32, n(n-1)/2.
 * Supported modes: FP32 (FP32 MFMA; every r within about 1e-7 of exact) and
 * split-BF16x3 (three BF16 products per sample, about 3x the FP32 kernel's
 * rate; r within split's 1e-5, so a count can differ from the exact one only
 * in permutations whose |r| lies that close to |r_obs|).  The plain 16-bit
 * modes are refused: their r error (1e-4 and more) would decide too many
 * counts. */
pcc_status pcc_permtest(const pcc_zdesc *zd, const void *z,
                        const int32_t *perms, int32_t P, int32_t *counts,
                        void *workspace, void *stream);

/* The permutation test on the all-pairs tiles, for rows of any length
 * (Sec. IV-A's test on profiles of thousands of samples, as in the
 * evaluation's data sets).  The observed r is computed first by the
 * all-pairs tile kernel on schedule cfg (NULL: the all-pairs default, with
 * 256-wide tiles when the S copies of a launch fill the grid with them) into the
 * workspace.  Then, per group of S permutations, S column-permuted copies
 * of Z are gathered into the workspace and one launch runs the tiles of the
 * upper triangle of Z against every copy with the same tile core, adding
 * |r_p| >= |r_obs| to that copy's count slot; the slots are summed at the
 * end.  An identity permutation reproduces r_obs bit for bit, so it counts.
 * counts as for pcc_permtest; the r of a pair is the all-pairs kernel's on
 * this schedule (the LDS kernels round in another order, so counts of the
 * two forms can differ where some |r_p| lies within rounding of |r_obs|).
 * workspace: device, 256-byte aligned, workspace_bytes >=
 * pcc_workspace_size(zd, 3), else PCC_E_WORKSPACE.  Modes as pcc_permtest. */
pcc_status pcc_permtest_tiles(const pcc_zdesc *zd, const void *z, const int32_t *perms,
                              int32_t P, int32_t *counts, const pcc_tile_cfg *cfg,
                              void *workspace, size_t workspace_bytes, void *stream);

/* Largest l_pad of the LDS form of pcc_permtest (its job's permuted
 * profiles and, in FP32, the other panel too stay in LDS): 608 in FP32 and
 * 992 in split on gfx950.  Longer rows take the tiled form.  0 for modes the
 * permutation test does not support. */
int64_t pcc_permtest_max_l(pcc_mode_t mode);

/* ---- Uneven batches -----------------------------------------------------
 * One item per dataset.  The plan uploads a descriptor table into the
 * caller's workspace and records, into one hipGraph, a counter reset and
 * one persistent kernel: its workgroups first transform every dataset
 * (Eq. (4)), drawing row groups from a device counter, then draw tile jobs
 * from a second device counter over the concatenated job space (dynamic
 * distribution with a shared integer counter, Sec. III-B).  Between the two
 * phases a workgroup waits until every row group is done; the wait needs
 * no co-residency of the grid (only running workgroups claim row groups) and
 * is bounded.  Launching the plan replays the graph on a stream. */
typedef struct {
  const void *x;      /* device input, n x l, pitch ldx, type xt */
  int64_t ldx;
  int64_t n, l;
  int32_t xt;         /* pcc_in_t */
  int32_t tile;       /* 256 or 128, 0 = library default for (n, l) */
  void *z;            /* device, pcc_z_layout(n, l, mode).bytes bytes */
  float *r;           /* device, n(n-1)/2 floats */
} pcc_batch_item;

typedef struct pcc_batch_plan pcc_batch_plan;

/* Workspace bytes a batch of D items needs (the workspace must be 256-byte
 * aligned; pcc_batch_plan_create gives PCC_E_WORKSPACE otherwise). */
size_t pcc_batch_workspace_size(int32_t D);

/* Build a plan (host work + one synchronous upload of the descriptor table
 * on `stream`).  Items must stay valid for the plan's life; all items use
 * `mode` (PCC_FP32, PCC_SPLIT_BF16X3, PCC_BF16 or PCC_FP16; PCC_FP64 gives
 * PCC_E_MODE) and have n >= 2. */
pcc_status pcc_batch_plan_create(int32_t D, const pcc_batch_item *items,
                                 pcc_mode_t mode, void *workspace,
                                 size_t workspace_bytes, void *stream,
                                 pcc_batch_plan **plan);
/* Replay the plan's graph on `stream` (asynchronous).  The plan's job
 * counters live in its workspace and every launch resets and consumes them:
 * a plan may have at most one launch in flight.  Launches of one plan on one
 * stream are ordered and safe; launching it again on another stream first
 * requires that stream to wait for the previous launch (an event), otherwise
 * the two launches race on the counters and tiles are skipped or computed
 * twice.  Distinct plans (distinct workspaces) may run concurrently. */
pcc_status pcc_batch_plan_launch(pcc_batch_plan *plan, void *stream);
/* Total tile jobs of the plan (for accounting). */
int64_t pcc_batch_plan_jobs(const pcc_batch_plan *plan);
pcc_status pcc_batch_plan_destroy(pcc_batch_plan *plan);

/* Most datasets one pcc_batch_run_noalloc call takes. */
#define PCC_BATCH_NOALLOC_MAX_D 256

/* The uneven batch of a plan, run directly, with no allocation at all: for
 * callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Computes exactly
 * what a plan of the same items and mode computes when launched (same
 * kernels, same job order: bit-identical z and r), asynchronously on
 * `stream`, without creating a graph or a workspace.
 *   items  as for pcc_batch_plan_create; the caller passes every input and
 *          output buffer.  Need only stay valid until the call returns (the
 *          descriptors travel as kernel arguments).
 *   D      1 <= D <= PCC_BATCH_NOALLOC_MAX_D; a larger D gives PCC_E_SHAPE.
 * Scratch: the descriptor table and the job counters live in a file-scope
 * device array of the library (about 39 KB; each GPU the library runs on
 * holds its own copy until the process ends).  Its address is looked up on
 * the first call on a device, so make that first call outside stream
 * capture.  Every call on one GPU shares that array and rewrites it (the
 * counters are zeroed by a kernel, not by a memset): calls that overlap on
 * one GPU (two streams, two threads, two captured graphs replayed at once)
 * race and may skip or repeat tiles, so order them (one stream, or events).
 * Launches kernels only: no hipMalloc, hipFree, memcpy or memset, so the
 * call can be recorded under stream capture.  Errors: PCC_E_ARG / _MODE /
 * _SHAPE for the arguments (nothing launched), PCC_E_HIP for a failed
 * launch. */
pcc_status pcc_batch_run_noalloc(int32_t D, const pcc_batch_item *items, pcc_mode_t mode,
                                 void *stream);

/* ---- Job maps, host side, for tests and tooling -------------------------
 * Inclusive map over an m x m triangle (diagonal counted in), Eq. (9)-(15):
 * J = F_m(y) + x - y with F_m(y) = y(2m - y + 1)/2; inverse by Eq. (14)-(15)
 * evaluated in FP64, then corrected in int64 so that F_m(y) <= J < F_m(y+1)
 * holds exactly. */
int64_t pcc_job_of_cell(int64_t m, int64_t y, int64_t x);
void pcc_cell_of_job(int64_t m, int64_t J, int64_t *y, int64_t *x);
/* Exclusive (strict upper) map over n profiles: J' = F_{n-1}(y) + x-1-y. */
int64_t pcc_packed_index(int64_t n, int64_t y, int64_t x);
void pcc_packed_cell(int64_t n, int64_t Jp, int64_t *y, int64_t *x);
/* Vector forms: cells of `count` ids starting at J0 (host arrays).
 * diag != 0: inclusive map over m; diag == 0: exclusive map over m. */
pcc_status pcc_cells_host(int64_t m, int32_t diag, int64_t J0, int64_t count,
                          int64_t *y, int64_t *x);
/* Tile order of a schedule: the tile cell of `count` consecutive job ids
 * starting at J0 under cfg->order/cfg->band over an m x m tile triangle. */
pcc_status pcc_tile_order_host(int64_t m, const pcc_tile_cfg *cfg, int64_t J0,
                               int64_t count, int64_t *yt, int64_t *xt);
/* Tile order of a non-symmetric schedule over an mr x mc tile rectangle
 * (Eq. (7)-(8) for order 0, bands of cfg->band tile rows for order 1). */
pcc_status pcc_rect_tile_order_host(int64_t mr, int64_t mc, const pcc_tile_cfg *cfg,
                                    int64_t J0, int64_t count, int64_t *yt, int64_t *xt);
/* Device form of pcc_cells_host, computed by the same device code the tile
 * kernels use; y and x are device arrays of `count` entries. */
pcc_status pcc_cells_device(int64_t m, int32_t diag, int64_t J0, int64_t count,
                            int64_t *y, int64_t *x, void *stream);

/* ---- Autotuning ---------------------------------------------------------
 * Time each candidate schedule of pcc_allpairs on the caller's z (r is
 * overwritten) with hipEvents and return the fastest in *best.  `cands`
 * may be NULL with ncands == 0: the built-in list of
 * pcc_autotune_default_count() candidates (both tile sizes, the paper's row
 * order and bands of 2, 4, 8 and 16 tile rows).  times_ms (host, nullable)
 * gets the median time of every candidate timed: ncands entries, or
 * pcc_autotune_default_count() entries for the built-in list, so it must
 * hold max(ncands, pcc_autotune_default_count()) floats to be safe. */
pcc_status pcc_autotune(const pcc_zdesc *zd, const void *z, float *r,
                        const pcc_tile_cfg *cands, int32_t ncands,
                        int32_t reps, pcc_tile_cfg *best, float *times_ms,
                        void *stream);

/* Number of candidates in pcc_autotune's built-in list. */
int32_t pcc_autotune_default_count(void);

/* Number of compute units of the current device (0 if none). */
int32_t pcc_device_cus(void);

#ifdef __cplusplus
}
#endif
#endif /* PCC_H */
