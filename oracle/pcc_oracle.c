/*
 * FP64 CPU oracle for all-pairs Pearson correlation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or helper with the
 * HIP path.
 *
 * Every function is the plain definition, written out, in double precision:
 *   - pair values follow Eq. (1) literally: both means are recomputed for
 *     every pair, then the three centred sums, then the quotient;
 *   - the variable transformation follows Eq. (4) with the square restored
 *     in the denominator (as the variable-transformation algorithm computes
 *     it): mean, sum of squared deviations, reciprocal square root, scaled
 *     deviations;
 *   - non-symmetric all-pairs (two variable sets, Sec. III-B) is Eq. (1)
 *     for every cell of the nx x ny job matrix, row by row;
 *   - job numbering follows the symmetric all-pairs framework (Sec. III-B):
 *     upper-triangle cells numbered left to right, top to bottom, by
 *     counting, never by the closed-form map;
 *   - the permutation test counts permutations whose |r| is at least the
 *     observed |r| (evaluation section: permutation tests for significance).
 *
 * Readings where the paper is silent: a pair with a zero (or non-finite)
 * sum of squared deviations has r = NaN; r is clamped to [-1, 1] (Eq. (1)
 * bounds it there) with NaN kept; the diagonal is excluded from pair output.
 *
 * OpenMP only distributes independent pairs over threads; the arithmetic of
 * each pair is sequential and identical to a single-threaded run.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

static double clamp_unit(double r) {
  if (r > 1.0) return 1.0;
  if (r < -1.0) return -1.0;
  return r; /* NaN passes through: both comparisons are false */
}

/* Eq. (1), literally, for two rows of length l. */
static double pearson_literal(const double *u, const double *v, int64_t l) {
  double su = 0.0, sv = 0.0;
  for (int64_t k = 0; k < l; ++k) {
    su += u[k];
    sv += v[k];
  }
  const double mu = su / (double)l;
  const double mv = sv / (double)l;
  double sxy = 0.0, sxx = 0.0, syy = 0.0;
  for (int64_t k = 0; k < l; ++k) {
    const double du = u[k] - mu;
    const double dv = v[k] - mv;
    sxy += du * dv;
    sxx += du * du;
    syy += dv * dv;
  }
  if (!(sxx > 0.0) || !(syy > 0.0)) return NAN; /* zero or NaN spread */
  return clamp_unit(sxy / sqrt(sxx * syy));
}

/* Every pair i < j of the n rows of X (row pitch ld), written to out[] in
 * the order i = 0..n-1, j = i+1..n-1 (the strict upper triangle, row by row).
 * The start of each row of out[] is found by counting, not by a formula. */
int oracle_pearson_packed(const double *X, int64_t n, int64_t l, int64_t ld,
                          double *out) {
  if (!X || !out || n < 0 || l < 1 || ld < l) return -1;
  int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!start) return -2;
  int64_t c = 0;
  for (int64_t i = 0; i < n; ++i) {
    start[i] = c;
    for (int64_t j = i + 1; j < n; ++j) ++c;
  }
  start[n] = c;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i) {
    int64_t t = start[i];
    for (int64_t j = i + 1; j < n; ++j) out[t++] = pearson_literal(X + i * ld, X + j * ld, l);
  }
  free(start);
  return 0;
}

/* Non-symmetric all-pairs (Sec. III-B): r of row i of X (nx rows, pitch
 * ldx) and row j of Y (ny rows, pitch ldy), both of l samples, written to
 * out[i * ny + j] for every i and j (the whole job matrix, row by row). */
int oracle_pearson_xy(const double *X, int64_t nx, int64_t ldx, const double *Y, int64_t ny,
                      int64_t ldy, int64_t l, double *out) {
  if (!X || !Y || !out || nx < 0 || ny < 0 || l < 1 || ldx < l || ldy < l) return -1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < nx; ++i)
    for (int64_t j = 0; j < ny; ++j) out[i * ny + j] = pearson_literal(X + i * ldx, Y + j * ldy, l);
  return 0;
}

/* r for an explicit list of pairs (any order of i and j, i == j allowed). */
int oracle_pearson_pairs(const double *X, int64_t n, int64_t l, int64_t ld,
                         const int64_t *I, const int64_t *J, int64_t np,
                         double *out) {
  if (!X || !I || !J || !out || l < 1 || ld < l) return -1;
  for (int64_t p = 0; p < np; ++p)
    if (I[p] < 0 || I[p] >= n || J[p] < 0 || J[p] >= n) return -3;
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t p = 0; p < np; ++p) out[p] = pearson_literal(X + I[p] * ld, X + J[p] * ld, l);
  return 0;
}

/* Eq. (4) with the squared deviations in the denominator, row by row:
 * mean, sum of squared deviations M2, then U = (X - mean) / sqrt(M2).
 * A row with M2 == 0 (or non-finite) gets U = NaN. */
int oracle_transform(const double *X, int64_t n, int64_t l, int64_t ld,
                     double *U, double *mean, double *m2) {
  if (!X || l < 1 || ld < l) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const double *x = X + i * ld;
    double s = 0.0;
    for (int64_t k = 0; k < l; ++k) s += x[k];
    const double mu = s / (double)l;
    double q = 0.0;
    for (int64_t k = 0; k < l; ++k) q += (x[k] - mu) * (x[k] - mu);
    if (mean) mean[i] = mu;
    if (m2) m2[i] = q;
    if (U) {
      const double d = sqrt(q);
      for (int64_t k = 0; k < l; ++k) U[i * l + k] = (q > 0.0) ? (x[k] - mu) / d : NAN;
    }
  }
  return 0;
}

/* All pairs i < j with |r| >= thr, found by scanning every pair; written in
 * (i, j) order.  Returns the true number of such pairs (may exceed cap). */
int64_t oracle_edges(const double *X, int64_t n, int64_t l, int64_t ld,
                     double thr, int64_t cap, int64_t *EI, int64_t *EJ,
                     double *ER) {
  if (!X || l < 1 || ld < l) return -1;
  int64_t found = 0;
  for (int64_t i = 0; i < n; ++i) {
    double *row = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!row) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t j = i + 1; j < n; ++j) row[j] = pearson_literal(X + i * ld, X + j * ld, l);
    for (int64_t j = i + 1; j < n; ++j) {
      if (fabs(row[j]) >= thr) { /* false for NaN */
        if (found < cap) {
          EI[found] = i;
          EJ[found] = j;
          ER[found] = row[j];
        }
        ++found;
      }
    }
    free(row);
  }
  return found;
}

/* Permutation test on listed pairs (i, j): the second row is permuted.
 * perms holds P permutations of 0..l-1 (row p: position k takes sample
 * perms[p*l + k]).  counts[q] = #{p : |r_p| >= |r_obs|}, or -1 when r_obs is
 * NaN; gap[q] = min_p | |r_p| - |r_obs| | (how close the nearest decision
 * was), NaN when r_obs is NaN.  With c_lo and c_hi (nullable), the counts a
 * computation whose |r| values are each off by less than band/2 can reach:
 * c_lo[q] = #{p : |r_p| >= |r_obs| + band}, c_hi[q] = #{p : |r_p| >= |r_obs| -
 * band} (-1 both when r_obs is NaN). */
int oracle_permcounts(const double *X, int64_t n, int64_t l, int64_t ld,
                      const int32_t *perms, int32_t P, const int64_t *I,
                      const int64_t *J, int64_t np, int32_t *counts,
                      double *gap, double band, int32_t *c_lo, int32_t *c_hi) {
  if (!X || !perms || !I || !J || !counts || l < 1 || ld < l || P < 0) return -1;
  for (int64_t q = 0; q < np; ++q)
    if (I[q] < 0 || I[q] >= n || J[q] < 0 || J[q] >= n) return -3;
  for (int64_t t = 0; t < (int64_t)P * l; ++t)
    if (perms[t] < 0 || perms[t] >= l) return -4;
  int bad = 0;
#pragma omp parallel
  {
    double *tmp = (double *)malloc(sizeof(double) * (size_t)l);
    if (!tmp) {
#pragma omp atomic write
      bad = 1;
    }
#pragma omp for schedule(dynamic, 16)
    for (int64_t q = 0; q < np; ++q) {
      if (!tmp) continue;
      const double *u = X + I[q] * ld;
      const double *v = X + J[q] * ld;
      const double robs = pearson_literal(u, v, l);
      if (isnan(robs)) {
        counts[q] = -1;
        if (gap) gap[q] = NAN;
        if (c_lo) c_lo[q] = -1;
        if (c_hi) c_hi[q] = -1;
        continue;
      }
      const double aobs = fabs(robs);
      int32_t c = 0, lo = 0, hi = 0;
      double g = INFINITY;
      for (int32_t p = 0; p < P; ++p) {
        const int32_t *pi = perms + (int64_t)p * l;
        for (int64_t k = 0; k < l; ++k) tmp[k] = v[pi[k]];
        const double ap = fabs(pearson_literal(u, tmp, l));
        if (ap >= aobs) ++c;
        if (ap >= aobs + band) ++lo;
        if (ap >= aobs - band) ++hi;
        const double d = fabs(ap - aobs);
        if (d < g) g = d;
      }
      counts[q] = c;
      if (gap) gap[q] = g;
      if (c_lo) c_lo[q] = lo;
      if (c_hi) c_hi[q] = hi;
    }
    free(tmp);
  }
  return bad ? -2 : 0;
}

/* Sequential numbering of the upper triangle of an n x n job matrix
 * (Sec. III-B): ids 0, 1, 2, ... assigned left to right, top to bottom.
 * diag != 0 counts the major diagonal in (cells y <= x), diag == 0 leaves it
 * out (cells y < x).  ys/xs receive the cell of every id.  Returns the count. */
int64_t oracle_enumerate_upper(int64_t n, int32_t diag, int64_t *ys, int64_t *xs) {
  int64_t id = 0;
  for (int64_t y = 0; y < n; ++y) {
    for (int64_t x = diag ? y : y + 1; x < n; ++x) {
      if (ys) ys[id] = y;
      if (xs) xs[id] = x;
      ++id;
    }
  }
  return id;
}
