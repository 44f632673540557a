/* Reference CPU implementation of the exact 2D least-median-of-squares line.
 *
 * TEST INFRASTRUCTURE ONLY: see lms_oracle.h. Plain, slow and meant to be
 * checked by eye against the paper:
 *
 *   1. For every pair of points with different x, take the pair's slope
 *      theta = (y_j - y_i) / (x_j - x_i). In the dual plane this is the
 *      u-coordinate of the intersection of the two dual lines (Section 3.2),
 *      and equioscillation (Section 3.3) says one end of the optimal bracelet
 *      sits on such an intersection.
 *   2. At that slope, evaluate every point's intercept z_k = y_k - theta*x_k.
 *      This is the dual lines' vertical intersections, negated (Algorithm 1,
 *      the loop over intersection points).
 *   3. Sort the z_k and find the narrowest window of h consecutive values: the
 *      shortest bracelet cut by h dual lines at this slope (Section 3.2), i.e.
 *      the thinnest slab at this slope holding h points (Section 3.1).
 *   4. Keep the minimum over all pairs (Algorithm 1, the final reduction) and
 *      return the slab's bisector and half-height (Section 3.1).
 *
 * Step 3 takes the best window at each slope instead of the single bracelet
 * hanging from the vertex at a fixed rank offset. Both searches reach the same
 * minimum, and the windowed form needs no reading of which tied rank the
 * vertex occupies.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math).
 */
#include "lms_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int cmp_f64(const void* a, const void* b) {
  const double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* Intercepts at slope theta, sorted ascending, into z[0..n). */
static void sorted_intercepts(const double* xy, int64_t n, double theta, double* z) {
  for (int64_t k = 0; k < n; ++k) z[k] = fma(-theta, xy[2 * k], xy[2 * k + 1]);
  qsort(z, (size_t)n, sizeof(double), cmp_f64);
}

/* Narrowest window of h consecutive sorted values; the lowest one on ties. */
static void narrowest_window(const double* z, int64_t n, int64_t h, double* width,
                             double* z_lo, double* z_hi) {
  int64_t best_s = 0;
  double best = z[h - 1] - z[0];
  for (int64_t s = 1; s + h <= n; ++s) {
    const double w = z[s + h - 1] - z[s];
    if (w < best) {
      best = w;
      best_s = s;
    }
  }
  *width = best;
  *z_lo = z[best_s];
  *z_hi = z[best_s + h - 1];
}

static int check_args(const double* xy, int64_t n, int64_t* h) {
  if (!xy || n < 2) return LMS_ORACLE_ERR_ARG;
  if (*h == 0) *h = n / 2 + 1;
  if (*h < 2 || *h > n) return LMS_ORACLE_ERR_ARG;
  for (int64_t k = 0; k < 2 * n; ++k)
    if (!isfinite(xy[k])) return LMS_ORACLE_ERR_NONFINITE;
  return LMS_ORACLE_OK;
}

typedef struct {
  double width, theta, z_lo, z_hi;
  int64_t i, j;
} best_t;

/* Canonical order of candidate results: (width, theta, z_lo), then (i, j). */
static int better(const best_t* a, const best_t* b) {
  if (a->width != b->width) return a->width < b->width;
  if (a->theta != b->theta) return a->theta < b->theta;
  if (a->z_lo != b->z_lo) return a->z_lo < b->z_lo;
  if (a->i != b->i) return a->i < b->i;
  return a->j < b->j;
}

int lms_oracle_solve(const double* xy, int64_t n, int64_t h, int nthreads,
                     lms_oracle_result* out) {
  if (!out) return LMS_ORACLE_ERR_ARG;
  memset(out, 0, sizeof(*out));
  out->theta1 = out->theta2 = out->half_width = out->width = NAN;
  out->z_lo = out->z_hi = NAN;
  out->pair_i = out->pair_j = -1;
  int st = check_args(xy, n, &h);
  out->status = st;
  out->h = (int32_t)h;
  if (st != LMS_ORACLE_OK) return st;

  int all_x_equal = 1;
  for (int64_t k = 1; k < n; ++k)
    if (xy[2 * k] != xy[0]) all_x_equal = 0;

  best_t best = {INFINITY, 0.0, 0.0, 0.0, -1, -1};
  int64_t candidates = 0, vertical = 0;

  if (all_x_equal) {
    /* No pair has a finite slope. Any slope gives the same slab height,
     * since every residual moves by the same amount; take theta1 = 0 and
     * the narrowest window of the y values. */
    double* z = (double*)malloc((size_t)n * sizeof(double));
    sorted_intercepts(xy, n, 0.0, z);
    narrowest_window(z, n, h, &best.width, &best.z_lo, &best.z_hi);
    free(z);
    best.theta = 0.0;
    vertical = n * (n - 1) / 2;
    out->status = st = LMS_ORACLE_OK_DEGENERATE;
  } else {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel reduction(+ : candidates, vertical)
    {
      double* z = (double*)malloc((size_t)n * sizeof(double));
      best_t mine = {INFINITY, 0.0, 0.0, 0.0, -1, -1};
#pragma omp for schedule(dynamic, 1)
      for (int64_t i = 0; i < n - 1; ++i) {
        for (int64_t j = i + 1; j < n; ++j) {
          const double dx = xy[2 * j] - xy[2 * i];
          if (xy[2 * j] == xy[2 * i]) {
            ++vertical;
            continue;
          }
          ++candidates;
          best_t c;
          c.theta = (xy[2 * j + 1] - xy[2 * i + 1]) / dx;
          c.i = i;
          c.j = j;
          sorted_intercepts(xy, n, c.theta, z);
          narrowest_window(z, n, h, &c.width, &c.z_lo, &c.z_hi);
          if (better(&c, &mine)) mine = c;
        }
      }
#pragma omp critical
      {
        if (better(&mine, &best)) best = mine;
      }
      free(z);
    }
  }

  out->theta1 = best.theta;
  out->theta2 = 0.5 * (best.z_lo + best.z_hi);
  out->width = best.width;
  out->half_width = 0.5 * best.width;
  out->z_lo = best.z_lo;
  out->z_hi = best.z_hi;
  out->pair_i = best.i;
  out->pair_j = best.j;
  out->candidates = candidates;
  out->vertical = vertical;
  return st;
}

int lms_oracle_window(const double* xy, int64_t n, int64_t h, double theta,
                      double* width, double* z_lo, double* z_hi) {
  int st = check_args(xy, n, &h);
  if (st != LMS_ORACLE_OK) return st;
  double* z = (double*)malloc((size_t)n * sizeof(double));
  double w, lo, hi;
  sorted_intercepts(xy, n, theta, z);
  narrowest_window(z, n, h, &w, &lo, &hi);
  free(z);
  if (width) *width = w;
  if (z_lo) *z_lo = lo;
  if (z_hi) *z_hi = hi;
  return LMS_ORACLE_OK;
}

int lms_oracle_eval_pairs(const double* xy, int64_t n, int64_t h,
                          const int64_t* pairs, int64_t m, int nthreads,
                          double* theta, double* width, double* z_lo, double* z_hi) {
  int st = check_args(xy, n, &h);
  if (st != LMS_ORACLE_OK) return st;
  if (m < 0 || (m > 0 && !pairs)) return LMS_ORACLE_ERR_ARG;
  for (int64_t t = 0; t < m; ++t)
    if (pairs[2 * t] < 0 || pairs[2 * t] >= n || pairs[2 * t + 1] < 0 ||
        pairs[2 * t + 1] >= n || pairs[2 * t] == pairs[2 * t + 1])
      return LMS_ORACLE_ERR_ARG;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    double* z = (double*)malloc((size_t)n * sizeof(double));
#pragma omp for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; ++t) {
      int64_t i = pairs[2 * t], j = pairs[2 * t + 1];
      if (i > j) {
        const int64_t s = i;
        i = j;
        j = s;
      }
      double th = NAN, w = INFINITY, lo = NAN, hi = NAN;
      if (xy[2 * j] != xy[2 * i]) {
        th = (xy[2 * j + 1] - xy[2 * i + 1]) / (xy[2 * j] - xy[2 * i]);
        sorted_intercepts(xy, n, th, z);
        narrowest_window(z, n, h, &w, &lo, &hi);
      }
      if (theta) theta[t] = th;
      if (width) width[t] = w;
      if (z_lo) z_lo[t] = lo;
      if (z_hi) z_hi[t] = hi;
    }
    free(z);
  }
  return LMS_ORACLE_OK;
}

int lms_oracle_anchored(const double* xy, int64_t n, int64_t h, int64_t i, int64_t j,
                        double* up, double* dn) {
  int st = check_args(xy, n, &h);
  if (st != LMS_ORACLE_OK) return st;
  if (i < 0 || j < 0 || i >= n || j >= n || i == j || !up || !dn) return LMS_ORACLE_ERR_ARG;
  if (i > j) {
    const int64_t s = i;
    i = j;
    j = s;
  }
  *up = *dn = INFINITY;
  if (xy[2 * i] == xy[2 * j]) return LMS_ORACLE_OK;
  const double theta = (xy[2 * j + 1] - xy[2 * i + 1]) / (xy[2 * j] - xy[2 * i]);
  const double c = fma(-theta, xy[2 * i], xy[2 * i + 1]);
  double* a = (double*)malloc((size_t)n * sizeof(double));
  double* b = (double*)malloc((size_t)n * sizeof(double));
  int64_t na = 0, nb = 0;
  for (int64_t k = 0; k < n; ++k) {
    const double d = (k == i || k == j) ? 0.0 : fma(-theta, xy[2 * k], xy[2 * k + 1]) - c;
    if (d >= 0.0) a[na++] = d;
    if (d <= 0.0) b[nb++] = -d;
  }
  qsort(a, (size_t)na, sizeof(double), cmp_f64);
  qsort(b, (size_t)nb, sizeof(double), cmp_f64);
  if (na >= h) *up = a[h - 1];
  if (nb >= h) *dn = b[h - 1];
  free(a);
  free(b);
  return LMS_ORACLE_OK;
}

double lms_oracle_hth_abs_residual(const double* xy, int64_t n, int64_t h,
                                   double theta1, double theta2) {
  if (check_args(xy, n, &h) != LMS_ORACLE_OK) return NAN;
  double* r = (double*)malloc((size_t)n * sizeof(double));
  for (int64_t k = 0; k < n; ++k) r[k] = fabs(fma(-theta1, xy[2 * k], xy[2 * k + 1]) - theta2);
  qsort(r, (size_t)n, sizeof(double), cmp_f64);
  const double v = r[h - 1];
  free(r);
  return v;
}
