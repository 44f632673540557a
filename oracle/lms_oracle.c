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

/* ------------------------------------------------------------------------
 * The same exact search, skipping slopes that provably cannot win.
 *
 * The exhaustive search above costs about 100 core-hours at 16384 points.
 * This variant returns the same result (every field bitwise) with far fewer
 * evaluations of F. It uses one fact beyond the definition:
 *
 *   Lipschitz bound. For slopes a and b, |F(a) - F(b)| <= L |a - b| with
 *   L = max x - min x. For a fixed set H of h points the slab height
 *   max_H z - min_H z, z = y - theta x, changes with theta at the rate
 *   x_q - x_p of its current top and bottom points, at most L in size; F is
 *   the minimum over all H of such functions, so it inherits the bound.
 *
 * Every F here is computed exactly as in lms_oracle_solve (same intercepts,
 * same sort, same window scan), so the two agree bitwise on every slope that
 * is evaluated. A slope is skipped only when an evaluated slope a gives
 *   F(theta) >= F(a) - L |theta - a| - (rounding allowances) > best so far,
 * so it can neither beat nor tie the final minimum. Slopes equal in binary64
 * have the same intercepts, hence the same window: one evaluation serves all
 * pairs with that slope, and the smallest (i, j) among them is kept, as the
 * exhaustive search's tie rule would.
 *
 * Rounding allowance at slope t: the computed intercepts and differences
 * each carry an error below 2^-53 M(t), M(t) = max|y| + |t| max|x|, so the
 * computed F is within 4 * 2^-53 M(t) of the exact one; 2^-46 M(t) is used.
 * ---------------------------------------------------------------------- */

typedef struct {
  double theta;
  int32_t i, j;
} pair_slope_t;

static int cmp_pair_slope(const void* a, const void* b) {
  const pair_slope_t* p = (const pair_slope_t*)a;
  const pair_slope_t* q = (const pair_slope_t*)b;
  if (p->theta != q->theta) return (p->theta > q->theta) - (p->theta < q->theta);
  if (p->i != q->i) return (p->i > q->i) - (p->i < q->i);
  return (p->j > q->j) - (p->j < q->j);
}

typedef struct {
  const double* xy;
  int64_t n, h;
  const pair_slope_t* s; /* sorted pair slopes */
  const int64_t* g;      /* start of each group of equal slopes; g[ng] = #pairs */
  int64_t ng;
  double* F;             /* computed width per group (NaN = not evaluated) */
  double L, xmax, ymax;
  double best;           /* smallest width found so far */
  int64_t evaluated;
} bound_ctx;

static double allowance(const bound_ctx* c, double t) {
  return ldexp(c->ymax + fabs(t) * c->xmax, -46);
}

/* Evaluate group k (its slope's narrowest window); keeps the best width. */
static double eval_group(bound_ctx* c, int64_t k, double* z) {
  const double t = c->s[c->g[k]].theta;
  double w, lo, hi;
  sorted_intercepts(c->xy, c->n, t, z);
  narrowest_window(z, c->n, c->h, &w, &lo, &hi);
  c->F[k] = w;
#pragma omp critical(lms_oracle_bound)
  {
    if (w < c->best) c->best = w;
    c->evaluated++;
  }
  return w;
}

/* Groups strictly between evaluated groups a < b: skip them all if the bound
 * from a and b exceeds the best width, else evaluate the middle one and split. */
static void search_between(bound_ctx* c, int64_t a, int64_t b, double* z) {
  if (b - a < 2) return;
  const double ta = c->s[c->g[a]].theta, tb = c->s[c->g[b]].theta;
  const double p = c->s[c->g[a + 1]].theta, q = c->s[c->g[b - 1]].theta;
  const double Fa = c->F[a] - allowance(c, ta), Fb = c->F[b] - allowance(c, tb);
  const double L = c->L * (1.0 + 0x1p-40);
  /* On [p, q], F >= max(Fa - L (t - ta), Fb - L (tb - t)); each term below is a
   * lower bound of that maximum over the whole interval. */
  double lb = Fa - L * (q - ta);
  const double from_b = Fb - L * (tb - p);
  const double meet = 0.5 * (Fa + Fb - L * (tb - ta));
  if (from_b > lb) lb = from_b;
  if (meet > lb) lb = meet;
  lb -= fmax(allowance(c, p), allowance(c, q)) + ldexp(fabs(c->F[a]) + fabs(c->F[b]), -46);
  double best;
#pragma omp atomic read
  best = c->best;
  if (lb > best) return;
  const int64_t m = a + (b - a) / 2;
  eval_group(c, m, z);
  search_between(c, a, m, z);
  search_between(c, m, b, z);
}

int lms_oracle_solve_bounded(const double* xy, int64_t n, int64_t h, int nthreads,
                             lms_oracle_result* out, int64_t* evaluated) {
  if (!out) return LMS_ORACLE_ERR_ARG;
  if (evaluated) *evaluated = -1;
  int64_t hh = h;
  int st = check_args(xy, n, &hh);
  if (st != LMS_ORACLE_OK || n > INT32_MAX) return lms_oracle_solve(xy, n, h, nthreads, out);

  /* all pair slopes with x_i != x_j, as the exhaustive search computes them */
  int64_t m = 0, vertical = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j) m += xy[2 * j] != xy[2 * i];
  pair_slope_t* s = (pair_slope_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(*s));
  if (!s) return lms_oracle_solve(xy, n, h, nthreads, out);
  int finite = 1;
  int64_t t = 0;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j) {
      if (xy[2 * j] == xy[2 * i]) {
        ++vertical;
        continue;
      }
      s[t].theta = (xy[2 * j + 1] - xy[2 * i + 1]) / (xy[2 * j] - xy[2 * i]);
      s[t].i = (int32_t)i;
      s[t].j = (int32_t)j;
      finite &= isfinite(s[t].theta) != 0;
      ++t;
    }
  if (m == 0 || !finite) { /* all x equal, or overflowing slopes: no bound to use */
    free(s);
    return lms_oracle_solve(xy, n, h, nthreads, out);
  }
  qsort(s, (size_t)m, sizeof(*s), cmp_pair_slope);

  int64_t ng = 0;
  int64_t* g = (int64_t*)malloc((size_t)(m + 1) * sizeof(int64_t));
  for (int64_t k = 0; k < m; ++k)
    if (k == 0 || s[k].theta != s[k - 1].theta) g[ng++] = k;
  g[ng] = m;

  bound_ctx c;
  c.xy = xy;
  c.n = n;
  c.h = hh;
  c.s = s;
  c.g = g;
  c.ng = ng;
  c.F = (double*)malloc((size_t)ng * sizeof(double));
  for (int64_t k = 0; k < ng; ++k) c.F[k] = NAN;
  double xlo = xy[0], xhi = xy[0];
  c.xmax = c.ymax = 0.0;
  for (int64_t k = 0; k < n; ++k) {
    xlo = fmin(xlo, xy[2 * k]);
    xhi = fmax(xhi, xy[2 * k]);
    c.xmax = fmax(c.xmax, fabs(xy[2 * k]));
    c.ymax = fmax(c.ymax, fabs(xy[2 * k + 1]));
  }
  c.L = xhi - xlo;
  c.best = INFINITY;
  c.evaluated = 0;

#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  /* a coarse pass of evenly spaced groups (both ends included), then the
   * intervals between them, each searched independently */
  const int64_t K = ng < 4096 ? ng : 4096;
  int64_t* anchor = (int64_t*)malloc((size_t)K * sizeof(int64_t));
  for (int64_t k = 0; k < K; ++k) anchor[k] = K == 1 ? 0 : (ng - 1) * k / (K - 1);
#pragma omp parallel
  {
    double* z = (double*)malloc((size_t)n * sizeof(double));
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 0; k < K; ++k) eval_group(&c, anchor[k], z);
#pragma omp for schedule(dynamic, 1)
    for (int64_t k = 1; k < K; ++k) search_between(&c, anchor[k - 1], anchor[k], z);
    free(z);
  }

  /* the canonical minimum over the evaluated groups; a group's first pair
   * is its smallest (i, j) */
  best_t best = {INFINITY, 0.0, 0.0, 0.0, -1, -1};
  double* z = (double*)malloc((size_t)n * sizeof(double));
  for (int64_t k = 0; k < ng; ++k) {
    if (!(c.F[k] <= c.best)) continue; /* skipped (NaN) or wider than the best */
    best_t cand;
    cand.theta = s[g[k]].theta;
    cand.i = s[g[k]].i;
    cand.j = s[g[k]].j;
    sorted_intercepts(xy, n, cand.theta, z);
    narrowest_window(z, n, hh, &cand.width, &cand.z_lo, &cand.z_hi);
    if (better(&cand, &best)) best = cand;
  }
  free(z);

  memset(out, 0, sizeof(*out));
  out->status = LMS_ORACLE_OK;
  out->h = (int32_t)hh;
  out->theta1 = best.theta;
  out->theta2 = 0.5 * (best.z_lo + best.z_hi);
  out->width = best.width;
  out->half_width = 0.5 * best.width;
  out->z_lo = best.z_lo;
  out->z_hi = best.z_hi;
  out->pair_i = best.i;
  out->pair_j = best.j;
  out->candidates = m;
  out->vertical = vertical;
  if (evaluated) *evaluated = c.evaluated;
  free(anchor);
  free(c.F);
  free(g);
  free(s);
  return LMS_ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * Algorithm 1 as the paper states it: one bracelet hanging from every
 * intersection point of two dual lines (Section 3.4, Algorithm 1).
 *
 * For the vertex of pair (i, j) at slope theta: take every point's intercept
 * z_k = fma(-theta, x_k, y_k) (the dual lines cut by the vertical line through
 * the vertex, negated), with the pair's own two members set to exactly
 * c = z_i (in exact arithmetic they are equal), and sort them. The vertex
 * occupies every rank whose value equals c: ranks r_lo..r_hi. A bracelet
 * spans h consecutive ranks with the vertex at one end; its length is the
 * distance from c to the other end.
 *
 *   rule LITERAL: the vertex rank is k = r_lo and the far end is
 *     X[(k + n/2) mod n] as printed. For even n and the default h
 *     (h - 1 = n/2) that is the upward bracelet from k when it fits and
 *     otherwise, through the wrap, the downward one ending at k; that reading
 *     (up from k if it fits, else down to k if it fits) is used for every
 *     (n, h).
 *   rule TIED: upward from the lower tied rank r_lo and downward from the
 *     upper tied rank r_hi, the shorter of the two that fit. This is the
 *     reading under which the minimum over vertices is the LMS width: the
 *     optimal slab's boundary passes through the vertex with the rest of the
 *     slab on one side, whichever rank the tie is given.
 *
 * The minimum bracelet over all vertices is taken by the key (length, theta,
 * lower end), then (i, j) (Algorithm 1, the final reduction), and translated
 * back to the line (slope theta, intercept at the bracelet's midpoint).
 * ---------------------------------------------------------------------- */

/* Bracelet hanging from the vertex of pair (i, j), i < j, x_i != x_j. */
static void vertex_bracelet(const double* xy, int64_t n, int64_t h, int rule, int64_t i,
                            int64_t j, double* X, best_t* b) {
  const double theta = (xy[2 * j + 1] - xy[2 * i + 1]) / (xy[2 * j] - xy[2 * i]);
  const double c = fma(-theta, xy[2 * i], xy[2 * i + 1]);
  for (int64_t k = 0; k < n; ++k)
    X[k] = (k == i || k == j) ? c : fma(-theta, xy[2 * k], xy[2 * k + 1]);
  qsort(X, (size_t)n, sizeof(double), cmp_f64);
  int64_t r_lo = 0;
  while (X[r_lo] < c) ++r_lo;
  int64_t r_hi = r_lo;
  while (r_hi + 1 < n && X[r_hi + 1] == c) ++r_hi;
  /* far ends: upward from r_lo, downward to r_hi (LITERAL: both from r_lo) */
  const int64_t top = r_lo + h - 1;
  const int64_t bot = (rule == LMS_ORACLE_RULE_LITERAL ? r_lo : r_hi) - h + 1;
  double up = INFINITY, dn = INFINITY;
  if (top < n) up = X[top] - c;
  if (bot >= 0 && (rule != LMS_ORACLE_RULE_LITERAL || top >= n)) dn = c - X[bot];
  b->theta = theta;
  b->i = i;
  b->j = j;
  b->width = INFINITY;
  b->z_lo = b->z_hi = NAN;
  /* on equal lengths the lower bracelet, as for the window scan */
  if (dn <= up && dn < INFINITY) {
    b->width = dn;
    b->z_lo = X[bot];
    b->z_hi = c;
  } else if (up < INFINITY) {
    b->width = up;
    b->z_lo = c;
    b->z_hi = X[top];
  }
}

int lms_oracle_bracelets(const double* xy, int64_t n, int64_t h, int rule, int nthreads,
                         lms_oracle_result* out) {
  if (!out) return LMS_ORACLE_ERR_ARG;
  if (rule != LMS_ORACLE_RULE_TIED && rule != LMS_ORACLE_RULE_LITERAL) return LMS_ORACLE_ERR_ARG;
  int st = lms_oracle_solve(xy, n, h, 1, out); /* argument checks; all-x-equal answer */
  if (st != LMS_ORACLE_OK) return st;
  int64_t hh = out->h;
  best_t best = {INFINITY, 0.0, 0.0, 0.0, -1, -1};
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    double* X = (double*)malloc((size_t)n * sizeof(double));
    best_t mine = {INFINITY, 0.0, 0.0, 0.0, -1, -1};
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < n - 1; ++i)
      for (int64_t j = i + 1; j < n; ++j) {
        if (xy[2 * j] == xy[2 * i]) continue;
        best_t b;
        vertex_bracelet(xy, n, hh, rule, i, j, X, &b);
        if (better(&b, &mine)) mine = b;
      }
#pragma omp critical
    {
      if (better(&mine, &best)) best = mine;
    }
    free(X);
  }
  out->theta1 = best.theta;
  out->theta2 = 0.5 * (best.z_lo + best.z_hi);
  out->width = best.width;
  out->half_width = 0.5 * best.width;
  out->z_lo = best.z_lo;
  out->z_hi = best.z_hi;
  out->pair_i = best.i;
  out->pair_j = best.j;
  return LMS_ORACLE_OK;
}
