/* Reference CPU implementation of the exact 2D least-median-of-squares line.
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the package's smoke check and
 * the benchmark's CPU-baseline leg load this library. The product path never
 * calls it, and it shares no code with the GPU library.
 *
 * Paper: Shapira & Hassner, "GPU-Based Computation of 2D Least Median of
 * Squares with Applications to Fast and Robust Line Detection" (arXiv
 * 1510.01041).
 *   - Section 1, Eq. (1): the model y = x*theta1 + theta2 + e and the LMS
 *     criterion, the median of the squared residuals r = y - x*theta1 - theta2.
 *   - Section 3.1: the LMS line bisects the thinnest vertical slab holding
 *     half of the points.
 *   - Sections 3.3 and 3.4.1: equioscillation, which puts one end of the
 *     optimal bracelet on an intersection of two dual lines, so that searching
 *     the slopes of all point pairs is exhaustive.
 *
 * Notation: h is the number of points the slab must hold (default
 * floor(n/2)+1, the low median). For a slope theta, z_k = y_k - theta*x_k and
 * F(theta) is the narrowest width z_(s+h-1) - z_(s) over windows of h
 * consecutive order statistics. The LMS half-width w* is min F / 2 over the
 * pair slopes, and the squared median residual is w*^2.
 *
 * All arithmetic is IEEE binary64 with round-to-nearest; z uses a fused
 * multiply-add, z = fma(-theta, x, y).
 */
#ifndef LMS_ORACLE_H
#define LMS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LMS_ORACLE_OK = 0,
  LMS_ORACLE_OK_DEGENERATE = 1, /* all x equal: theta1 := 0 */
  LMS_ORACLE_ERR_ARG = -1,      /* n < 2, h outside [2, n], or a null pointer */
  LMS_ORACLE_ERR_NONFINITE = -2 /* a coordinate is NaN or infinite */
};

typedef struct {
  double theta1, theta2; /* the line y = theta1*x + theta2 */
  double half_width;     /* w = (z_hi - z_lo)/2, the h-th smallest |residual| */
  double width;          /* z_hi - z_lo */
  double z_lo, z_hi;     /* the window's ends at slope theta1 */
  int64_t pair_i, pair_j; /* first pair (i < j) whose slope attains the result */
  int64_t candidates;     /* pairs evaluated (x_i != x_j) */
  int64_t vertical;       /* pairs skipped because x_i == x_j */
  int32_t status, h;
} lms_oracle_result;

/* Exhaustive FP64 search. xy is n interleaved (x, y) pairs in host memory;
 * h = 0 selects floor(n/2)+1. nthreads <= 0 uses the OpenMP default.
 * Ties between slopes go to the smallest (width, theta, z_lo), then to the
 * smallest (i, j). Returns the status, also stored in out->status. */
int lms_oracle_solve(const double* xy, int64_t n, int64_t h, int nthreads,
                     lms_oracle_result* out);

/* The same result as lms_oracle_solve (every field), from fewer evaluations
 * of F: a slope is skipped only when the Lipschitz bound of F in theta
 * (constant max x - min x), measured from evaluated slopes and less rounding
 * allowances, proves it wider than the best width found. Slopes equal in
 * binary64 share one evaluation. Needs about 16 bytes per pair of host
 * memory. evaluated (may be NULL) receives the number of distinct slopes
 * whose window was computed. */
int lms_oracle_solve_bounded(const double* xy, int64_t n, int64_t h, int nthreads,
                             lms_oracle_result* out, int64_t* evaluated);

/* F(theta) at one slope: the narrowest h-window of z = fma(-theta, x, y);
 * among equally narrow windows the lowest one. Writes width, z_lo, z_hi. */
int lms_oracle_window(const double* xy, int64_t n, int64_t h, double theta,
                      double* width, double* z_lo, double* z_hi);

/* F at the slopes of m given pairs (pairs[2t], pairs[2t+1]); the slope is
 * computed with the smaller index first. A vertical pair gets width = +inf and
 * theta = NaN. Outputs are arrays of length m (any of them may be NULL). */
int lms_oracle_eval_pairs(const double* xy, int64_t n, int64_t h,
                          const int64_t* pairs, int64_t m, int nthreads,
                          double* theta, double* width, double* z_lo, double* z_hi);

/* Anchored widths of pair (i, j): with c = z_i at the pair's slope and both
 * members taken as exactly c, up = the h-th smallest of {z_k - c >= 0} and
 * dn = the h-th smallest of {c - z_k >= 0} (+inf when fewer than h qualify). */
int lms_oracle_anchored(const double* xy, int64_t n, int64_t h, int64_t i, int64_t j,
                        double* up, double* dn);

/* h-th smallest |y_k - theta1*x_k - theta2| (residual by fma), for checking
 * that a returned line really holds h points within its half-width. */
double lms_oracle_hth_abs_residual(const double* xy, int64_t n, int64_t h,
                                   double theta1, double theta2);

/* Algorithm 1 as stated (Section 3.4): the bracelet hanging from each vertex
 * (pair slope), with the pair's members set to exactly z_i, the intercepts
 * sorted, and the far end h - 1 ranks away from the vertex rank; the minimum
 * over vertices by (length, theta, lower end), then (i, j). `rule` says which
 * rank a vertex tied with other values takes:
 *   LMS_ORACLE_RULE_TIED    upward from the lowest tied rank and downward from
 *                           the highest (exact: the minimum is the LMS width);
 *   LMS_ORACLE_RULE_LITERAL the printed X[(k + |P|/2) mod |P|] with k the
 *                           lowest tied rank (misses the optimum on many sets).
 * All x equal: the answer of lms_oracle_solve. Fields as lms_oracle_solve;
 * candidates and vertical count the pairs as there. */
enum { LMS_ORACLE_RULE_TIED = 0, LMS_ORACLE_RULE_LITERAL = 1 };
int lms_oracle_bracelets(const double* xy, int64_t n, int64_t h, int rule, int nthreads,
                         lms_oracle_result* out);

#ifdef __cplusplus
}
#endif
#endif
