// Algorithm 1 of the paper as it is stated (Section 3.4), with the three
// kernels of Section 3.6 recast for gfx950. It is the ablation that lms_solve
// is measured against: every vertex of the dual arrangement is materialised,
// and every vertex gets a full sort of the n intercepts.
//
//   k_alg1_vertices   all n(n-1)/2 vertices (pair slopes) into an array, from
//                     16x16 tiles of pairs whose row and column points are
//                     staged in LDS (the tiles below the diagonal exit).
//   k_alg1_bracelets  one workgroup per vertex, N2/2 threads (N2 = next power
//                     of two >= n, +inf padding): the intercepts of all points
//                     at the vertex's slope, a bitonic sort in LDS, and the
//                     bracelet that hangs from the vertex, h - 1 ranks away.
//   k_alg1_reduce     canonical minimum over the bracelet array, per block,
//   k_alg1_final      then over the blocks; translation back to the line.
//
// The vertex rank: the pair's own two intercepts are set to exactly
// c = z_i (equal in exact arithmetic), and the vertex occupies every rank whose
// value equals c, ranks r_lo..r_hi. Rule LMS_RULE_TIED takes the upward
// bracelet from r_lo and the downward one ending at r_hi, the shorter that
// fits; its minimum is the LMS width. Rule LMS_RULE_LITERAL takes the printed
// X[(k + |P|/2) mod |P|] with k = r_lo (up from k when it fits, else down to
// k): a vertex tied at two ranks then sees only one side, and the minimum can
// miss the optimum.
//
// Work is O(n^3 log^2 n) and memory O(n^2): sizes up to LMS_ALG1_MAX_N.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <string>

#include "lms.h"
#include "lms_device.h"
#include "lms_host.h"

namespace {

using lms_dev::Best;
using lms_dev::better;
using lms_host::fail;

constexpr int kTile = 16;
constexpr int kReduceNT = 1024;
constexpr int kWorkspaceTag = 3;

__global__ __launch_bounds__(kTile * kTile) void k_alg1_vertices(const double* __restrict__ xy,
                                                                 int n, double* __restrict__ vth,
                                                                 unsigned* __restrict__ vij) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bj < bi) return;  // every pair of this tile has i > j
  __shared__ double2 row[kTile], col[kTile];
  const int tx = threadIdx.x, ty = threadIdx.y;
  if (ty == 0) {
    const int j = bj * kTile + tx;
    col[tx] = j < n ? make_double2(xy[2 * j], xy[2 * j + 1]) : make_double2(0.0, 0.0);
  } else if (ty == 1) {
    const int i = bi * kTile + tx;
    row[tx] = i < n ? make_double2(xy[2 * i], xy[2 * i + 1]) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const int i = bi * kTile + ty, j = bj * kTile + tx;
  if (i < j && j < n) {
    const double2 a = row[ty], b = col[tx];
    const long long t = (long long)i * n - (long long)i * (i + 1) / 2 + (j - i - 1);
    // a vertical pair (equal x) has no vertex: NaN marks it
    vth[t] = a.x == b.x ? NAN : (b.y - a.y) / (b.x - a.x);
    vij[t] = (unsigned)i | ((unsigned)j << 16);
  }
}

// Ascending bitonic sort of X[0..N2) by N2/2 threads, one compare-exchange
// per thread and stage.
template <int N2>
__device__ __forceinline__ void bitonic_sort(double* X) {
  const int t = threadIdx.x;
  for (int size = 2; size <= N2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const int lo = 2 * t - (t & (stride - 1));
      const int hi = lo + stride;
      const bool asc = (lo & size) == 0;
      const double a = X[lo], b = X[hi];
      if ((a > b) == asc && a != b) {
        X[lo] = b;
        X[hi] = a;
      }
      __syncthreads();
    }
  }
}

template <int N2>
__global__ __launch_bounds__(N2 / 2) void k_alg1_bracelets(const double* __restrict__ xy, int n,
                                                           int h, int rule,
                                                           const double* __restrict__ vth,
                                                           const unsigned* __restrict__ vij,
                                                           double4* __restrict__ rec) {
  constexpr int NT = N2 / 2;
  __shared__ double X[N2];
  const long long t = blockIdx.x;
  const double theta = vth[t];
  if (theta != theta) {  // vertical pair: no vertex
    if (threadIdx.x == 0) rec[t] = make_double4(INFINITY, NAN, NAN, NAN);
    return;
  }
  const unsigned ij = vij[t];
  const int i = (int)(ij & 0xFFFFu), j = (int)(ij >> 16);
  const double c = fma(-theta, xy[2 * i], xy[2 * i + 1]);
  for (int k = threadIdx.x; k < N2; k += NT)
    X[k] = (k == i || k == j) ? c : (k < n ? fma(-theta, xy[2 * k], xy[2 * k + 1]) : INFINITY);
  __syncthreads();
  bitonic_sort<N2>(X);
  if (threadIdx.x != 0) return;
  // ranks of the vertex: [r_lo, r_hi] hold exactly c
  int lo = 0, hi = n;  // first index with X >= c
  while (lo < hi) {
    const int m = (lo + hi) >> 1;
    if (X[m] < c) lo = m + 1; else hi = m;
  }
  const int r_lo = lo;
  hi = n;  // first index with X > c
  while (lo < hi) {
    const int m = (lo + hi) >> 1;
    if (X[m] <= c) lo = m + 1; else hi = m;
  }
  const int r_hi = lo - 1;
  const int top = r_lo + h - 1;
  const int bot = (rule == LMS_RULE_LITERAL ? r_lo : r_hi) - h + 1;
  double up = INFINITY, dn = INFINITY;
  if (top < n) up = X[top] - c;
  if (bot >= 0 && (rule != LMS_RULE_LITERAL || top >= n)) dn = c - X[bot];
  double4 r = make_double4(INFINITY, theta, NAN, NAN);
  if (dn <= up && dn < INFINITY) r = make_double4(dn, theta, X[bot], c);  // lower on a tie
  else if (up < INFINITY) r = make_double4(up, theta, c, X[top]);
  rec[t] = r;
}

// Canonical minimum over records [0, V) per block (grid-stride), with the
// vertical pairs counted; the block's best goes to part[blockIdx.x].
__global__ __launch_bounds__(kReduceNT) void k_alg1_reduce(const double4* __restrict__ rec,
                                                           const unsigned* __restrict__ vij,
                                                           long long V, Best* __restrict__ part,
                                                           unsigned long long* __restrict__ vert) {
  __shared__ Best s[kReduceNT];
  __shared__ unsigned long long s_v[kReduceNT / 64];
  Best b{INFINITY, 0.0, 0.0, 0.0, UINT_MAX, UINT_MAX};
  unsigned long long nv = 0;
  for (long long t = blockIdx.x * (long long)kReduceNT + threadIdx.x; t < V;
       t += (long long)gridDim.x * kReduceNT) {
    const double4 r = rec[t];
    if (r.y != r.y) {
      ++nv;
      continue;
    }
    const unsigned ij = vij[t];
    const Best c{r.x, r.y, r.z, r.w, ij & 0xFFFFu, ij >> 16};
    if (better(c, b)) b = c;
  }
  s[threadIdx.x] = b;
  for (int o = 32; o > 0; o >>= 1) nv += __shfl_xor(nv, o);
  if ((threadIdx.x & 63) == 0) s_v[threadIdx.x >> 6] = nv;
  __syncthreads();
  for (int w = kReduceNT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w && better(s[threadIdx.x + w], s[threadIdx.x])) s[threadIdx.x] = s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s[0];
    unsigned long long tot = 0;
    for (int k = 0; k < kReduceNT / 64; ++k) tot += s_v[k];
    vert[blockIdx.x] = tot;
  }
}

// Minimum over the blocks; input checks; all x equal; the lms_result.
__global__ __launch_bounds__(kReduceNT) void k_alg1_final(const double* __restrict__ xy, int n,
                                                          int h, long long V,
                                                          const Best* __restrict__ part,
                                                          const unsigned long long* __restrict__ vert,
                                                          int G, lms_result* __restrict__ out) {
  __shared__ double X[2 * kReduceNT];
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  for (int k = threadIdx.x; k < 2 * n; k += kReduceNT)
    if (!isfinite(xy[k])) s_bad = 1;
  __syncthreads();
  if (s_bad) {
    if (threadIdx.x == 0) {
      lms_result o{};
      o.theta1 = o.theta2 = o.half_width = o.width = o.z_lo = o.z_hi = NAN;
      o.pair_i = o.pair_j = -1;
      o.status = LMS_ERR_NONFINITE;
      o.h = h;
      *out = o;
    }
    return;
  }
  __shared__ unsigned long long s_nv;
  if (threadIdx.x == 0) {
    unsigned long long v = 0;
    for (int g = 0; g < G; ++g) v += vert[g];
    s_nv = v;
  }
  __syncthreads();
  const unsigned long long nv = s_nv;
  if (threadIdx.x == 0 && nv < (unsigned long long)V) {
    Best b{INFINITY, 0.0, 0.0, 0.0, UINT_MAX, UINT_MAX};
    for (int g = 0; g < G; ++g)
      if (better(part[g], b)) b = part[g];
    lms_result o{};
    o.theta1 = b.th;
    o.theta2 = 0.5 * (b.lo + b.hi);
    o.width = b.w;
    o.half_width = 0.5 * b.w;
    o.z_lo = b.lo;
    o.z_hi = b.hi;
    o.pair_i = (int)b.a;
    o.pair_j = (int)b.b;
    o.status = LMS_OK;
    o.h = h;
    o.candidates = (unsigned long long)V - nv;
    o.vertical = nv;
    o.survivors = o.candidates;  // every vertex is sorted
    o.point_evals = o.candidates * (unsigned long long)n;
    *out = o;
  }
  if (nv < (unsigned long long)V) return;  // uniform across the block: thread 0 alone
  // every pair is vertical (all x equal): slope 0 and the narrowest window of y
  for (int k = threadIdx.x; k < 2 * kReduceNT; k += kReduceNT) X[k] = k < n ? xy[2 * k + 1] : INFINITY;
  __syncthreads();
  bitonic_sort<2 * kReduceNT>(X);
  if (threadIdx.x == 0) {
    int s = 0;
    double w = X[h - 1] - X[0];
    for (int q = 1; q + h <= n; ++q)
      if (X[q + h - 1] - X[q] < w) {
        w = X[q + h - 1] - X[q];
        s = q;
      }
    lms_result o{};
    o.theta1 = 0.0;
    o.theta2 = 0.5 * (X[s] + X[s + h - 1]);
    o.width = w;
    o.half_width = 0.5 * w;
    o.z_lo = X[s];
    o.z_hi = X[s + h - 1];
    o.pair_i = o.pair_j = -1;
    o.status = LMS_OK_DEGENERATE;
    o.h = h;
    o.vertical = (unsigned long long)V;
    *out = o;
  }
}

template <int N2>
void launch_bracelets(hipStream_t s, long long V, const double* xy, int n, int h, int rule,
                      const double* vth, const unsigned* vij, double4* rec) {
  hipLaunchKernelGGL(k_alg1_bracelets<N2>, dim3((unsigned)V), dim3(N2 / 2), 0, s, xy, n, h, rule,
                     vth, vij, rec);
}

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" lms_status lms_solve_bracelets(const double* d_xy, int64_t n, int64_t h, int32_t rule,
                                          lms_result* d_out, void* stream) {
  lms_host::clear_error();
  if (!d_xy || !d_out) return fail(LMS_ERR_ARG, "null pointer");
  if (n < 2 || n > LMS_ALG1_MAX_N)
    return fail(LMS_ERR_ARG, "n must be in [2, " + std::to_string(LMS_ALG1_MAX_N) + "]");
  if (h == 0) h = n / 2 + 1;
  if (h < 2 || h > n) return fail(LMS_ERR_ARG, "h must be in [2, n]");
  if (rule != LMS_RULE_TIED && rule != LMS_RULE_LITERAL)
    return fail(LMS_ERR_ARG, "rule must be LMS_RULE_TIED or LMS_RULE_LITERAL");
  hipStream_t s = (hipStream_t)stream;
  const long long V = n * (n - 1) / 2;
  const int G = (int)std::min<long long>(4 * lms_host::num_cu(), (V + kReduceNT - 1) / kReduceNT);
  const size_t o_vij = up256((size_t)V * sizeof(double));
  const size_t o_rec = o_vij + up256((size_t)V * sizeof(unsigned));
  const size_t o_part = o_rec + up256((size_t)V * sizeof(double4));
  const size_t o_vert = o_part + up256((size_t)G * sizeof(Best));
  const size_t total = o_vert + up256((size_t)G * sizeof(unsigned long long));
  char* base = nullptr;
  lms_status st = lms_host::get_workspace(kWorkspaceTag, stream, total, &base);
  if (st != LMS_OK) return st;
  double* vth = (double*)base;
  unsigned* vij = (unsigned*)(base + o_vij);
  double4* rec = (double4*)(base + o_rec);
  Best* part = (Best*)(base + o_part);
  unsigned long long* vert = (unsigned long long*)(base + o_vert);
  const int T = (int)((n + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_alg1_vertices, dim3(T, T), dim3(kTile, kTile), 0, s, d_xy, (int)n, vth, vij);
  int n2 = 128;
  while (n2 < n) n2 <<= 1;
  switch (n2) {
    case 128: launch_bracelets<128>(s, V, d_xy, (int)n, (int)h, rule, vth, vij, rec); break;
    case 256: launch_bracelets<256>(s, V, d_xy, (int)n, (int)h, rule, vth, vij, rec); break;
    case 512: launch_bracelets<512>(s, V, d_xy, (int)n, (int)h, rule, vth, vij, rec); break;
    case 1024: launch_bracelets<1024>(s, V, d_xy, (int)n, (int)h, rule, vth, vij, rec); break;
    default: launch_bracelets<2048>(s, V, d_xy, (int)n, (int)h, rule, vth, vij, rec); break;
  }
  hipLaunchKernelGGL(k_alg1_reduce, dim3(G), dim3(kReduceNT), 0, s, rec, vij, V, part, vert);
  hipLaunchKernelGGL(k_alg1_final, dim3(1), dim3(kReduceNT), 0, s, d_xy, (int)n, (int)h, V, part,
                     vert, G, d_out);
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(LMS_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(err));
  return LMS_OK;
}
