// Exact 2D least-median-of-squares line search for gfx950 (MI355X).
//
// Method (arXiv 1510.01041): the LMS line is the bisector of the thinnest
// vertical slab holding h points (Section 3.1, Eq. (1)); its slope is the
// slope of some pair of points, a vertex of the dual arrangement (Sections
// 3.2-3.3), so scanning every pair slope is exact (Algorithm 1, Section 3.4.1).
//
// The paper materialises all vertices and fully sorts n dual intercepts per
// vertex. Here the per-vertex work is a count instead of a sort:
//
//   prep      one block: finiteness, centring, FP32 copy, seed pairs.
//   recheck   one block per entry: FP64 intercepts z = fma(-theta, x, y), a
//             bitonic sort in LDS and the narrowest-window scan. Runs first on
//             the seed pairs to give an FP64 width bound W, then on the screen
//             survivors.
//   screen    the hot path. Each wavefront takes an anchor point i and 64
//             partners j at a time; lanes hold the points (registers, plus LDS
//             beyond 4096 points). For a pair's slope it counts in FP32 how many
//             points lie within W + tau of the anchor's intercept (one FMA and
//             one compare per point, ballot + scalar popcount per 64 points),
//             and rejects the pair as soon as h can no longer be reached. Pairs
//             that pass both this band test and the anchored one-sided tests
//             go to the FP64 recheck.
//   finalize  one block: canonical minimum over all rechecked entries.
//
// Soundness of the FP32 screen: tau bounds the FP32 error of every anchored
// residual against exact arithmetic, and W bounds the optimal width from
// above. The optimal slab has a pair of points at one edge (equioscillation),
// so that pair's anchored window of width <= W holds h points and passes the
// test, reaches the FP64 recheck and gives the same bits as the reference.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstddef>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <array>
#include <vector>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <utility>

#include "lms.h"
#include "lms_device.h"
#include "lms_host.h"

namespace {

using namespace lms_dev;
using lms_host::fail;
constexpr int kDefaultSeeds = 127;
constexpr long long kScreenCap = 1ll << 24;     // survivor slots beyond the seeds
constexpr int kRegChunks = 64;                  // points per lane kept in VGPRs (max)
constexpr int kPathSingle = 0;                  // tuning-table key of lms_solve
constexpr int kNetPoints = 2048;                // points the seed network pools over

constexpr int kPrunedBins = 2048;  // bins per anchor of the pruned slope-bin screen

// Per-solve state in device memory.
struct __align__(16) Ctx {
  int n, h, n_pad, n_seeds;
  int status, all_x_equal, argminx, argmaxx;
  double cx, cy;      // centre (midrange) used for the FP32 copy
  double fx, fy;      // scales of the FP32 copy (powers of two; f32_scale)
  double xh, yh;      // bounds on |x - cx| and |y - cy|
  double xabs, yabs;  // max |x|, max |y| of the raw input
  double xr, yr;      // bounds on max x - min x and max y - min y
  double th_lo, th_hi;  // every pair that can be optimal has its slope in here
  unsigned long long wbound;  // FP64 width bound, as bits (monotone atomicMin)
  unsigned int n_entries;     // seeds + survivors appended so far
  unsigned int overflow;
  unsigned int next_item;     // work counter of the exhaustive screen
  unsigned int n_cands;       // pairs passed by the slope-bin screen
  unsigned int cand_overflow;
  unsigned int bins;          // slope bins per anchor (0: no slope-bin screen)
  int n_live;                 // anchors left by the slope range (-1: no range)
};

// Search counters, each spread over kSlots addresses (slot = block index mod
// kSlots) so that the waves of a launch do not all hit one address;
// finalize_block adds the slots. They live right after the Ctx in the workspace.
enum { ST_VERT, ST_SCREENED, ST_BAND, ST_EVALS, ST_DEVALS, ST_FORCED, ST_BIN, kStats };
constexpr int kSlots = 64;
struct Stats {
  unsigned long long v[kStats][kSlots];
};
constexpr size_t kStatsOffset = (sizeof(Ctx) + 255) & ~size_t(255);

__device__ __forceinline__ void stat_add(Ctx* ctx, int k, unsigned long long v) {
  if (v) {
    Stats* st = reinterpret_cast<Stats*>(reinterpret_cast<char*>(ctx) + kStatsOffset);
    atomicAdd(&st->v[k][blockIdx.x % kSlots], v);
  }
}

// ---------------------------------------------------------------- prep

// Extremes of a range of points: the smallest x (the lowest index among
// equal ones), the largest x (the lowest index among equal ones), the y
// extremes and whether every coordinate is finite. Merging is exact and
// order-free.
struct __align__(16) PrepPart {
  double mnx, mxx, mny, mxy;
  int amn, amx, fin, pad;
};

__device__ __forceinline__ void prep_merge(PrepPart& a, double mn2, int amn2, double mx2, int amx2,
                                           double my2, double My2, int fin2) {
  if (mn2 < a.mnx || (mn2 == a.mnx && amn2 < a.amn)) { a.mnx = mn2; a.amn = amn2; }
  if (mx2 > a.mxx || (mx2 == a.mxx && amx2 < a.amx)) { a.mxx = mx2; a.amx = amx2; }
  a.mny = fmin(a.mny, my2);
  a.mxy = fmax(a.mxy, My2);
  a.fin &= fin2;
}

constexpr int kPrepNT = 1024;
// workgroups of the prep kernel: one per 1024 points, at most 16
int prep_blocks(int n) { return std::max(1, std::min(16, (n + 1023) / 1024)); }

// Extremes of all n points by the whole workgroup (every workgroup of k_prep
// computes the same ones: the merge is exact and order-free). Eight loads in
// flight at a time.
__device__ __forceinline__ PrepPart prep_extremes(const double* __restrict__ xy, int n) {
  __shared__ PrepPart s_p[kPrepNT / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  PrepPart a{INFINITY, -INFINITY, INFINITY, -INFINITY, INT_MAX, INT_MAX, 1, 0};
  constexpr int U = 8;
  for (int k0 = t; k0 < n; k0 += U * kPrepNT) {
    double2 q[U];
#pragma unroll
    for (int u = 0; u < U; ++u) q[u] = point_clamped(xy, k0 + u * kPrepNT, n);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * kPrepNT;
      if (k < n)
        prep_merge(a, q[u].x, k, q[u].x, k, q[u].y, q[u].y,
                   isfinite(q[u].x) && isfinite(q[u].y) ? 1 : 0);
    }
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1)
    prep_merge(a, __shfl_xor(a.mnx, m), __shfl_xor(a.amn, m), __shfl_xor(a.mxx, m),
               __shfl_xor(a.amx, m), __shfl_xor(a.mny, m), __shfl_xor(a.mxy, m),
               __shfl_xor(a.fin, m));
  if (lane == 0) s_p[wv] = a;
  __syncthreads();
  PrepPart b = s_p[0];
  for (int w = 1; w < kPrepNT / 64; ++w)
    prep_merge(b, s_p[w].mnx, s_p[w].amn, s_p[w].mxx, s_p[w].amx, s_p[w].mny, s_p[w].mxy,
               s_p[w].fin);
  return b;
}

// Every workgroup finds the extremes of all points (the same in each) and
// writes its share of the FP32 copy; workgroup 0 also writes the context,
// zeroes the search counters and writes the seed pairs.
__global__ __launch_bounds__(kPrepNT) void k_prep(const double* __restrict__ xy, int n, int h,
                                                  int n_pad, Ctx* ctx, float2* __restrict__ xy32,
                                                  uint2* __restrict__ entries, int n_seeds,
                                                  int n_random, unsigned long long seed_key,
                                                  unsigned bins, int cap) {
  const int t = threadIdx.x;
  const PrepPart a = prep_extremes(xy, n);
  const bool finite = a.fin != 0;
  const double minx = a.mnx, maxx = a.mxx, miny = a.mny, maxy = a.mxy;
  const double cx = minx + 0.5 * (maxx - minx), cy = miny + 0.5 * (maxy - miny);
  if (blockIdx.x == 0) {
    if (t == 0) {
      Ctx c;
      memset(&c, 0, sizeof(c));
      c.n = n; c.h = h; c.n_pad = n_pad; c.n_seeds = n_seeds;
      c.bins = bins;
      c.status = finite ? LMS_OK : LMS_ERR_NONFINITE;
      c.all_x_equal = finite && (minx == maxx);
      c.argminx = a.amn; c.argmaxx = a.amx;
      c.cx = cx; c.cy = cy;
      c.xh = fmax(fabs(minx - cx), fabs(maxx - cx)) * (1.0 + 0x1p-40);
      c.yh = fmax(fabs(miny - cy), fabs(maxy - cy)) * (1.0 + 0x1p-40);
      c.fx = f32_scale(c.xh);
      c.fy = f32_scale(c.yh);
      c.xabs = fmax(fabs(minx), fabs(maxx));
      c.yabs = fmax(fabs(miny), fabs(maxy));
      c.xr = (maxx - minx) * (1.0 + 0x1p-50);
      c.yr = (maxy - miny) * (1.0 + 0x1p-50);
      c.th_lo = -INFINITY;
      c.th_hi = INFINITY;
      c.n_live = -1;
      c.wbound = 0x7FF0000000000000ull;  // +inf
      c.n_entries = (unsigned)n_seeds;
      // all x equal: slope 0 is the answer; it is re-evaluated exactly as the
      // one survivor (the seeds give bounds only)
      if (c.all_x_equal && n_seeds < cap) {
        entries[n_seeds] = make_uint2(kDegenerate, kDegenerate);
        c.n_entries = (unsigned)n_seeds + 1u;
      }
      *ctx = c;
    }
    Stats* st = reinterpret_cast<Stats*>(reinterpret_cast<char*>(ctx) + kStatsOffset);
    for (int k = t; k < kStats * kSlots; k += kPrepNT) (&st->v[0][0])[k] = 0ull;
    // Seed entries: the extreme-x pair (never vertical unless all x are
    // equal), then n_random random pairs from a counter-based SplitMix64
    // stream. Slots past those (window pairs, written later) start as the
    // extreme-x pair.
    if (finite) {
      for (int e = t; e < n_seeds; e += kPrepNT) {
        uint2 p;
        if ((e == 0 || e > n_random) && minx == maxx) {
          p = make_uint2(kDegenerate, kDegenerate);
        } else if (e == 0 || e > n_random) {
          p = make_uint2((unsigned)min(a.amn, a.amx), (unsigned)max(a.amn, a.amx));
        } else {
          const unsigned long long r =
              mix64(seed_key + 0x9E3779B97F4A7C15ull * (unsigned long long)(e + 1));
          const unsigned aa = (unsigned)((r >> 32) % (unsigned long long)n);
          unsigned bb = (unsigned)((r & 0xFFFFFFFFull) % (unsigned long long)(n - 1));
          if (bb >= aa) ++bb;
          p = make_uint2(min(aa, bb), max(aa, bb));
        }
        entries[e] = p;
      }
    }
  }
  if (!finite) return;
  const float qnan = __int_as_float(0x7FC00000);
  // the same scales thread 0 of workgroup 0 stores (same inputs, same operations)
  const double fx = f32_scale(fmax(fabs(minx - cx), fabs(maxx - cx)) * (1.0 + 0x1p-40));
  const double fy = f32_scale(fmax(fabs(miny - cy), fabs(maxy - cy)) * (1.0 + 0x1p-40));
  for (int k = blockIdx.x * kPrepNT + t; k < n_pad; k += gridDim.x * kPrepNT) {
    float2 p = make_float2(qnan, qnan);
    if (k < n)
      p = make_float2((float)((xy[2 * k] - cx) * fx), (float)((xy[2 * k + 1] - cy) * fy));
    xy32[k] = p;
  }
}

void launch_prep(hipStream_t s, const double* xy, int n, int h, int n_pad, Ctx* ctx,
                 float2* xy32, uint2* entries, int n_seeds, int n_random,
                 unsigned long long seed_key, unsigned bins, int cap) {
  const int G = prep_blocks(n);
  hipLaunchKernelGGL(k_prep, dim3(G), dim3(kPrepNT), 0, s, xy, n, h, n_pad, ctx, xy32, entries,
                     n_seeds, n_random, seed_key, bins, cap);
}

// ---------------------------------------------------------------- finalize

// The canonical minimum over the exact records by (width, theta, z_lo, i, j)
// and the lms_result, by the NT threads of one workgroup (k_finalize).
template <int NT>
__device__ void finalize_block(Ctx* ctx, const uint2* __restrict__ entries,
                               const double4* __restrict__ res, int cap, lms_result* out) {
  __shared__ Best sb[NT / 64];
  __shared__ unsigned long long s_stat[kStats];
  const Ctx c = *ctx;
  const int t = threadIdx.x;
  // the counters' slots: one load per thread (not a chain of kSlots loads)
  if (t < kStats) s_stat[t] = 0ull;
  __syncthreads();
  {
    const Stats* st = reinterpret_cast<const Stats*>(reinterpret_cast<char*>(ctx) + kStatsOffset);
    for (int q = t; q < kStats * kSlots; q += NT) {
      const unsigned long long v = (&st->v[0][0])[q];
      if (v) atomicAdd(&s_stat[q / kSlots], v);
    }
  }
  Best b = {INFINITY, INFINITY, INFINITY, INFINITY, 0xFFFFFFFFu, 0xFFFFFFFFu};
  const unsigned end = c.status < 0 ? 0u : min(c.n_entries, (unsigned)cap);
  for (unsigned e = t; e < end; e += blockDim.x) {
    const double4 r = res[e];
    if (!(r.x <= INFINITY) || r.x == INFINITY) continue;  // vertical or NaN
    const uint2 p = entries[e];
    const Best q = {r.x, r.y, r.z, r.w, p.x, p.y};
    if (better(q, b)) b = q;
  }
  // the canonical minimum: by wavefront (shuffles), then across wavefronts
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const Best q = {__shfl_xor(b.w, m), __shfl_xor(b.th, m), __shfl_xor(b.lo, m),
                    __shfl_xor(b.hi, m), (unsigned)__shfl_xor((int)b.a, m),
                    (unsigned)__shfl_xor((int)b.b, m)};
    if (better(q, b)) b = q;
  }
  if ((t & 63) == 0) sb[t >> 6] = b;
  __syncthreads();
  if (t != 0) return;
  for (int w = 1; w < NT / 64; ++w)
    if (better(sb[w], b)) b = sb[w];
  lms_result o;
  memset(&o, 0, sizeof(o));
  o.h = c.h;
  const unsigned long long pairs = (unsigned long long)c.n * (unsigned long long)(c.n - 1) / 2;
  int st = c.status;
  if (st >= 0 && c.overflow) st = LMS_ERR_CAPACITY;
  if (st >= 0 && c.all_x_equal) st = LMS_OK_DEGENERATE;
  if (st >= 0 && !(b.w < INFINITY)) st = LMS_ERR_DEVICE;
  o.status = st;
  if (st < 0) {
    o.theta1 = o.theta2 = o.half_width = o.width = o.z_lo = o.z_hi = NAN;
    o.pair_i = o.pair_j = -1;
  } else {
    o.theta1 = b.th;
    o.theta2 = 0.5 * (b.lo + b.hi);
    o.width = b.w;
    o.half_width = 0.5 * b.w;
    o.z_lo = b.lo;
    o.z_hi = b.hi;
    o.pair_i = b.a == kDegenerate ? -1 : (int)b.a;
    o.pair_j = b.b == kDegenerate ? -1 : (int)b.b;
  }
  o.vertical = c.all_x_equal ? pairs : s_stat[ST_VERT];
  o.candidates = pairs - o.vertical;
  o.survivors = c.n_entries > (unsigned)c.n_seeds ? c.n_entries - (unsigned)c.n_seeds : 0u;
  o.point_evals = s_stat[ST_EVALS];
  o.dir_evals = s_stat[ST_DEVALS];
  o.band_pass = s_stat[ST_BAND];
  o.bin_pass = s_stat[ST_BIN];
  o.bins = c.n_live >= 0 ? (unsigned long long)kPrunedBins : c.bins;
  *out = o;
}

constexpr int kFinalNT = 256;
__global__ __launch_bounds__(kFinalNT) void k_finalize(Ctx* ctx, const uint2* __restrict__ entries,
                                                       const double4* __restrict__ res, int cap,
                                                       lms_result* out) {
  finalize_block<kFinalNT>(ctx, entries, res, cap, out);
}

// ---------------------------------------------------------------- FP64 window

// One block per entry [begin, min(n_entries, cap)): re-evaluates the pair's
// slope in FP64. With update_bound, also lowers the width bound.
template <int N2, int NT>
__device__ __forceinline__ void recheck_body(const double* __restrict__ xy, Ctx* ctx,
                                             const uint2* __restrict__ entries,
                                             double4* __restrict__ res, int begin, int cap,
                                             int update_bound) {
  __shared__ double z[N2];
  const Ctx c = *ctx;
  if (c.status < 0) return;
  const unsigned end = min(c.n_entries, (unsigned)cap);
  for (unsigned e = begin + blockIdx.x; e < end; e += gridDim.x) {
    const uint2 p = entries[e];
    double theta = 0.0;
    if (p.x != kDegenerate) {
      const double xl = xy[2 * p.x], xr = xy[2 * p.y];
      if (xl == xr) {
        if (threadIdx.x == 0) res[e] = make_double4(INFINITY, NAN, NAN, NAN);
        continue;
      }
      theta = (xy[2 * p.y + 1] - xy[2 * p.x + 1]) / (xr - xl);
    }
    double w, lo, hi;
    window_f64<N2, NT>(xy, c.n, c.h, theta, z, &w, &lo, &hi);
    if (threadIdx.x == 0) {
      res[e] = make_double4(w, theta, lo, hi);
      if (update_bound)
        atomicMin(&ctx->wbound,
                  (unsigned long long)__double_as_longlong(width_bound(w, theta, c.xabs, c.yabs)));
    }
  }
}

template <int N2, int NT>
__global__ __launch_bounds__(NT) void k_recheck(const double* __restrict__ xy, Ctx* ctx,
                                                const uint2* __restrict__ entries,
                                                double4* __restrict__ res, int begin, int cap,
                                                int update_bound) {
  recheck_body<N2, NT>(xy, ctx, entries, res, begin, cap, update_bound);
}

// The same re-evaluation split over several workgroups per entry, for
// n > kSplitChunk, to cut the latency of a few large sorts: workgroup
// (p, y) of k_sort_chunks sorts intercepts p C .. p C + C - 1 (+inf past n) of
// entry begin + y into tmp[y NP + p C ..]; workgroup y of k_merge_window then
// merges the NP / C sorted runs of entry begin + y and takes its narrowest
// window. Entries past the slots [begin, begin + slots) are re-evaluated whole
// by k_merge_window's workgroups in turn. Results equal k_recheck's: the
// sorted values are the same.
constexpr int kSplitChunk = 512;
constexpr int kSplitNT = 256;
constexpr int kSplitSlots = 512;  // entries per launch pair (tmp: slots x NP doubles)
constexpr int kFinalSlots = 128;       // split slots of the survivors' re-evaluation,
constexpr int kFinalSlotsLarge = 512;  // n > 4096 (a whole sort is slower there)

__device__ __forceinline__ bool entry_slope(const double* __restrict__ xy, uint2 p, double* theta) {
  *theta = 0.0;
  if (p.x == kDegenerate) return true;
  const double xl = xy[2 * p.x], xr = xy[2 * p.y];
  if (xl == xr) return false;
  *theta = (xy[2 * p.y + 1] - xy[2 * p.x + 1]) / (xr - xl);
  return true;
}

template <int C, int NT>
__global__ __launch_bounds__(NT) void k_sort_chunks(const double* __restrict__ xy,
                                                    const Ctx* ctx,
                                                    const uint2* __restrict__ entries, int begin,
                                                    int cap, int slots, double* __restrict__ tmp,
                                                    int np, const double* __restrict__ thetas) {
  constexpr int E = C / NT;
  __shared__ double z[C];
  if (ctx->status < 0) return;
  const unsigned end = min(thetas ? (unsigned)cap : min(ctx->n_entries, (unsigned)cap),
                           (unsigned)begin + (unsigned)slots);
  const int n = ctx->n, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k0 = blockIdx.x * C;
  for (unsigned y = blockIdx.y; begin + y < end; y += gridDim.y) {
    double theta = thetas ? thetas[begin + y] : 0.0;
    if (thetas ? !(theta == theta) : !entry_slope(xy, entries[begin + y], &theta)) continue;
    double v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int k = k0 + (wave * E + r) * 64 + lane;
      const double2 p = point_clamped(xy, k, n);
      v[r] = k < n ? fma(-theta, p.x, p.y) : INFINITY;
    }
    sort_regs<C, NT>(v, z);
    double* out = tmp + (size_t)y * np + k0;
#pragma unroll
    for (int r = 0; r < E; ++r) out[(wave * E + r) * 64 + lane] = v[r];
    __syncthreads();  // z is reused by the next entry's sort
  }
}

template <int NP, int NT>
__device__ __forceinline__ void merge_window_body(const double* __restrict__ xy, Ctx* ctx,
                                                  const uint2* __restrict__ entries,
                                                  double4* __restrict__ res, int begin, int cap,
                                                  int update_bound,
                                                  const double* __restrict__ tmp, int slots,
                                                  const double* __restrict__ thetas) {
  __shared__ double z[NP + NP / 16];  // merge_slot layout (NP for whole sorts)
  const Ctx c = *ctx;
  if (c.status < 0) return;
  const unsigned end = thetas ? (unsigned)cap : min(c.n_entries, (unsigned)cap);
  const unsigned split_end = min(end, (unsigned)begin + (unsigned)slots);
  auto finish = [&](unsigned e, double w, double theta, double lo, double hi) {
    if (threadIdx.x == 0) {
      res[e] = make_double4(w, theta, lo, hi);
      if (update_bound)
        atomicMin(&ctx->wbound,
                  (unsigned long long)__double_as_longlong(width_bound(w, theta, c.xabs, c.yabs)));
    }
  };
  for (unsigned e = begin + blockIdx.x; e < split_end; e += gridDim.x) {
    double theta = thetas ? thetas[e] : 0.0;
    if (thetas ? !(theta == theta) : !entry_slope(xy, entries[e], &theta)) {
      if (threadIdx.x == 0) res[e] = make_double4(INFINITY, NAN, NAN, NAN);
      continue;
    }
    const double* src = tmp + (size_t)(e - begin) * NP;
    {
      // all of a thread's loads in flight together, then the LDS stores
      constexpr int L = NP / NT;
      double v[L];
#pragma unroll
      for (int r = 0; r < L; ++r) v[r] = src[threadIdx.x + r * NT];
#pragma unroll
      for (int r = 0; r < L; ++r) z[merge_slot(threadIdx.x + r * NT)] = v[r];
    }
    __syncthreads();
    merge_runs<NP, NT>(z, kSplitChunk);
    double w, lo, hi;
    window_scan_at<NT>(z, merge_slot, c.n, c.h, &w, &lo, &hi);
    finish(e, w, theta, lo, hi);
  }
  for (unsigned e = split_end + blockIdx.x; e < end; e += gridDim.x) {
    double theta = thetas ? thetas[e] : 0.0;
    if (thetas ? !(theta == theta) : !entry_slope(xy, entries[e], &theta)) {
      if (threadIdx.x == 0) res[e] = make_double4(INFINITY, NAN, NAN, NAN);
      continue;
    }
    double w, lo, hi;
    window_f64<NP, NT>(xy, c.n, c.h, theta, z, &w, &lo, &hi);
    finish(e, w, theta, lo, hi);
  }
}

template <int NP, int NT>
__global__ __launch_bounds__(NT) void k_merge_window(const double* __restrict__ xy, Ctx* ctx,
                                                     const uint2* __restrict__ entries,
                                                     double4* __restrict__ res, int begin,
                                                     int cap, int update_bound,
                                                     const double* __restrict__ tmp, int slots,
                                                     const double* __restrict__ thetas) {
  merge_window_body<NP, NT>(xy, ctx, entries, res, begin, cap, update_bound, tmp, slots, thetas);
}

// Seed bounds. The screen needs only an upper bound W on the optimal width,
// and any window of h points at any slope gives one: so for each seed entry
// a window of at least h intercepts z_k = fma(-theta, x_k, y_k) is found
// without sorting. Level 1 counts the z in kSeedBins equal buckets over
// [min z, max z] and takes the shortest run of buckets holding h; each
// further level (LV in all) re-buckets the points of the previous run,
// widened by its length on either side, over their span and does the same.
// The window's ends are the smallest and largest z of the points in the
// final run (at least h of them), so its FP64 width z_hi - z_lo is at least
// F(theta) and, with the last level's buckets at about 1 / kSeedBins^LV of
// the z range, within a few of them of the narrowest h-window near the runs. The record
// (+inf, theta, z_lo, z_hi) keeps the entry out of the exact minimum (the
// optimal pair survives the screen at any W >= the optimal width); its
// window still serves the bin map's centre and window pairs. One workgroup
// per entry.
constexpr int kSeedBins = 4096;
constexpr int kSeedExactMax = 2048;  // smaller sets: exact seed windows (k_recheck)

// Shortest run of buckets [b, b + len) with P[b + len] - P[b] >= h in the
// exclusive prefix sums P[0..NB] (lowest b on ties), by the NT threads;
// len = INT_MAX if there is none. Each thread takes NB / NT consecutive
// starts; once it has a run of length L, a start needs a binary search only
// if one read shows a shorter run from it.
template <int NB, int NT>
__device__ __forceinline__ void shortest_run(const unsigned* P, unsigned h, int* b_out,
                                             int* len_out) {
  constexpr int S = NB / NT;
  const int b0 = threadIdx.x * S;
  const unsigned top = P[NB];
  double best = INFINITY;  // run length, as a double for block_argmin
  int bb = INT_MAX;
  for (int b = b0; b < b0 + S; ++b) {
    const unsigned pb = P[b];
    if (top - pb < h) break;  // no run from here on
    int hi = NB;
    if (bb != INT_MAX) {
      hi = min(b + (int)best - 1, NB);
      if (P[hi] - pb < h) continue;  // nothing shorter from b
    }
    int lo = b + 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (P[mid] - pb >= h) hi = mid; else lo = mid + 1;
    }
    best = lo - b;
    bb = b;
  }
  block_argmin<NT>(best, bb);
  *b_out = bb;
  *len_out = bb == INT_MAX ? INT_MAX : (int)best;
}

// Exclusive prefix sums of hist[0..NB) into hist[0..NB] (hist[NB] = total)
// by the NT threads. Ends with a barrier.
template <int NB, int NT>
__device__ __forceinline__ void prefix_counts(unsigned* hist, unsigned* part) {
  constexpr int S = NB / NT;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  unsigned v[S];
  unsigned run = 0;
#pragma unroll
  for (int r = 0; r < S; ++r) { v[r] = run; run += hist[t * S + r]; }
  unsigned x = run;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    const unsigned y = __shfl_up(x, m);
    if (lane >= m) x += y;
  }
  if (lane == 63) part[wave] = x;
  __syncthreads();
  unsigned off = x - run;
  for (int w = 0; w < wave; ++w) off += part[w];
#pragma unroll
  for (int r = 0; r < S; ++r) hist[t * S + r] = v[r] + off;
  if (t == NT - 1) hist[NB] = off + run;
  __syncthreads();
}

template <int NT, int E, int LV>
__global__ __launch_bounds__(NT) void k_seed_bounds(const double* __restrict__ xy, Ctx* ctx,
                                                    const uint2* __restrict__ entries,
                                                    double4* __restrict__ res, int begin,
                                                    int cap, int update_bound) {
  constexpr int NB = kSeedBins;
  static_assert(E <= 32, "point mask is 32 bits");
  // E >= 16: the intercepts live in LDS (128 KiB at 16384 points), which
  // leaves the registers to the levels' counting and searches
  constexpr bool ZL = E >= 16;
  __shared__ unsigned hist[NB + 1];
  __shared__ double s_z[ZL ? NT * E : 1];
  __shared__ unsigned s_part[NT / 64];
  const Ctx c = *ctx;
  if (c.status < 0) return;
  const unsigned end = min(c.n_entries, (unsigned)cap);
  const int n = c.n, t = threadIdx.x;
  for (unsigned e = begin + blockIdx.x; e < end; e += gridDim.x) {
    double theta;
    if (!entry_slope(xy, entries[e], &theta)) {
      if (t == 0) res[e] = make_double4(INFINITY, NAN, NAN, NAN);
      continue;
    }
    // the thread's intercepts z_k, k = t + r NT: in registers, or in LDS
    double zr[ZL ? 1 : E];
    auto zat = [&](int r) -> double { return ZL ? s_z[t + r * NT] : zr[r]; };
    unsigned alive = 0u;  // bit r: z_k is in the current level's domain
    double zmn = INFINITY, zmx = -INFINITY;
    constexpr int G = E < 8 ? E : 8;  // loads in flight together
#pragma unroll
    for (int r0 = 0; r0 < E; r0 += G) {
      double2 p[G];
#pragma unroll
      for (int g = 0; g < G; ++g) p[g] = point_clamped(xy, t + (r0 + g) * NT, n);
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int r = r0 + g, k = t + r * NT;
        const double z = k < n ? fma(-theta, p[g].x, p[g].y) : 0.0;
        if (ZL) s_z[k] = z;
        else zr[r] = z;
        if (k < n) {
          alive |= 1u << r;
          zmn = fmin(zmn, z);
          zmx = fmax(zmx, z);
        }
      }
    }
    block_min_max<NT>(zmn, zmx);
    double lo = zmn, hi = zmx;  // the whole set: n >= h points
    const double span = zmx - zmn;
    if (span > 0.0 && span < INFINITY) {
      // Level l < LV buckets its domain over [za, za + NB / sc). The next domain
      // is the run widened by its length on either side, so that a narrowest
      // window which the run's bucket edges cut stays whole; it holds the
      // run's h points, so every level finds a run (else the whole range
      // stands).
      double za = zmn, sc = NB / span;
      int r0 = 0, len = NB;
      auto bucket = [&](double v) { return (int)fmin(fmax((v - za) * sc, 0.0), (double)(NB - 1)); };
      for (int l = 0; l < LV; ++l) {
        for (int b = t; b <= NB; b += NT) hist[b] = 0u;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < E; ++r)
          if ((alive >> r) & 1u) atomicAdd(&hist[bucket(zat(r))], 1u);
        __syncthreads();
        prefix_counts<NB, NT>(hist, s_part);
        shortest_run<NB, NT>(hist, (unsigned)c.h, &r0, &len);
        if (len == INT_MAX) break;
        const bool last = l + 1 == LV;
        const int q0 = last ? r0 : max(r0 - len, 0), q1 = last ? r0 + len : min(r0 + 2 * len, NB);
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const int b = bucket(zat(r));
          if (b < q0 || b >= q1) alive &= ~(1u << r);
        }
        if (!last) {
          const double w = (q1 - q0) / sc;
          za += q0 / sc;
          sc = w > 0.0 ? NB / w : 0.0;
        }
      }
      // the last run's own points: their smallest and largest z
      double mn = INFINITY, mx = -INFINITY;
#pragma unroll
      for (int r = 0; r < E; ++r)
        if ((alive >> r) & 1u) { mn = fmin(mn, zat(r)); mx = fmax(mx, zat(r)); }
      block_min_max<NT>(mn, mx);
      if (len != INT_MAX) {
        lo = mn;
        hi = mx;
      }
    }
    if (t == 0) {
      res[e] = make_double4(INFINITY, theta, lo, hi);
      const double w = hi - lo;
      if (update_bound && w >= 0.0 && w < INFINITY)
        atomicMin(&ctx->wbound,
                  (unsigned long long)__double_as_longlong(width_bound(w, theta, c.xabs, c.yabs)));
    }
    __syncthreads();  // hist is reused by the next entry
  }
}

// Seed bounds of entries [begin, min(n_entries, cap)), `grid` workgroups of
// 1024 threads, each holding E intercepts (the levels are latency-bound:
// more threads shorten each one's share of the counts, sums and searches).
// Two levels up to 4096 points, three above: the larger sets' screen is more
// sensitive to a bound a few 1e-4 loose, and a level costs about 8 us.
void launch_seed_bounds(hipStream_t s, int n, int grid, const double* xy, Ctx* ctx,
                        const uint2* e, double4* res, int begin, int cap, int upd) {
  if (n <= 1024)
    hipLaunchKernelGGL((k_seed_bounds<1024, 1, 2>), dim3(grid), dim3(1024), 0, s, xy, ctx, e, res, begin, cap, upd);
  else if (n <= 4096)
    hipLaunchKernelGGL((k_seed_bounds<1024, 4, 2>), dim3(grid), dim3(1024), 0, s, xy, ctx, e, res, begin, cap, upd);
  else
    hipLaunchKernelGGL((k_seed_bounds<1024, 16, 3>), dim3(grid), dim3(1024), 0, s, xy, ctx, e, res, begin, cap, upd);
}

// ---------------------------------------------------------------- slope range
//
// A pair can be optimal only if its slope theta has F(theta) <= W: its
// anchored window of width W holds h points. F is Lipschitz in theta with
// constant xr (each intercept moves by (theta - theta') x_k), so an exact
// F(theta_g) > W excludes the slopes within (F(theta_g) - W) / xr of
// theta_g. And for |theta| >= |theta_g| of the same sign,
// F(theta) >= F(theta_g) - yr (F(theta) / |theta| is the narrowest window of
// y / theta - x, Lipschitz in 1 / theta with constant yr). kGridSide slopes
// on either side of the best seed slope tc, at offsets d0 2^k, are evaluated
// exactly; where their exclusions join up from the far end inwards, the
// slopes beyond are ruled out, which leaves [th_lo, th_hi] around tc.
constexpr int kGridSide = 16;
constexpr int kGrid = 2 * kGridSide;

// Grid slopes: entry 2k at tc + d0 2^k, entry 2k + 1 at tc - d0 2^k, with d0
// 2^-13 of the y / x aspect ratio. One block.
template <int NT>
__global__ __launch_bounds__(NT) void k_grid_slopes(const Ctx* ctx, const double4* seed_res,
                                                    int n_res, const double4* seed_rec,
                                                    int n_rec, double* grid_theta) {
  const double tc = best_slope<NT>(seed_res, n_res, seed_rec, n_rec);
  const Ctx& c = *ctx;
  const double d0 = c.xh > 0.0 && c.yh > 0.0 ? 0x1p-13 * (c.yh / c.xh) : 0x1p-13;
  if (threadIdx.x < kGridSide) {
    const double d = ldexp(d0, threadIdx.x);
    grid_theta[2 * threadIdx.x] = tc + d;
    grid_theta[2 * threadIdx.x + 1] = tc - d;
  }
}

// [lo, hi] from the grid's exact windows (width in .x, as in k_recheck; NaN
// or +inf widths exclude nothing) against the bound W, by the whole block
// (all threads call; the result goes to every thread); (-inf, +inf) when the
// far grid slopes are not ruled out. With `refine`, entries kGrid..2 kGrid-1
// are a second grid, of ascending slopes inside the range, whose exclusions
// then move the range's ends inwards.
template <int NT>
__device__ void slope_range(const Ctx& c, double W, const double* __restrict__ grid_theta,
                            const double4* __restrict__ grid_res, bool refine, double* lo_out,
                            double* hi_out) {
  static_assert(NT >= 2 * kGrid, "one thread per grid slope");
  __shared__ double s_t[2 * kGrid], s_m[2 * kGrid], s_r[2 * kGrid], s_lohi[2];
  const int t = threadIdx.x;
  const bool usable = W < INFINITY && c.xr > 0.0 && c.xr < INFINITY && c.yr < INFINITY;
  if (usable && t < (refine ? 2 * kGrid : kGrid)) {
    // lower bound of the exact width at grid slope t, minus W, and the
    // radius it excludes
    const double th = grid_theta[t], w = grid_res[t].x;
    const double err = 4.0 * 0x1p-53 * (c.yabs + fabs(th) * c.xabs);
    const double m = w < INFINITY ? (w - err) * (1.0 - 0x1p-50) - W : -1.0;
    s_t[t] = th;
    s_m[t] = m;
    s_r[t] = m > 0.0 ? m / c.xr * (1.0 - 0x1p-40) : 0.0;
  }
  __syncthreads();
  if (t == 0) {
    double lo = -INFINITY, hi = INFINITY;
    if (usable) {
      {  // upper side: entries 2k
        const int far = 2 * (kGridSide - 1);
        if (s_t[far] > 0.0 && s_m[far] > c.yr * (1.0 + 0x1p-40)) {
          double from = s_t[far] - s_r[far];
          for (int k = kGridSide - 2; k >= 0; --k) {
            const double r = s_r[2 * k], th = s_t[2 * k];
            if (!(r > 0.0) || th + r < from) break;
            from = fmin(from, th - r);
          }
          hi = from;
        }
      }
      {  // lower side: entries 2k + 1
        const int far = 2 * (kGridSide - 1) + 1;
        if (s_t[far] < 0.0 && s_m[far] > c.yr * (1.0 + 0x1p-40)) {
          double to = s_t[far] + s_r[far];
          for (int k = kGridSide - 2; k >= 0; --k) {
            const double r = s_r[2 * k + 1], th = s_t[2 * k + 1];
            if (!(r > 0.0) || th - r > to) break;
            to = fmax(to, th + r);
          }
          lo = to;
        }
      }
    }
    if (!(lo < hi)) {  // (never, as the best seed slope is not excluded)
      lo = -INFINITY;
      hi = INFINITY;
    }
    if (refine && lo > -INFINITY && hi < INFINITY) {
      // from each end inwards, while the second grid's exclusions join up
      double a = lo, b = hi;
      for (int k = kGrid; k < 2 * kGrid; ++k) {
        const double r = s_r[k], th = s_t[k];
        if (r > 0.0 && th - r <= a) a = fmax(a, th + r);
        else if (!(th + r < a)) break;
      }
      for (int k = 2 * kGrid - 1; k >= kGrid; --k) {
        const double r = s_r[k], th = s_t[k];
        if (r > 0.0 && th + r >= b) b = fmin(b, th - r);
        else if (!(th - r > b)) break;
      }
      if (a < b) {  // (always, as above)
        lo = a;
        hi = b;
      }
    }
    s_lohi[0] = lo;
    s_lohi[1] = hi;
  }
  __syncthreads();
  *lo_out = s_lohi[0];
  *hi_out = s_lohi[1];
}

// The pruned screen spreads a slope range over kPrunedBins bins (defined
// with the Ctx); a range so wide that their centre would be over 4 times
// coarser than the full screen's (NB bins, scale kBinMag x-range / y-range)
// stays with the full screen.
__device__ bool narrow_range(const Ctx& c, double lo, double hi) {
  if (!(lo > -INFINITY && hi < INFINITY) || c.bins == 0u) return false;
  const unsigned nb = 1u << (31 - __builtin_clz(c.bins));
  const double sc_full = fmin(fmax(c.yh > 0.0 ? kBinMag * c.xh / c.yh : 1.0, 0x1p-100), 0x1p100);
  const double dl = 0.5 * (hi - lo);
  return 3.0 / dl * 4.0 >= sc_full * (double)(nb / kPrunedBins);
}

// Second grid: kGrid ascending slopes spread over the range of the first
// grid's windows against the bound they left; NaN (the windows of the grid
// kernels skip them) when that range is not narrow enough to prune with.
// One block.
__global__ __launch_bounds__(64) void k_grid_refine(const Ctx* ctx, double* grid_theta,
                                                    const double4* grid_res) {
  const Ctx c = *ctx;
  const double W = __longlong_as_double((long long)c.wbound);
  const double Wl = W * (1.0 + 0x1p-50) * (1.0 + 0x1p-40);
  double lo = -INFINITY, hi = INFINITY;
  if (c.status == LMS_OK && !c.all_x_equal)
    slope_range<64>(c, Wl, grid_theta, grid_res, false, &lo, &hi);
  const int t = threadIdx.x;
  if (t < kGrid)
    grid_theta[kGrid + t] = narrow_range(c, lo, hi) ? lo + (t + 0.5) * ((hi - lo) / kGrid) : NAN;
}

// Anchors the slope range leaves. With th in [lo, hi] = [tm - dl, tm + dl], a
// point's residual from anchor i, Dy - th Dx, is within dl xr of its value
// at tm, which is the difference of the keys z = y - tm x. So the points
// that can be in the anchor's upper window [0, W] at a slope of the range
// have keys in [z_i - s, z_i + W + s], s = dl xr (plus the keys' roundings),
// and those of the lower window [-W, 0] in [z_i - W - s, z_i + s]. An anchor
// whose key intervals hold fewer than h points each is in no pair that can
// be optimal; a pair's partner has its key in the anchor's intervals too.
//
// Block 0 sorts the points into kRangeBuckets buckets of equal key width
// (counting sort: perm lists the points bucket by bucket, sxy holds them in
// that order) and lists the anchors that are left, each with the range
// [r0, r1) of perm that covers the intervals that can reach h (whole
// buckets: a superset). The other workgroups count the vertical pairs
// (equal x), which the pruned screen no longer meets: equal x share a bucket
// of a hash of their bits (-0 taken as +0), so a counting sort by that hash
// and compares within each bucket find them all. Without a finite range
// nothing changes.
constexpr int kRangeBuckets = 4096;
constexpr int kRangeMinN = 4096, kRefineMinN = 8192;

// Exclusive prefix sum of the kRangeBuckets counts in cur into start and cur
// (insertion cursors); start[kRangeBuckets] = the total. All NT threads call;
// ends with a barrier.
template <int NT>
__device__ void bucket_starts(unsigned* start, unsigned* cur, unsigned* part) {
  constexpr int S = kRangeBuckets / NT;
  static_assert(S * NT == kRangeBuckets, "buckets per thread");
  const int t = threadIdx.x, lane = t & 63;
  unsigned v[S], run = 0;
#pragma unroll
  for (int r = 0; r < S; ++r) {
    v[r] = run;
    run += cur[t * S + r];
  }
  unsigned x = run;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    const unsigned y = __shfl_up(x, m);
    if (lane >= m) x += y;
  }
  if (lane == 63) part[t >> 6] = x;
  __syncthreads();
  unsigned off = x - run;
  for (int w = 0; w < (t >> 6); ++w) off += part[w];
#pragma unroll
  for (int r = 0; r < S; ++r) {
    start[t * S + r] = v[r] + off;
    cur[t * S + r] = v[r] + off;
  }
  if (t == NT - 1) start[kRangeBuckets] = off + run;
  __syncthreads();
}

template <int NT, int E>
__global__ __launch_bounds__(NT) void k_range(const double* __restrict__ xy, Ctx* ctx,
                                              const double* __restrict__ grid_theta,
                                              const double4* __restrict__ grid_res,
                                              bool refine, unsigned* __restrict__ perm,
                                              double2* __restrict__ sxy,
                                              uint2* __restrict__ live) {
  __shared__ unsigned s_start[kRangeBuckets + 1], s_cur[kRangeBuckets];
  __shared__ unsigned s_part[NT / 64];
  __shared__ unsigned s_live;
  __shared__ unsigned short s_xperm[LMS_MAX_N];
  const Ctx c = *ctx;
  if (c.status != LMS_OK || c.all_x_equal) return;
  const int n = c.n, h = c.h, t = threadIdx.x, lane = t & 63;
  const double W = __longlong_as_double((long long)c.wbound);
  // the bins count the windows of width W (1 + 2^-50)
  const double Wl = W * (1.0 + 0x1p-50) * (1.0 + 0x1p-40);
  double lo, hi;
  slope_range<NT>(c, Wl, grid_theta, grid_res, refine, &lo, &hi);
  if (!(lo > -INFINITY && hi < INFINITY)) return;  // n_live stays -1
  {  // the pairs' computed slopes carry a relative error below 2^-39
    const double m = 0x1p-30 * fmax(fabs(lo), fabs(hi)) + 0x1p-1000;
    lo -= m;
    hi += m;
  }
  if (!narrow_range(c, lo, hi)) return;
  if (blockIdx.x > 0) {
    // vertical pairs (i < j, x_i == x_j): every one of these workgroups
    // hashes all x, then takes its share of the hash-ordered positions
    auto hb = [](double x) {
      const unsigned long long u = (unsigned long long)__double_as_longlong(x + 0.0);
      return (int)((u * 0x9E3779B97F4A7C15ull) >> (64 - 12));
    };
    static_assert(kRangeBuckets == 1 << 12, "hash buckets");
    for (int b = t; b < kRangeBuckets; b += NT) s_cur[b] = 0u;
    int hk[E];  // the thread's points' hash buckets (loads all in flight together)
    {
      double xk[E];
#pragma unroll
      for (int e = 0; e < E; ++e) xk[e] = xy[2 * min(t + e * NT, n - 1)];
#pragma unroll
      for (int e = 0; e < E; ++e) hk[e] = hb(xk[e]);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (t + e * NT < n) atomicAdd(&s_cur[hk[e]], 1u);
    __syncthreads();
    bucket_starts<NT>(s_start, s_cur, s_part);
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (t + e * NT < n) s_xperm[atomicAdd(&s_cur[hk[e]], 1u)] = (unsigned short)(t + e * NT);
    __syncthreads();
    unsigned long long cnt = 0;
    const int nv = (int)gridDim.x - 1;
    for (int p = (blockIdx.x - 1) * NT + t; p < n; p += nv * NT) {
      const double xk = xy[2 * s_xperm[p]];
      const int end = (int)s_start[hb(xk) + 1];
      for (int q = p + 1; q < end; ++q) cnt += xy[2 * s_xperm[q]] == xk ? 1u : 0u;
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) cnt += __shfl_xor(cnt, m);
    if (lane == 0) stat_add(ctx, ST_VERT, cnt);
    return;
  }
  const double tm = lo + 0.5 * (hi - lo);
  const double dl = fmax(hi - tm, tm - lo) * (1.0 + 0x1p-40);
  // two key roundings, each below 2^-53 (|y| + |tm| |x|)
  const double s = dl * c.xr * (1.0 + 0x1p-40) + 8.0 * 0x1p-53 * (c.yabs + fabs(tm) * c.xabs);
  // only the keys stay in registers (points are read again for the copy)
  double z[E];
  double mn = INFINITY, mx = -INFINITY;
#pragma unroll
  for (int e0 = 0; e0 < E; e0 += 8) {  // up to 8 loads in flight together
    constexpr int G = E < 8 ? E : 8;
    double2 pt[G];
#pragma unroll
    for (int g = 0; g < G; ++g) pt[g] = point_clamped(xy, t + (e0 + g) * NT, n);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int e = e0 + g, k = t + e * NT;
      z[e] = k < n ? fma(-tm, pt[g].x, pt[g].y) : 0.0;
      if (k < n) {
        mn = fmin(mn, z[e]);
        mx = fmax(mx, z[e]);
      }
    }
  }
  block_min_max<NT>(mn, mx);
  // bucket of a key: monotone in the key (a rounded difference, a rounded
  // product by sc >= 0, truncation, clamps), so a key interval maps into the
  // buckets between those of its ends
  const double span = mx - mn;
  const double sc = span > 0.0 && span < INFINITY ? kRangeBuckets / span : 0.0;
  auto bucket = [&](double v) {
    const double f = (v - mn) * sc;
    return f >= (double)(kRangeBuckets - 1) ? kRangeBuckets - 1 : (f > 0.0 ? (int)f : 0);
  };
  for (int b = t; b < kRangeBuckets; b += NT) s_cur[b] = 0u;
  if (t == 0) s_live = 0u;
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e)
    if (t + e * NT < n) atomicAdd(&s_cur[bucket(z[e])], 1u);
  __syncthreads();
  bucket_starts<NT>(s_start, s_cur, s_part);
  __syncthreads();
  // anchors left, with the perm range of the intervals that can reach h
  // (before the copy, so that the keys are dead by then)
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = t + e * NT;
    bool keep = false;
    unsigned r0 = 0, r1 = 0;
    if (i < n) {
      const double zi = z[e];
      // interval ends, rounded outwards past the subtraction's rounding
      const double g = 0x1p-50 * (fabs(zi) + Wl + s);
      const int bA = bucket(zi - Wl - s - g), bB = bucket(zi - s - g);
      const int bC = bucket(zi + s + g), bD = bucket(zi + Wl + s + g);
      const unsigned cD = s_start[bC + 1] - s_start[bA], cU = s_start[bD + 1] - s_start[bB];
      const bool okU = cU >= (unsigned)h, okD = cD >= (unsigned)h;
      keep = okU || okD;
      r0 = okD ? s_start[bA] : s_start[bB];
      r1 = okU ? s_start[bD + 1] : s_start[bC + 1];
    }
    const unsigned long long mk = lane_mask(keep);
    if (mk) {
      unsigned base = 0;
      if (lane == 0) base = atomicAdd(&s_live, (unsigned)__popcll(mk));
      base = __shfl(base, 0);
      if (keep) live[base + __popcll(mk & ((1ull << lane) - 1ull))] = make_uint2((unsigned)i, r0 | (r1 << 16));
    }
  }
  // the sorted copy: positions first, then every point load at once
  unsigned pos[E];
#pragma unroll
  for (int e = 0; e < E; ++e)
    pos[e] = t + e * NT < n ? atomicAdd(&s_cur[bucket(z[e])], 1u) : 0u;
#pragma unroll
  for (int e0 = 0; e0 < E; e0 += 8) {  // up to 8 loads in flight together
    constexpr int G = E < 8 ? E : 8;
    double2 pt[G];
#pragma unroll
    for (int g = 0; g < G; ++g) pt[g] = point_clamped(xy, t + (e0 + g) * NT, n);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int e = e0 + g, k = t + e * NT;
      if (k < n) {
        perm[pos[e]] = (unsigned)k;
        sxy[pos[e]] = pt[g];
      }
    }
  }
  __syncthreads();
  if (t == 0) {
    ctx->th_lo = lo;
    ctx->th_hi = hi;
    ctx->n_live = (int)s_live;
  }
}

void launch_range(hipStream_t s, int n, int cu, const double* xy, Ctx* ctx,
                  const double* grid_theta, const double4* grid_res, bool refine,
                  unsigned* perm, double2* sxy, uint2* live) {
  // block 0: buckets and anchors; the others: vertical pairs, 1024 positions each
  const int grid = 1 + std::max(1, (n + 1023) / 1024);
  (void)cu;
  if (n <= 1024)
    hipLaunchKernelGGL((k_range<1024, 1>), dim3(grid), dim3(1024), 0, s, xy, ctx, grid_theta, grid_res, refine, perm, sxy, live);
  else if (n <= 4096)
    hipLaunchKernelGGL((k_range<1024, 4>), dim3(grid), dim3(1024), 0, s, xy, ctx, grid_theta, grid_res, refine, perm, sxy, live);
  else
    hipLaunchKernelGGL((k_range<1024, 16>), dim3(grid), dim3(1024), 0, s, xy, ctx, grid_theta, grid_res, refine, perm, sxy, live);
}

// F(theta) at arbitrary slopes (seed slopes and lms_eval_slopes).
template <int N2, int NT>
__global__ __launch_bounds__(NT) void k_eval_slopes(const double* __restrict__ xy, int n, int h,
                                                    const double* __restrict__ theta, int m,
                                                    double* __restrict__ out, Ctx* ctx,
                                                    double4* __restrict__ rec) {
  __shared__ double z[N2];
  if (ctx) {
    if (ctx->status < 0) return;
  }
  for (int e = blockIdx.x; e < m; e += gridDim.x) {
    const double th = theta[e];
    double w, lo, hi;
    window_f64<N2, NT>(xy, n, h, th, z, &w, &lo, &hi);
    if (threadIdx.x == 0) {
      if (out) { out[3 * e] = w; out[3 * e + 1] = lo; out[3 * e + 2] = hi; }
      if (rec) rec[e] = make_double4(w, th, lo, hi);
      if (ctx && isfinite(th))
        atomicMin(&ctx->wbound, (unsigned long long)__double_as_longlong(width_bound(w, th, ctx->xabs, ctx->yabs)));
    }
  }
}

// ---------------------------------------------------------------- window pairs

// Seed pairs from a candidate line: of m candidate windows (width, theta,
// z_lo, z_hi), take the narrowest, list the points whose FP64 intercept
// fma(-theta, x, y) lies in it (its h points, plus any tied at its ends) in
// index order, and draw `count` pairs among them into entries [first,
// first + count). When the line is close to the LMS line, most of those
// points are inliers, and a pair of them has a slope near the optimum, so
// its exact width tightens the bound far more than a random pair's.
constexpr int kWinNT = 1024;
__global__ __launch_bounds__(kWinNT) void k_window_pairs(const double* __restrict__ xy,
                                                         const Ctx* ctx,
                                                         const double4* __restrict__ cand, int m,
                                                         uint2* __restrict__ entries, int first,
                                                         int count, unsigned long long key) {
  __shared__ int list[LMS_MAX_N];
  __shared__ int s_wave[kWinNT / 64];
  __shared__ int s_best;
  const Ctx c = *ctx;
  if (c.status != LMS_OK || c.all_x_equal) return;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (t == 0) {  // narrowest window (z_hi - z_lo: exact or a seed bound's)
    int b = -1;
    for (int k = 0; k < m; ++k) {
      const double wk = cand[k].w - cand[k].z;
      if (wk < INFINITY && (b < 0 || wk < cand[b].w - cand[b].z)) b = k;
    }
    s_best = b;
  }
  __syncthreads();
  const int b = s_best;
  if (b < 0) return;  // no finite window: the slots keep the extreme-x pair
  const double4 w = cand[b];
  int total = 0;
  for (int base = 0; base < c.n; base += kWinNT) {
    const int k = base + t;
    bool in = false;
    if (k < c.n) {
      const double z = fma(-w.y, xy[2 * k], xy[2 * k + 1]);
      in = z >= w.z && z <= w.w;
    }
    const unsigned long long mk = __ballot(in);
    if (lane == 0) s_wave[wave] = __popcll(mk);
    __syncthreads();
    int before = total;
    for (int v = 0; v < wave; ++v) before += s_wave[v];
    if (in) list[before + __popcll(mk & ((1ull << lane) - 1ull))] = k;
    for (int v = 0; v < kWinNT / 64; ++v) total += s_wave[v];
    __syncthreads();
  }
  if (total < 2) return;
  for (int e = t; e < count; e += kWinNT) {
    const unsigned long long r = mix64(key + 0x9E3779B97F4A7C15ull * (unsigned long long)(e + 1));
    const int a = (int)((r >> 32) % (unsigned long long)total);
    int d = (int)((r & 0xFFFFFFFFull) % (unsigned long long)(total - 1));
    if (d >= a) ++d;
    const unsigned u = (unsigned)list[a], v = (unsigned)list[d];
    entries[first + e] = make_uint2(min(u, v), max(u, v));
  }
}

// ---------------------------------------------------------------- screen
//
__device__ __forceinline__ void append_entry(Ctx* ctx, uint2* entries, int cap, unsigned lo,
                                             unsigned hi) {
  const unsigned idx = atomicAdd(&ctx->n_entries, 1u);
  if (idx < (unsigned)cap) entries[idx] = make_uint2(lo, hi);
  else atomicOr(&ctx->overflow, 1u);
}

// Work item = (anchor i, block of G*64 partner offsets). Partners are
// j = (i + o) mod n for o = 1..P(i): every unordered pair appears once.
// fallback = 1: runs only if the slope-bin screen's list overflowed, which
// then has already counted and listed the vertical and forced pairs.
template <int R, bool LDS_PART, int NT>
__device__ __forceinline__ void screen_exhaustive(
    const double* __restrict__ xy, const float2* __restrict__ xy32, Ctx* ctx,
    uint2* __restrict__ entries, int cap, int G, int ipa, int n_items, int nq, int fallback) {
  extern __shared__ float2 lds[];
  const Ctx c = *ctx;
  if (c.status != LMS_OK || c.all_x_equal) return;
  if (fallback && !c.cand_overflow) return;
  const int n = c.n, h = c.h, lane = threadIdx.x & 63;
  if (LDS_PART) {
    for (int k = threadIdx.x; k < nq * 64; k += blockDim.x) lds[k] = xy32[64 * R + k];
    __syncthreads();
  }
  const double W = __longlong_as_double((long long)c.wbound);
  const int half = n >> 1;
  unsigned long long n_vert = 0, n_scr = 0, n_evals = 0, n_devals = 0, n_forced = 0;
  unsigned n_band = 0;
  for (;;) {
    int item = 0;
    if (lane == 0) item = (int)atomicAdd(&ctx->next_item, 1u);
    item = __shfl(item, 0);
    if (item >= n_items) break;
    const int i = item / ipa, blk = item - (item / ipa) * ipa;
    const float2 pi = xy32[i];
    // Reload the points for every item: an opaque base pointer keeps the
    // compiler from hoisting the loads and holding a second register copy.
    const float2* src = xy32;
    asm volatile("" : "+s"(src));
    float X[R], Y[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float2 p = src[lane + 64 * r];
      X[r] = p.x - pi.x;
      Y[r] = p.y - pi.y;
    }
    const int P = (n & 1) ? half : (i < half ? half : half - 1);
    for (int g = 0; g < G; ++g) {
      const int o = 1 + (blk * G + g) * 64 + lane;
      const bool valid = o <= P;
      int j = i + (valid ? o : 1);
      if (j >= n) j -= n;
      const int lo = min(i, j), hi = max(i, j);
      const double xl = xy[2 * lo], yl = xy[2 * lo + 1];
      const double xr = xy[2 * hi], yr = xy[2 * hi + 1];
      const bool vert = valid && (xl == xr);
      const double th = (yr - yl) / (xr - xl);
      const ScreenScalars sc = screen_scalars(th, W, c.fx, c.fy, c.xh, c.yh);
      const bool force = valid && !vert && sc.force;
      const bool test = valid && !vert && !force;
      const float th32 = test ? sc.th32 : 0.0f;
      const float thr = test ? sc.thr : 0.0f;
      const float ta = test ? sc.ta : 0.0f;
      const float nc = test ? -fmaf(-th32, pi.x, pi.y) : 0.0f;
      unsigned long long m = __ballot(test);
      if (!fallback) {
        n_vert += __popcll(__ballot(vert));
        n_forced += __popcll(__ballot(force));
        if (force) append_entry(ctx, entries, cap, (unsigned)lo, (unsigned)hi);
        n_scr += __popcll(m);
      }
      // With the LDS part, two candidates at a time while at least two remain:
      // each LDS read then serves both. (Registers only, the pairing's extra
      // scalar registers cost more than the overlap gains.)
      while (LDS_PART && (m & (m - 1))) {
        const int ca = __ffsll((long long)m) - 1;
        m &= m - 1;
        const int cb = __ffsll((long long)m) - 1;
        m &= m - 1;
        const PairTest2 pt = test_pair2<R, LDS_PART>(
            X, Y, lds, nq, -lane_f(th32, ca), lane_f(thr, ca), lane_f(ta, ca), lane_f(nc, ca),
            -lane_f(th32, cb), lane_f(thr, cb), lane_f(ta, cb), lane_f(nc, cb), h);
        n_evals += (unsigned)(pt.a.band_chunks + pt.b.band_chunks);
        n_band += (pt.a.split_chunks >= 0) + (pt.b.split_chunks >= 0);
        n_devals += (unsigned)(max(pt.a.split_chunks, 0) + max(pt.b.split_chunks, 0));
        if (lane == 0) {
          if (pt.a.keep)
            append_entry(ctx, entries, cap, (unsigned)lane_i(lo, ca), (unsigned)lane_i(hi, ca));
          if (pt.b.keep)
            append_entry(ctx, entries, cap, (unsigned)lane_i(lo, cb), (unsigned)lane_i(hi, cb));
        }
      }
      while (m) {
        const int cl = __ffsll((long long)m) - 1;
        m &= m - 1;
        const float nth = -lane_f(th32, cl);
        const PairTest pt = test_pair<R, LDS_PART>(X, Y, lds, nq, nth, lane_f(thr, cl),
                                                   lane_f(ta, cl), lane_f(nc, cl), h);
        n_evals += (unsigned)pt.band_chunks;
        if (pt.split_chunks >= 0) {
          ++n_band;
          n_devals += (unsigned)pt.split_chunks;
        }
        const int keep = pt.keep;
        if (keep && lane == 0)
          append_entry(ctx, entries, cap, (unsigned)lane_i(lo, cl), (unsigned)lane_i(hi, cl));
      }
    }
  }
  if (lane == 0) {
    stat_add(ctx, ST_VERT, n_vert);
    stat_add(ctx, ST_SCREENED, n_scr);
    stat_add(ctx, ST_BAND, n_band);
    stat_add(ctx, ST_EVALS, 64ull * n_evals);
    stat_add(ctx, ST_DEVALS, 64ull * n_devals);
    stat_add(ctx, ST_FORCED, n_forced);
  }
}

template <int R, bool LDS_PART, int NT>
__global__ __launch_bounds__(NT, 3) void k_screen(
    const double* __restrict__ xy, const float2* __restrict__ xy32, Ctx* ctx,
    uint2* __restrict__ entries, int cap, int G, int ipa, int n_items, int nq, int fallback) {
  screen_exhaustive<R, LDS_PART, NT>(xy, xy32, ctx, entries, cap, G, ipa, n_items, nq, fallback);
}

// ---------------------------------------------------------------- slope-bin screen
//
// Anchor i, point k, Dx = x_k - x_i, Dy = y_k - y_i (exact reals). The anchored
// residual d_k(theta) = Dy - theta Dx lies in the upper window [0, W] for theta
// in one closed interval and in the lower window [-W, 0] for theta in the
// adjacent one; both end at the slope of (i, k). The pair (i, j) has window
// counts U = #{k : 0 <= d_k <= W} and D = #{k : -W <= d_k <= 0} at its slope,
// and the optimal pair, with the optimal slab's boundary through both its
// points (Section 3.3), has U >= h or D >= h for every W >= the optimal width.
// Per anchor the kernel adds every point's two intervals to a difference
// array of slope bins in LDS (a compact monotone map of the slope, centred
// on the best seed slope), takes its prefix sum, and reads the bounds on U and D of each partner from
// the bin of its slope. Each interval is widened by a rigorous bound on its
// FP64 rounding's effect on the bins and by two bins (rounding of the bin map
// and of the partner's slope), so a bin's count is never below the exact count of any slope in
// it. Pairs whose bound reaches h are listed for the FP32 test.

template <int NB, int NT, bool WIDE>
__global__ __launch_bounds__(NT) void k_bins(const double* __restrict__ xy, Ctx* ctx,
                                             uint2* __restrict__ cands, int cand_cap,
                                             uint2* __restrict__ entries, int cap,
                                             const double4* __restrict__ seed_res,
                                             const double4* __restrict__ seed_rec, int n_rec) {
  // NB + NT bins, an odd number per thread in the prefix sum, and one word
  // for the decrements past the last bin
  constexpr int NBINS = NB + NT;
  constexpr int kRLog = __builtin_ctz(NB) - 1;  // the map spans bins [3, NB + 3]
  static_assert((NB % NT) == 0 && ((NB / NT) & 1) == 0, "bins must be 2^k per thread");
  // Up to 2^14 bins the insertion also stores each point's query code
  // (add_point_bins_coded) and the queries only read it. Larger bin arrays
  // leave no LDS for the codes: the queries compute the pair's bin
  // themselves. Either way the queries list the passing partners' offsets.
  // WIDE: for sets of more than NB / 2 points (fewer bins than 2 n, so more
  // workgroups fit a CU); no codes then.
  constexpr bool CODED = NB <= 16384 && !WIDE;
  // point loads in flight in the insertion loop (latency: the largest bin
  // arrays leave the fewest wavefronts per CU)
  constexpr int kPF = NB >= 32768 ? 3 : 2;
  // (rounded up to whole 16-byte words for the clearing stores)
  __shared__ __align__(16) unsigned bins[(NBINS + 4) & ~3];
  // codes of the n <= NB / 2 points (CODED), or partner offsets o - 1 that
  // pass (P(i) <= n / 2 <= LMS_MAX_N / 2)
  __shared__ unsigned short list[WIDE || NB / 2 >= LMS_MAX_N / 2 ? LMS_MAX_N / 2 : NB / 2];
  // CODED: the partner offsets o - 1 that pass (P(i) <= n / 2 <= NB / 4)
  __shared__ unsigned short plist[CODED ? NB / 4 : 1];
  // passes of the block's anchors so far, written out together (one
  // reservation per flush instead of one per anchor)
  constexpr int PB = 512;
  __shared__ uint2 pbuf[PB];
  __shared__ unsigned s_part[NT / 64];
  __shared__ unsigned s_all, s_cnt, s_base, s_fill;
  const Ctx c = *ctx;
  if (c.status != LMS_OK || c.all_x_equal || c.n_live >= 0) return;  // (k_bins_pruned)
  const int n = c.n, h = c.h, t = threadIdx.x, lane = t & 63;
  const double W = __longlong_as_double((long long)c.wbound);
  const double lim = uniform(W * (1.0 + 0x1p-50));
  BinFrame F = bin_frame(best_slope<NT>(seed_res, c.n_seeds, seed_rec, n_rec),
                         c.xh, c.yh, W, NBINS);
  F.tc = uniform(F.tc);  // (uniform values in scalar registers)
  F.sc = uniform(F.sc);
  F.q = uniform(F.q);
  const int half = n >> 1;
  // slopes whose FP32 test bound (affine in |theta|) would pass 1e29 go to the
  // FP64 entries; half the solved limit covers the roundings
  const double th_lim = uniform(screen_th_lim(c.fx, c.fy, c.xh, c.yh));
  const double2* pts = reinterpret_cast<const double2*>(xy);
  // per-wavefront counts (uniform)
  unsigned long long n_vert = 0, n_scr = 0, n_forced = 0, n_pass = 0;
  // reserves cnt list slots (thread 0; the base goes to s_base)
  auto reserve = [&](unsigned cnt) {
    const unsigned base = atomicAdd(&ctx->n_cands, cnt);
    if (base + cnt > (unsigned)cand_cap || base + cnt < base) atomicOr(&ctx->cand_overflow, 1u);
    s_base = base;
  };
  auto flush = [&]() {  // all threads; leaves s_fill = 0
    __syncthreads();
    const unsigned fill = s_fill;
    if (fill) {
      if (t == 0) reserve(fill);
      __syncthreads();
      const unsigned base = s_base;
      for (unsigned q = t; q < fill; q += NT)
        if (base + q < (unsigned)cand_cap) cands[base + q] = pbuf[q];
      __syncthreads();
      if (t == 0) s_fill = 0;
      __syncthreads();
    }
  };
  if (t == 0) s_fill = 0;
  // anchors round-robin over the blocks (no shared counter)
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    __syncthreads();  // the previous anchor's queries are done with the bins
    if (t == 0) {
      s_all = 0;
      s_cnt = 0;
    }
    for (int b = t; b < (NBINS + 4) / 4; b += NT) reinterpret_cast<uint4*>(bins)[b] = uint4{};
    __syncthreads();
    // the anchor in VGPRs (a vector load): a scalar load's wait would also
    // wait for every LDS operation in flight in the loop below
    int iv = i;
    asm volatile("" : "+v"(iv));
    const double2 pa = pts[iv];
    const double xi = uniform(pa.x), yi = uniform(pa.y);
    // 1. intervals of every point (packed counts: U in the low, D in the high half)
    unsigned all = 0;
    // kPF points per step; the loads of the next step's points are issued
    // before this step's work (clamped indices: no branch around a load)
    auto load = [&](int k) { return pts[(unsigned)min(k, n - 1)]; };
    auto insert = [&](const double2& v, int k) {
      if (CODED)
        add_point_bins_coded<kRLog>(bins, v.x - xi, v.y - yi, W, lim, F, th_lim, &list[k], all);
      else
        add_point_bins<kRLog>(bins, v.x - xi, v.y - yi, W, lim, F, all);
    };
    double2 cur[kPF], nxt[kPF];
#pragma unroll
    for (int q = 0; q < kPF; ++q) cur[q] = load(t + q * NT);
    int k0 = t;
    // steps whose next points are all in range: no clamp, no bounds test
    for (; k0 + (2 * kPF - 1) * NT < n; k0 += kPF * NT) {
#pragma unroll
      for (int q = 0; q < kPF; ++q) nxt[q] = pts[(unsigned)(k0 + (kPF + q) * NT)];
#pragma unroll
      for (int q = 0; q < kPF; ++q) insert(cur[q], k0 + q * NT);
#pragma unroll
      for (int q = 0; q < kPF; ++q) cur[q] = nxt[q];
    }
    // the last steps
    for (; k0 < n; k0 += kPF * NT) {
#pragma unroll
      for (int q = 0; q < kPF; ++q) nxt[q] = load(k0 + (kPF + q) * NT);
#pragma unroll
      for (int q = 0; q < kPF; ++q)
        if (k0 + q * NT < n) insert(cur[q], k0 + q * NT);
#pragma unroll
      for (int q = 0; q < kPF; ++q) cur[q] = nxt[q];
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) all += __shfl_xor(all, m);
    if (lane == 0) atomicAdd(&s_all, all);
    __syncthreads();
    // 2. prefix sum of the difference array
    scan_bins<NBINS, NT>(bins, s_part);
    __syncthreads();
    // 3. partners: j = (i + o) mod n, o = 1..P(i). A pair's bin comes from
    //    its offset to the anchor as in add_point_bins; without the far-point
    //    check its error is still relative (below 2^-44), so it is within one
    //    of the exact bin. Pairs whose |Dx| is outside the reciprocal's range,
    //    or whose slope is beyond the FP32 test's, go to the FP64 entries.
    const unsigned pall = s_all;
    const int P = (n & 1) ? half : (i < half ? half : half - 1);
    auto partner = [&](int o) { return i + o >= n ? i + o - n : i + o; };
    if (CODED) {
      for (int o0 = 1; o0 <= P; o0 += NT) {
        const int o = o0 + t;
        const bool valid = o <= P;
        const int j = partner(min(o, P));
        const unsigned cj = list[j];
        // read for every lane, with no branch (codes 0..2 read bins 0..2,
        // which no test uses)
        const unsigned pb = bins[cj];
        const unsigned long long mv = lane_mask(valid);
        const unsigned long long mt = lane_mask(cj > kCodePass) & mv;
        const unsigned long long mf = lane_mask(cj == kCodeFP64) & mv;
        const unsigned long long mp = lane_mask(bins_pass(pb, pall, h)) & mt;
        n_vert += __popcll(lane_mask(cj == kCodeVertical) & mv);
        n_forced += __popcll(mf);
        n_scr += __popcll(mt);
        n_pass += __popcll(mp);
        const bool pass = (mp >> lane) & 1ull;
        if (mf && ((mf >> lane) & 1ull))
          append_entry(ctx, entries, cap, (unsigned)min(i, j), (unsigned)max(i, j));
        if (mp) {
          unsigned base = 0;
          if (lane == 0) base = atomicAdd(&s_cnt, (unsigned)__popcll(mp));
          base = __shfl(base, 0);
          if (pass) plist[base + __popcll(mp & ((1ull << lane) - 1ull))] = (unsigned short)(o - 1);
        }
      }
    } else {
      // kPF partners per step, the next step's loads issued first (as in 1.)
      const int Pc = max(P, 1);
      double2 pc[kPF], pnx[kPF];
#pragma unroll
      for (int q = 0; q < kPF; ++q) pc[q] = pts[partner(min(1 + t + q * NT, Pc))];
      for (int s0 = 1; s0 <= P; s0 += kPF * NT) {
#pragma unroll
        for (int q = 0; q < kPF; ++q) pnx[q] = pts[partner(min(s0 + t + (kPF + q) * NT, Pc))];
#pragma unroll
        for (int q = 0; q < kPF; ++q) {
          const int o0 = s0 + q * NT;
          if (o0 > P) break;  // uniform
          const int o = o0 + t;
          const bool valid = o <= P;
          const double2 pj = pc[q];
          const double dx = pj.x - xi, dy = pj.y - yi, adx = fabs(dx);
          const bool vert = valid && dx == 0.0;
          const double r = recip(dx);
          const double th = dy * r;  // within a relative 2^-40 of the pair's slope
          const bool ok = adx >= 0x1p-900 && adx <= 0x1p900 && fabs(th) < th_lim;
          const bool force = valid && !vert && !ok;
          const bool test = valid && !vert && ok;
          bool pass = false;
          if (test) pass = bins_pass(bins[slope_bin<kRLog>(dx, dy, r, F)], pall, h);
          const unsigned long long mp = lane_mask(pass);
          n_vert += __popcll(lane_mask(vert));
          n_forced += __popcll(lane_mask(force));
          n_scr += __popcll(lane_mask(test));
          n_pass += __popcll(mp);
          if (force) {
            const int j = partner(o);
            append_entry(ctx, entries, cap, (unsigned)min(i, j), (unsigned)max(i, j));
          }
          if (mp) {
            unsigned base = 0;
            if (lane == 0) base = atomicAdd(&s_cnt, (unsigned)__popcll(mp));
            base = __shfl(base, 0);
            if (pass) list[base + __popcll(mp & ((1ull << lane) - 1ull))] = (unsigned short)(o - 1);
          }
        }
#pragma unroll
        for (int q = 0; q < kPF; ++q) pc[q] = pnx[q];
      }
    }
    __syncthreads();
    // 4. the anchor's passes: into the block's buffer, or straight out if they
    //    do not fit in it
    const unsigned cnt = s_cnt;
    if (cnt) {
      if (s_fill + cnt > (unsigned)PB) flush();
      const bool direct = cnt > (unsigned)PB;
      if (direct) {
        if (t == 0) reserve(cnt);
        __syncthreads();
      }
      const unsigned base = direct ? s_base : s_fill;
      auto put = [&](unsigned q, int j) {
        const uint2 pr = make_uint2((unsigned)i, (unsigned)j);
        if (!direct) pbuf[base + q] = pr;
        else if (base + q < (unsigned)cand_cap) cands[base + q] = pr;
      };
      const unsigned short* offs = CODED ? plist : list;
      for (unsigned q = t; q < cnt; q += NT) {
        int j = i + 1 + (int)offs[q];
        if (j >= n) j -= n;
        put(q, j);
      }
      if (!direct) {
        __syncthreads();
        if (t == 0) s_fill = base + cnt;
      }
    }
  }
  flush();
  if (lane == 0) {
    stat_add(ctx, ST_VERT, n_vert);
    stat_add(ctx, ST_SCREENED, n_scr);
    stat_add(ctx, ST_FORCED, n_forced);
    stat_add(ctx, ST_BIN, n_pass);
  }
}

// The slope-bin screen over the anchors the slope range leaves (k_range):
// only the points of their key intervals (the others are in no window of
// theirs at a slope of the range), and only the partners among those points
// whose slope bin can hold a slope of the range. The frame is centred on the
// best seed slope, as the full one, and scaled to spread the range over most
// of NBP bins (offsets up to 3 in map units), but no coarser near its centre
// than the full frame of nb_full bins. The points' codes and indices stay in
// LDS (runs hold at most NMAX points). Vertical pairs are counted by k_range.
// Does nothing without a range (then k_bins runs).
template <int NT, int NMAX>
__global__ __launch_bounds__(NT) void k_bins_pruned(const double* __restrict__ xy, Ctx* ctx,
                                                    uint2* __restrict__ cands, int cand_cap,
                                                    uint2* __restrict__ entries, int cap,
                                                    const double4* __restrict__ seed_res,
                                                    const double4* __restrict__ seed_rec,
                                                    int n_rec, const unsigned* __restrict__ perm,
                                                    const double2* __restrict__ sxy,
                                                    const uint2* __restrict__ live, int nb_full) {
  constexpr int NBP = kPrunedBins, NBINSP = NBP + NT, kRLogP = __builtin_ctz(NBP) - 1;
  static_assert((NBP % NT) == 0 && ((NBP / NT) & 1) == 0, "bins must be 2^k per thread");
  __shared__ __align__(16) unsigned bins[(NBINSP + 4) & ~3];  // whole 16-byte words
  __shared__ unsigned short pcode[NMAX], pidx[NMAX];
  constexpr int PB = 512;
  __shared__ uint2 pbuf[PB];
  __shared__ unsigned s_part[NT / 64];
  __shared__ unsigned s_all, s_cnt, s_base, s_fill, s_pos;
  const Ctx c = *ctx;
  if (c.status != LMS_OK || c.all_x_equal || c.n_live < 0) return;
  const int n = c.n, h = c.h, t = threadIdx.x, lane = t & 63;
  const double W = __longlong_as_double((long long)c.wbound);
  const double lim = uniform(W * (1.0 + 0x1p-50));
  const BinFrame F = bin_frame(best_slope<NT>(seed_res, c.n_seeds, seed_rec, n_rec),
                               c.xh, c.yh, W, NBINSP);
  const int half = n >> 1;
  const double th_lim = uniform(screen_th_lim(c.fx, c.fy, c.xh, c.yh));
  unsigned long long n_scr = 0, n_forced = 0, n_pass = 0;
  auto reserve = [&](unsigned cnt) {
    const unsigned base = atomicAdd(&ctx->n_cands, cnt);
    if (base + cnt > (unsigned)cand_cap || base + cnt < base) atomicOr(&ctx->cand_overflow, 1u);
    s_base = base;
  };
  auto flush = [&]() {  // all threads; leaves s_fill = 0
    __syncthreads();
    const unsigned fill = s_fill;
    if (fill) {
      if (t == 0) reserve(fill);
      __syncthreads();
      const unsigned base = s_base;
      for (unsigned q = t; q < fill; q += NT)
        if (base + q < (unsigned)cand_cap) cands[base + q] = pbuf[q];
      __syncthreads();
      if (t == 0) s_fill = 0;
      __syncthreads();
    }
  };
  if (t == 0) s_fill = 0;
  const int n_live = c.n_live;
  BinFrame FP = F;
  int blo = 0, bhi = 0;
  if (n_live >= 0) {
    const double tm = c.th_lo + 0.5 * (c.th_hi - c.th_lo);
    const double dl = fmax(c.th_hi - tm, tm - c.th_lo);
    double sc = fmax(3.0 / dl, F.sc * (double)(nb_full / NBP));
    if (fabs(F.tc) * sc > 0x1p20) sc = 0x1p20 / fabs(F.tc);
    FP.sc = fmin(fmax(sc, 0x1p-100), 0x1p100);
    FP.tc = fabs(F.tc) * FP.sc <= 0x1p20 ? F.tc : 0.0;
    FP.q = W < INFINITY ? 0x1p-46 * NBINSP * FP.sc : INFINITY;
    blo = fbin<kRLogP>((c.th_lo - FP.tc) * FP.sc) - 2;
    bhi = fbin<kRLogP>((c.th_hi - FP.tc) * FP.sc) + 2;
  }
  FP.tc = uniform(FP.tc);  // (uniform values in scalar registers)
  FP.sc = uniform(FP.sc);
  FP.q = uniform(FP.q);
  for (int q = blockIdx.x; q < n_live; q += gridDim.x) {
    __syncthreads();  // the previous anchor's queries are done with the bins
    if (t == 0) {
      s_all = 0;
      s_cnt = 0;
      s_pos = 0;
    }
    for (int b = t; b < (NBINSP + 4) / 4; b += NT) reinterpret_cast<uint4*>(bins)[b] = uint4{};
    __syncthreads();
    const uint2 lv = live[q];
    const int i = (int)lv.x, r0 = (int)(lv.y & 0xFFFFu), len = (int)(lv.y >> 16) - r0;
    const unsigned* run = perm + r0;
    const double2* rxy = sxy + r0;
    const double xi = xy[2 * i], yi = xy[2 * i + 1];
    unsigned all = 0;
    double2 nxt = t < len ? rxy[t] : make_double2(0.0, 0.0);
    for (int p = t; p < len; p += NT) {
      const double2 cur = nxt;
      if (p + NT < len) nxt = rxy[p + NT];
      pidx[p] = (unsigned short)run[p];
      add_point_bins_coded<kRLogP>(bins, cur.x - xi, cur.y - yi, W, lim, FP, th_lim, &pcode[p],
                                   all);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) all += __shfl_xor(all, m);
    if (lane == 0) atomicAdd(&s_all, all);
    __syncthreads();
    scan_bins<NBINSP, NT>(bins, s_part);
    __syncthreads();
    const unsigned pall = s_all;
    const int P = (n & 1) ? half : (i < half ? half : half - 1);
    // the anchor's partners are j = (i + o) mod n, o = 1..P
    auto owned = [&](int j) {
      const int o = j >= i ? j - i : j - i + n;
      return o >= 1 && o <= P;
    };
    auto index = [&](int p) { return (int)pidx[p]; };
    for (int p0 = 0; p0 < len; p0 += NT) {
      const int p = p0 + t;
      const int j = p < len ? index(p) : i;
      const bool valid = p < len && owned(j);
      const unsigned cj = valid ? pcode[p] : 0u;
      const bool force = valid && cj == kCodeFP64;
      const bool test = valid && cj > kCodePass && (int)cj >= blo && (int)cj <= bhi;
      const bool pass = test && bins_pass(bins[cj], pall, h);
      const unsigned long long mp = lane_mask(pass);
      n_forced += __popcll(lane_mask(force));
      n_scr += __popcll(lane_mask(test));
      n_pass += __popcll(mp);
      if (force) append_entry(ctx, entries, cap, (unsigned)min(i, j), (unsigned)max(i, j));
      if (pass) pcode[p] = kCodePass;
      if (mp && lane == 0) atomicAdd(&s_cnt, (unsigned)__popcll(mp));
    }
    __syncthreads();
    const unsigned cnt = s_cnt;
    if (cnt) {
      if (s_fill + cnt > (unsigned)PB) flush();
      const bool direct = cnt > (unsigned)PB;
      if (direct) {
        if (t == 0) reserve(cnt);
        __syncthreads();
      }
      const unsigned base = direct ? s_base : s_fill;
      for (int p0 = 0; p0 < len; p0 += NT) {
        const int p = p0 + t;
        const bool m = p < len && pcode[p] == kCodePass;
        const unsigned long long mm = lane_mask(m);
        if (mm) {
          unsigned q0 = 0;
          if (lane == 0) q0 = atomicAdd(&s_pos, (unsigned)__popcll(mm));
          q0 = __shfl(q0, 0);
          if (m) {
            const unsigned q2 = base + q0 + (unsigned)__popcll(mm & ((1ull << lane) - 1ull));
            const uint2 pr = make_uint2((unsigned)i, (unsigned)index(p));
            if (!direct) pbuf[q2] = pr;
            else if (q2 < (unsigned)cand_cap) cands[q2] = pr;
          }
        }
      }
      if (!direct) {
        __syncthreads();
        if (t == 0) s_fill = base + cnt;
      }
    }
  }
  flush();
  if (lane == 0) {
    stat_add(ctx, ST_SCREENED, n_scr);
    stat_add(ctx, ST_FORCED, n_forced);
    stat_add(ctx, ST_BIN, n_pass);
  }
}

// One listed pair per workgroup (see k_screen_list): chunk q of 64 points
// (xy32[64 q + lane], NaN padding past n counts as a miss) goes to wavefront
// q mod (NT / 64). Each wavefront counts B = #{|d| <= thr}, P = #{ta < d <=
// thr} and N = #{-thr <= d < -ta}; the pair survives iff B >= h and (N <= B - h
// or P <= B - h), the verdict of test_pair. Chunks below R use the
// anchor-shifted residual, the others the LDS form, as test_pair does.
template <int R, int NT>
__device__ __forceinline__ void screen_list_blocks(const double* __restrict__ xy,
                                                   const float2* __restrict__ xy32, const Ctx& c,
                                                   Ctx* ctx, const uint2* __restrict__ cands,
                                                   uint2* __restrict__ entries, int cap,
                                                   unsigned total, int chunks) {
  constexpr int NW = NT / 64;
  constexpr int U = 4;  // chunks per step (their loads issued together)
  __shared__ unsigned s_cnt[3];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, h = c.h;
  const double W = __longlong_as_double((long long)c.wbound);
  unsigned long long n_evals = 0, n_devals = 0;
  unsigned n_band = 0;
  for (unsigned e = blockIdx.x; e < total; e += gridDim.x) {
    if (t < 3) s_cnt[t] = 0u;
    __syncthreads();
    const uint2 cd = cands[e];
    const int lo = (int)min(cd.x, cd.y), hi = (int)max(cd.x, cd.y);
    const double th = (xy[2 * hi + 1] - xy[2 * lo + 1]) / (xy[2 * hi] - xy[2 * lo]);
    const ScreenScalars sc = screen_scalars(th, W, c.fx, c.fy, c.xh, c.yh);
    const float2 pi = xy32[cd.x];
    const float nth = -sc.th32, thr = sc.thr, ta = sc.ta;
    const float nc = -fmaf(-sc.th32, pi.x, pi.y);
    unsigned band = 0, above = 0, below = 0;
    for (int q0 = wave; q0 < chunks; q0 += U * NW) {
      float2 p[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u * NW;
        p[u] = xy32[64 * min(q, chunks - 1) + lane];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int q = q0 + u * NW;
        if (q < chunks) {  // uniform
          const float d = q < R ? fmaf(nth, p[u].x - pi.x, p[u].y - pi.y)
                                : fmaf(nth, p[u].x, p[u].y) + nc;
          band += (unsigned)__popcll(__ballot(fabsf(d) <= thr));
          above += (unsigned)__popcll(__ballot(d > ta && d <= thr));
          below += (unsigned)__popcll(__ballot(d < -ta && d >= -thr));
        }
      }
    }
    if (lane == 0) {
      atomicAdd(&s_cnt[0], band);
      atomicAdd(&s_cnt[1], above);
      atomicAdd(&s_cnt[2], below);
    }
    __syncthreads();
    const int B = (int)s_cnt[0], P = (int)s_cnt[1], N = (int)s_cnt[2];
    __syncthreads();  // s_cnt is cleared for the next pair
    n_evals += (unsigned)chunks;
    if (B >= h) {
      ++n_band;
      n_devals += (unsigned)chunks;
      if (t == 0 && (N <= B - h || P <= B - h))
        append_entry(ctx, entries, cap, (unsigned)lo, (unsigned)hi);
    }
  }
  if (t == 0) {
    stat_add(ctx, ST_BAND, n_band);
    stat_add(ctx, ST_EVALS, 64ull * n_evals);
    stat_add(ctx, ST_DEVALS, 64ull * n_devals);
  }
}

// FP32 test of the listed pairs: a wavefront takes a task of up to
// kListBlock consecutive list entries (mostly of one anchor, as the list is
// written per anchor), loads the points shifted by each distinct anchor among
// them, and runs the band and split tests of the exhaustive screen on every
// pair. A pair costs up to two serial passes over the points, so tasks shrink
// to one pair when the list is short and the wavefronts would otherwise idle.
// A list of at most kListPerBlock pairs per workgroup (the usual tens to
// hundreds) goes one pair per workgroup instead: its wavefronts share the
// point chunks and count the band and both one-sided sets in one pass, with
// the same residuals as the wavefront test (anchor-shifted form for the
// register chunks, the LDS form past them), so the verdicts are the same.
constexpr int kListBlock = 16;
constexpr int kListPerBlock = 4;
// fb_items > 0: if the list overflowed, the exhaustive screen of fb_items
// work items (G, ipa as for k_screen) runs here instead (one launch less).
template <int R, bool LDS_PART, int NT>
__global__ __launch_bounds__(NT, 3) void k_screen_list(
    const double* __restrict__ xy, const float2* __restrict__ xy32, Ctx* ctx,
    const uint2* __restrict__ cands, int cand_cap, uint2* __restrict__ entries, int cap, int nq,
    int G, int ipa, int fb_items) {
  extern __shared__ float2 lds[];
  const Ctx c = *ctx;
  if (c.status != LMS_OK || c.all_x_equal) return;
  if (c.cand_overflow) {
    if (fb_items > 0)
      screen_exhaustive<R, LDS_PART, NT>(xy, xy32, ctx, entries, cap, G, ipa, fb_items, nq, 1);
    return;
  }
  const int h = c.h, lane = threadIdx.x & 63;
  if (min(c.n_cands, (unsigned)cand_cap) <= (unsigned)kListPerBlock * gridDim.x) {
    screen_list_blocks<R, NT>(xy, xy32, c, ctx, cands, entries, cap,
                              min(c.n_cands, (unsigned)cand_cap), R + (LDS_PART ? nq : 0));
    return;
  }
  if (LDS_PART) {
    for (int k = threadIdx.x; k < nq * 64; k += blockDim.x) lds[k] = xy32[64 * R + k];
    __syncthreads();
  }
  const unsigned total = min(c.n_cands, (unsigned)cand_cap);
  const unsigned n_waves = gridDim.x * (blockDim.x / 64u);
  const unsigned task = max(1u, min((unsigned)kListBlock, (total + n_waves - 1u) / n_waves));
  const unsigned n_blocks = (total + task - 1u) / task;
  const double W = __longlong_as_double((long long)c.wbound);
  unsigned long long n_evals = 0, n_devals = 0;
  unsigned n_band = 0;
  int loaded = -1;
  float X[R], Y[R];
  float2 pi = make_float2(0.0f, 0.0f);
#pragma unroll
  for (int r = 0; r < R; ++r) X[r] = Y[r] = 0.0f;
  // Static round-robin over the tasks: no shared counter, so the waves that
  // find no work leave at once (a contended counter costs tens of us).
  const unsigned w0 = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / 64u) +
                                                     threadIdx.x / 64u);
  for (unsigned blk = w0; blk < n_blocks; blk += n_waves) {
    const unsigned e = blk * task + (unsigned)lane;
    const bool valid = (unsigned)lane < task && e < total;
    const uint2 cd = valid ? cands[e] : make_uint2(0u, 0u);
    const int ai = (int)cd.x, aj = (int)cd.y;
    unsigned long long todo = __ballot(valid);
    while (todo) {
      const int l0 = __ffsll((long long)todo) - 1;
      const int a = lane_i(ai, l0);
      const unsigned long long mine = __ballot(valid && ai == a) & todo;
      todo &= ~mine;
      if (a != loaded) {
        pi = xy32[a];
        const float2* src = xy32;
        asm volatile("" : "+s"(src));
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const float2 p = src[lane + 64 * r];
          X[r] = p.x - pi.x;
          Y[r] = p.y - pi.y;
        }
        loaded = a;
      }
      const bool me = (mine >> lane) & 1ull;
      const int j = me ? aj : (a == 0 ? 1 : 0);
      const int lo = min(a, j), hi = max(a, j);
      const double xl = xy[2 * lo], yl = xy[2 * lo + 1];
      const double xr = xy[2 * hi], yr = xy[2 * hi + 1];
      const double th = (yr - yl) / (xr - xl);
      const ScreenScalars sc = screen_scalars(th, W, c.fx, c.fy, c.xh, c.yh);
      const float th32 = me ? sc.th32 : 0.0f;
      const float thr = me ? sc.thr : 0.0f;
      const float ta = me ? sc.ta : 0.0f;
      const float nc = me ? -fmaf(-th32, pi.x, pi.y) : 0.0f;
      unsigned long long m = mine;
      while (m) {
        const int cl = __ffsll((long long)m) - 1;
        m &= m - 1;
        const PairTest pt = test_pair<R, LDS_PART>(X, Y, lds, nq, -lane_f(th32, cl),
                                                   lane_f(thr, cl), lane_f(ta, cl),
                                                   lane_f(nc, cl), h);
        n_evals += (unsigned)pt.band_chunks;
        if (pt.split_chunks >= 0) {
          ++n_band;
          n_devals += (unsigned)pt.split_chunks;
        }
        if (pt.keep && lane == 0)
          append_entry(ctx, entries, cap, (unsigned)lane_i(lo, cl), (unsigned)lane_i(hi, cl));
      }
    }
  }
  if (lane == 0) {
    stat_add(ctx, ST_BAND, n_band);
    stat_add(ctx, ST_EVALS, 64ull * n_evals);
    stat_add(ctx, ST_DEVALS, 64ull * n_devals);
  }
}

// Verdicts for explicit pairs (lms_screen_pairs): one wavefront per pair,
// same test as the screen kernel.
template <int R, bool LDS_PART, int NT>
__global__ __launch_bounds__(NT) void k_screen_pairs(
    const double* __restrict__ xy, const float2* __restrict__ xy32, const Ctx* ctx, double W,
    const int* __restrict__ pairs, int m, int* __restrict__ verdict, int nq) {
  extern __shared__ float2 lds[];
  const Ctx c = *ctx;
  if (c.status < 0) return;
  const int lane = threadIdx.x & 63;
  if (LDS_PART) {
    for (int k = threadIdx.x; k < nq * 64; k += blockDim.x) lds[k] = xy32[64 * R + k];
    __syncthreads();
  }
  const int wpb = blockDim.x / 64;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
  for (int t = blockIdx.x * wpb + wave; t < m; t += gridDim.x * wpb) {
    const int a = pairs[2 * t], b = pairs[2 * t + 1];
    if (a < 0 || b < 0 || a >= c.n || b >= c.n) {
      if (lane == 0) verdict[t] = -1;
      continue;
    }
    const int lo = min(a, b), hi = max(a, b);
    const int i = a;  // anchor on the first member as given
    const double xl = xy[2 * lo], yl = xy[2 * lo + 1], xr = xy[2 * hi], yr = xy[2 * hi + 1];
    if (xl == xr) {
      if (lane == 0) verdict[t] = 2;
      continue;
    }
    const double th = (yr - yl) / (xr - xl);
    const ScreenScalars sc = screen_scalars(th, W, c.fx, c.fy, c.xh, c.yh);
    if (sc.force) {
      if (lane == 0) verdict[t] = 1;
      continue;
    }
    const float2 pi = xy32[i];
    float X[R], Y[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float2 p = xy32[lane + 64 * r];
      X[r] = p.x - pi.x;
      Y[r] = p.y - pi.y;
    }
    const float th32 = sc.th32;
    // per-pair scalars in SGPRs, as in the screen kernel
    const PairTest pt = test_pair<R, LDS_PART>(
        X, Y, lds, nq, lane_f(-th32, 0), lane_f(sc.thr, 0), lane_f(sc.ta, 0),
        lane_f(-fmaf(-th32, pi.x, pi.y), 0), c.h);
    if (lane == 0) verdict[t] = pt.keep;
  }
}

// ---------------------------------------------------------------- host side

struct Layout {
  size_t ctx, xy32, entries, res, rec, cands, sort_tmp, grid, range, net, total;
};

// n_rec: windows of the device seed slopes (kept only for window pairs);
// cand_cap: list of the slope-bin screen's passes; sort_tmp: doubles of the
// split FP64 re-evaluation
Layout layout(int n_pad, long long cap, long long n_rec = 0, long long cand_cap = 0,
              long long sort_tmp = 0, bool net = false) {
  auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
  Layout L;
  L.ctx = 0;
  L.xy32 = up(kStatsOffset + sizeof(Stats));
  L.entries = L.xy32 + up((size_t)n_pad * sizeof(float2));
  L.res = L.entries + up((size_t)cap * sizeof(uint2));
  L.rec = L.res + up((size_t)cap * sizeof(double4));
  L.cands = L.rec + up((size_t)n_rec * sizeof(double4));
  L.sort_tmp = L.cands + up((size_t)cand_cap * sizeof(uint2));
  L.grid = L.sort_tmp + up((size_t)sort_tmp * sizeof(double));
  L.range = L.grid + up(2 * kGrid * (sizeof(double) + sizeof(double4)));
  L.net = L.range + up((size_t)n_pad * (sizeof(unsigned) + sizeof(uint2) + sizeof(double2)));
  // the network's slope (one double), then its inference scratch
  L.total = L.net + (net ? up(sizeof(double)) + up(lms_host::net_infer_bytes(1)) : 0);
  return L;
}

int next_pow2(int v) {
  int p = 64;
  while (p < v) p <<= 1;
  return p;
}

// Points per lane kept in VGPRs for the screen: the smallest supported count
// covering n, or the maximum with the rest in LDS.
int pick_R(int n) {
  static const int Rs[] = {1, 2, 4, 8, 16, 24, 32, 48, 64};
  for (int r : Rs)
    if (64 * r >= n) return r;
  return kRegChunks;
}

template <int N2>
void launch_recheck_n2(hipStream_t s, int grid, const double* xy, Ctx* ctx, const uint2* e,
                       double4* res, int begin, int cap, int upd) {
  constexpr int NT = N2 >= 2048 ? 1024 : 256;
  hipLaunchKernelGGL((k_recheck<N2, NT>), dim3(grid), dim3(NT), 0, s, xy, ctx, e, res, begin, cap,
                     upd);
}

// gy: workgroups per chunk (each sorts that chunk of entries y, y + gy, ...);
// grid: k_merge_window's workgroups.
template <int NP>
void launch_split_np(hipStream_t s, int grid, int gy, int slots, const double* xy, Ctx* ctx,
                     const uint2* e, double4* res, int begin, int cap, int upd, double* tmp,
                     const double* thetas) {
  constexpr int NT = NP >= 2048 ? 1024 : 256;
  hipLaunchKernelGGL((k_sort_chunks<kSplitChunk, kSplitNT>), dim3(NP / kSplitChunk, gy),
                     dim3(kSplitNT), 0, s, xy, ctx, e, begin, cap, slots, tmp, NP, thetas);
  hipLaunchKernelGGL((k_merge_window<NP, NT>), dim3(grid), dim3(NT), 0, s, xy, ctx, e, res, begin,
                     cap, upd, tmp, slots, thetas);
}

// Number of entries that one split launch pair sorts in pieces (0: whole-sort
// path, for n <= kSplitChunk).
int split_slots(int n, int expected) {
  if (next_pow2(n) <= kSplitChunk) return 0;
  return std::max(1, std::min(expected, kSplitSlots));
}

// Re-evaluation of entries [begin, min(n_entries, cap)) in FP64. The split
// path takes the first `slots` of them (tmp holds slots x next_pow2(n)
// doubles), gy at a time per chunk; `grid` workgroups merge them and sort any
// further ones whole.
void launch_recheck(hipStream_t s, int n, int grid, const double* xy, Ctx* ctx, const uint2* e,
                    double4* res, int begin, int cap, int upd, double* tmp, int slots, int gy,
                    const double* thetas = nullptr) {
  if (tmp && slots > 0) {
    gy = std::max(1, std::min(gy, slots));
    switch (next_pow2(n)) {
      case 1024: launch_split_np<1024>(s, grid, gy, slots, xy, ctx, e, res, begin, cap, upd, tmp, thetas); return;
      case 2048: launch_split_np<2048>(s, grid, gy, slots, xy, ctx, e, res, begin, cap, upd, tmp, thetas); return;
      case 4096: launch_split_np<4096>(s, grid, gy, slots, xy, ctx, e, res, begin, cap, upd, tmp, thetas); return;
      case 8192: launch_split_np<8192>(s, grid, gy, slots, xy, ctx, e, res, begin, cap, upd, tmp, thetas); return;
      default: launch_split_np<16384>(s, grid, gy, slots, xy, ctx, e, res, begin, cap, upd, tmp, thetas); return;
    }
  }
  switch (next_pow2(n)) {
    case 64: launch_recheck_n2<64>(s, grid, xy, ctx, e, res, begin, cap, upd); break;
    case 128: launch_recheck_n2<128>(s, grid, xy, ctx, e, res, begin, cap, upd); break;
    case 256: launch_recheck_n2<256>(s, grid, xy, ctx, e, res, begin, cap, upd); break;
    case 512: launch_recheck_n2<512>(s, grid, xy, ctx, e, res, begin, cap, upd); break;
    case 1024: launch_recheck_n2<1024>(s, grid, xy, ctx, e, res, begin, cap, upd); break;
    case 2048: launch_recheck_n2<2048>(s, grid, xy, ctx, e, res, begin, cap, upd); break;
    case 4096: launch_recheck_n2<4096>(s, grid, xy, ctx, e, res, begin, cap, upd); break;
    case 8192: launch_recheck_n2<8192>(s, grid, xy, ctx, e, res, begin, cap, upd); break;
    default: launch_recheck_n2<16384>(s, grid, xy, ctx, e, res, begin, cap, upd); break;
  }
}

template <int N2>
void launch_eval_n2(hipStream_t s, int grid, const double* xy, int n, int h, const double* th,
                    int m, double* out, Ctx* ctx, double4* rec) {
  constexpr int NT = N2 >= 2048 ? 1024 : 256;
  hipLaunchKernelGGL((k_eval_slopes<N2, NT>), dim3(grid), dim3(NT), 0, s, xy, n, h, th, m, out,
                     ctx, rec);
}

void launch_eval(hipStream_t s, int grid, const double* xy, int n, int h, const double* th, int m,
                 double* out, Ctx* ctx, double4* rec = nullptr) {
  switch (next_pow2(n)) {
    case 64: launch_eval_n2<64>(s, grid, xy, n, h, th, m, out, ctx, rec); break;
    case 128: launch_eval_n2<128>(s, grid, xy, n, h, th, m, out, ctx, rec); break;
    case 256: launch_eval_n2<256>(s, grid, xy, n, h, th, m, out, ctx, rec); break;
    case 512: launch_eval_n2<512>(s, grid, xy, n, h, th, m, out, ctx, rec); break;
    case 1024: launch_eval_n2<1024>(s, grid, xy, n, h, th, m, out, ctx, rec); break;
    case 2048: launch_eval_n2<2048>(s, grid, xy, n, h, th, m, out, ctx, rec); break;
    case 4096: launch_eval_n2<4096>(s, grid, xy, n, h, th, m, out, ctx, rec); break;
    case 8192: launch_eval_n2<8192>(s, grid, xy, n, h, th, m, out, ctx, rec); break;
    default: launch_eval_n2<16384>(s, grid, xy, n, h, th, m, out, ctx, rec); break;
  }
}

// Threads per block of the screen: 256 when all points sit in registers;
// with the LDS part one block per CU shares the LDS copy, so it is as large
// as the register budget allows.
template <int R, bool L>
constexpr int screen_threads() {
  return !L ? 256 : (R == 64 ? 768 : 1024);
}

template <int R, bool L>
hipError_t launch_screen_rl(hipStream_t s, int cu, const double* xy, const float2* xy32, Ctx* ctx,
                            uint2* e, int cap, int G, int ipa, int n_items, int nq, int fb) {
  constexpr int nt = screen_threads<R, L>();
  const size_t shm = L ? (size_t)nq * 64 * sizeof(float2) : 0;
  if (L) {
    (void)hipFuncSetAttribute((const void*)k_screen<R, L, nt>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    (void)hipGetLastError();
  }
  const long long per_block = nt / 64;
  const long long need = (n_items + per_block - 1) / per_block;
  // persistent blocks: as many as fit on the chip at once
  static int resident_regs = 0;  // register-only form: no LDS, so fixed per kernel
  int resident = L ? 0 : resident_regs;
  if (resident == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_screen<R, L, nt>, nt,
                                                     shm) != hipSuccess || nb < 1) {
      (void)hipGetLastError();
      nb = L ? 1 : 3;
    }
    resident = nb;
    if (!L) resident_regs = nb;
  }
  const int grid = (int)std::max<long long>(1, std::min<long long>(need, (long long)cu * resident));
  hipLaunchKernelGGL((k_screen<R, L, nt>), dim3(grid), dim3(nt), shm, s, xy, xy32, ctx, e, cap, G,
                     ipa, n_items, nq, fb);
  return hipGetLastError();
}

hipError_t launch_screen(hipStream_t s, int R, bool L, int cu, const double* xy,
                         const float2* xy32, Ctx* ctx, uint2* e, int cap, int G, int ipa,
                         int n_items, int nq, int fb = 0) {
#define LMS_SCREEN_CASE(RR, LL) \
  return launch_screen_rl<RR, LL>(s, cu, xy, xy32, ctx, e, cap, G, ipa, n_items, nq, fb)
  if (L) {
    switch (R) {
      case 1: LMS_SCREEN_CASE(1, true);
      case 16: LMS_SCREEN_CASE(16, true);
      case 32: LMS_SCREEN_CASE(32, true);
      default: LMS_SCREEN_CASE(64, true);
    }
  }
  switch (R) {
    case 1: LMS_SCREEN_CASE(1, false);
    case 2: LMS_SCREEN_CASE(2, false);
    case 4: LMS_SCREEN_CASE(4, false);
    case 8: LMS_SCREEN_CASE(8, false);
    case 16: LMS_SCREEN_CASE(16, false);
    case 24: LMS_SCREEN_CASE(24, false);
    case 32: LMS_SCREEN_CASE(32, false);
    case 48: LMS_SCREEN_CASE(48, false);
    default: LMS_SCREEN_CASE(64, false);
  }
#undef LMS_SCREEN_CASE
}

template <int R, bool L>
hipError_t launch_pairs_rl(hipStream_t s, const double* xy, const float2* xy32, const Ctx* ctx,
                           double W, const int* pairs, int m, int* verdict, int nq) {
  constexpr int nt = screen_threads<R, L>();
  const size_t shm = L ? (size_t)nq * 64 * sizeof(float2) : 0;
  if (L) {
    (void)hipFuncSetAttribute((const void*)k_screen_pairs<R, L, nt>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    (void)hipGetLastError();
  }
  const int wpb = nt / 64;
  const int grid = std::max(1, std::min(4096, (m + wpb - 1) / wpb));
  hipLaunchKernelGGL((k_screen_pairs<R, L, nt>), dim3(grid), dim3(nt), shm, s, xy, xy32, ctx, W,
                     pairs, m, verdict, nq);
  return hipGetLastError();
}

hipError_t launch_pairs(hipStream_t s, int R, bool L, const double* xy, const float2* xy32,
                        const Ctx* ctx, double W, const int* pairs, int m, int* verdict, int nq) {
#define LMS_PAIRS_CASE(RR, LL) \
  return launch_pairs_rl<RR, LL>(s, xy, xy32, ctx, W, pairs, m, verdict, nq)
  if (L) {
    switch (R) {
      case 1: LMS_PAIRS_CASE(1, true);
      case 16: LMS_PAIRS_CASE(16, true);
      case 32: LMS_PAIRS_CASE(32, true);
      default: LMS_PAIRS_CASE(64, true);
    }
  }
  switch (R) {
    case 1: LMS_PAIRS_CASE(1, false);
    case 2: LMS_PAIRS_CASE(2, false);
    case 4: LMS_PAIRS_CASE(4, false);
    case 8: LMS_PAIRS_CASE(8, false);
    case 16: LMS_PAIRS_CASE(16, false);
    case 24: LMS_PAIRS_CASE(24, false);
    case 32: LMS_PAIRS_CASE(32, false);
    case 48: LMS_PAIRS_CASE(48, false);
    default: LMS_PAIRS_CASE(64, false);
  }
#undef LMS_PAIRS_CASE
}

// Slope-bin screen: threads per block for NB bins (the prefix sum holds
// NB / NT bins per thread in registers).
template <int NB>
constexpr int bins_threads() {
  return NB >= 32768 ? 1024 : (NB >= 8192 ? 512 : 256);
}

template <int NB, bool WIDE>
hipError_t launch_bins_nb(hipStream_t s, int cu, int n, const double* xy, Ctx* ctx, uint2* cands,
                          int cand_cap, uint2* e, int cap, const double4* res,
                          const double4* rec, int n_rec) {
  constexpr int nt = bins_threads<NB>();
  static int resident = 0;
  if (resident == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_bins<NB, nt, WIDE>, nt,
                                                     0) != hipSuccess || nb < 1) {
      (void)hipGetLastError();
      nb = 1;
    }
    resident = nb;
  }
  const int grid = std::max(1, std::min(n, cu * resident));
  hipLaunchKernelGGL((k_bins<NB, nt, WIDE>), dim3(grid), dim3(nt), 0, s, xy, ctx, cands, cand_cap,
                     e, cap, res, rec, rec ? n_rec : 0);
  return hipGetLastError();
}

template <int NT, int NMAX>
hipError_t launch_pruned_nt(hipStream_t s, int cu, int n, const double* xy, Ctx* ctx,
                            uint2* cands, int cand_cap, uint2* e, int cap, const double4* res,
                            const double4* rec, int n_rec, const unsigned* perm,
                            const double2* sxy, const uint2* live, int nb_full) {
  static int resident = 0;
  if (resident == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_bins_pruned<NT, NMAX>,
                                                     NT, 0) != hipSuccess || nb < 1) {
      (void)hipGetLastError();
      nb = 1;
    }
    resident = nb;
  }
  const int grid = std::max(1, std::min(n, cu * resident));
  hipLaunchKernelGGL((k_bins_pruned<NT, NMAX>), dim3(grid), dim3(NT), 0, s, xy, ctx, cands,
                     cand_cap, e, cap, res, rec, rec ? n_rec : 0, perm, sxy, live, nb_full);
  return hipGetLastError();
}

hipError_t launch_bins(hipStream_t s, int nb_log2, int cu, int n, const double* xy, Ctx* ctx,
                       uint2* cands, int cand_cap, uint2* e, int cap, const double4* res,
                       const double4* rec, int n_rec, const unsigned* perm,
                       const double2* sxy, const uint2* live) {
  // the full screen, then (with a slope range; each kernel returns at once
  // when the other one's case holds) the pruned one
  hipError_t err;
  // fewer bins than 2 n: the WIDE form (no codes, room for n / 2 passes)
  const bool wide = (1 << nb_log2) < 2 * n;
  switch (nb_log2 * 2 + (wide ? 1 : 0)) {
    case 22: err = launch_bins_nb<2048, false>(s, cu, n, xy, ctx, cands, cand_cap, e, cap, res, rec, n_rec); break;
    case 23: err = launch_bins_nb<2048, true>(s, cu, n, xy, ctx, cands, cand_cap, e, cap, res, rec, n_rec); break;
    case 24: err = launch_bins_nb<4096, false>(s, cu, n, xy, ctx, cands, cand_cap, e, cap, res, rec, n_rec); break;
    case 25: err = launch_bins_nb<4096, true>(s, cu, n, xy, ctx, cands, cand_cap, e, cap, res, rec, n_rec); break;
    case 26: err = launch_bins_nb<8192, false>(s, cu, n, xy, ctx, cands, cand_cap, e, cap, res, rec, n_rec); break;
    case 27: err = launch_bins_nb<8192, true>(s, cu, n, xy, ctx, cands, cand_cap, e, cap, res, rec, n_rec); break;
    case 28: err = launch_bins_nb<16384, false>(s, cu, n, xy, ctx, cands, cand_cap, e, cap, res, rec, n_rec); break;
    case 29: err = launch_bins_nb<16384, true>(s, cu, n, xy, ctx, cands, cand_cap, e, cap, res, rec, n_rec); break;
    default: err = launch_bins_nb<32768, false>(s, cu, n, xy, ctx, cands, cand_cap, e, cap, res, rec, n_rec); break;
  }
  if (err != hipSuccess || !live) return err;
  const int nb_full = 1 << nb_log2;
  if (n <= 4096)
    return launch_pruned_nt<256, 4096>(s, cu, n, xy, ctx, cands, cand_cap, e, cap, res, rec, n_rec,
                                       perm, sxy, live, nb_full);
  if (n <= 8192)
    return launch_pruned_nt<512, 8192>(s, cu, n, xy, ctx, cands, cand_cap, e, cap, res, rec, n_rec,
                                       perm, sxy, live, nb_full);
  // (512 threads: two workgroups per CU; 1024 fit only one, at 5 % more time)
  return launch_pruned_nt<512, 16384>(s, cu, n, xy, ctx, cands, cand_cap, e, cap, res, rec, n_rec,
                                      perm, sxy, live, nb_full);
}

template <int R, bool L>
hipError_t launch_list_rl(hipStream_t s, int cu, const double* xy, const float2* xy32, Ctx* ctx,
                          const uint2* cands, int cand_cap, uint2* e, int cap, int nq, int G,
                          int ipa, int fb_items) {
  constexpr int nt = screen_threads<R, L>();
  const size_t shm = L ? (size_t)nq * 64 * sizeof(float2) : 0;
  if (L) {
    (void)hipFuncSetAttribute((const void*)k_screen_list<R, L, nt>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    (void)hipGetLastError();
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_screen_list<R, L, nt>, nt,
                                                   shm) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  // persistent blocks, but no more than the list (or the fallback's work
  // items) could ever occupy one pair each
  const long long need =
      ((long long)std::max(cand_cap, fb_items) + nt / 64 - 1) / (nt / 64);
  const int grid = (int)std::max<long long>(1, std::min<long long>((long long)cu * nb, need));
  hipLaunchKernelGGL((k_screen_list<R, L, nt>), dim3(grid), dim3(nt), shm, s, xy, xy32, ctx,
                     cands, cand_cap, e, cap, nq, G, ipa, fb_items);
  return hipGetLastError();
}

// fb_items > 0: the exhaustive screen's work items, run by the same launch if
// the list overflows.
hipError_t launch_list(hipStream_t s, int R, bool L, int cu, const double* xy, const float2* xy32,
                       Ctx* ctx, const uint2* cands, int cand_cap, uint2* e, int cap, int nq,
                       int G, int ipa, int fb_items) {
#define LMS_LIST_CASE(RR, LL) \
  return launch_list_rl<RR, LL>(s, cu, xy, xy32, ctx, cands, cand_cap, e, cap, nq, G, ipa, fb_items)
  if (L) {
    switch (R) {
      case 1: LMS_LIST_CASE(1, true);
      case 16: LMS_LIST_CASE(16, true);
      case 32: LMS_LIST_CASE(32, true);
      default: LMS_LIST_CASE(64, true);
    }
  }
  switch (R) {
    case 1: LMS_LIST_CASE(1, false);
    case 2: LMS_LIST_CASE(2, false);
    case 4: LMS_LIST_CASE(4, false);
    case 8: LMS_LIST_CASE(8, false);
    case 16: LMS_LIST_CASE(16, false);
    case 24: LMS_LIST_CASE(24, false);
    case 32: LMS_LIST_CASE(32, false);
    case 48: LMS_LIST_CASE(48, false);
    default: LMS_LIST_CASE(64, false);
  }
#undef LMS_LIST_CASE
}

// Default slope bins per anchor: about 2n, at least 2^11, at most 2^15.
// Bins per anchor for 2^nb_log2 nominal ones: one more per thread of k_bins.
unsigned bins_count(int nb_log2) {
  const int nb = 1 << nb_log2;
  return (unsigned)(nb + (nb >= 32768 ? 1024 : (nb >= 8192 ? 512 : 256)));
}

// 2 n bins up to 4096 points (codes in LDS); above, 2^13 in the WIDE form:
// at 16384 points it keeps two workgroups per CU where 2^15 bins keep one,
// and its full screen took 0.80 ms against 1.03 ms (integer set, 16384
// points, MI355X).
int default_bins_log2(int n) {
  int b = 11;
  while (b < 13 && (1 << b) < 2 * n) ++b;
  return b;
}

struct Plan {
  int n, h, R, nq, n_pad, n_seeds;
  bool lds;
  long long cap;
};

lms_status make_plan(const void* d_xy, int64_t n, int64_t h, Plan* p, int tile_regs = 0) {
  if (!d_xy) return fail(LMS_ERR_ARG, "null point pointer");
  if (n < 2 || n > LMS_MAX_N)
    return fail(LMS_ERR_ARG, "n must be in [2, " + std::to_string(LMS_MAX_N) + "]");
  if (h == 0) h = n / 2 + 1;
  if (h < 2 || h > n) return fail(LMS_ERR_ARG, "h must be in [2, n]");
  p->n = (int)n;
  p->h = (int)h;
  p->R = pick_R((int)n);
  if (tile_regs < 0 || tile_regs > kRegChunks)
    return fail(LMS_ERR_ARG, "tile_regs must be in [0, 64]");
  if (tile_regs > 0 && tile_regs < p->R) {
    // fewer register chunks than the points need: the rest streams from LDS
    p->R = tile_regs >= 64 ? 64 : tile_regs >= 32 ? 32 : tile_regs >= 16 ? 16 : 1;
  }
  p->lds = 64 * p->R < n;
  if (p->lds && p->R != 1 && p->R != 16 && p->R != 32 && p->R != 64)
    return fail(LMS_ERR_ARG, "unsupported register tile");
  p->nq = p->lds ? (int)((n - 64 * p->R + 63) / 64) : 0;
  p->n_pad = 64 * (p->R + p->nq);
  return LMS_OK;
}

// Everything one solve needs, from its arguments and options.
struct Setup {
  Plan p;
  const double* xy = nullptr;
  lms_result* out = nullptr;
  unsigned flags = 0;
  int seeds = 0, window_pairs = 0, bins_log2 = 0, G = 1, ipa = 1;
  int final_slots = 0;
  bool no_prune = false, use_bins = false;
  const float* net = nullptr;  // seed-network parameters (the slope is computed in the solve)
  bool range = false, refine = false;  // slope range: first grid; second grid
  const double* seed_theta = nullptr;
  int64_t n_seed_theta = 0;
  long long pairs = 0, cand_cap = 0, n_items = 0;
  Layout L;
};

lms_status make_setup(const double* d_xy, int64_t n, int64_t h, lms_result* d_out,
                      const lms_options* opt, Setup* S) {
  if (opt && opt->struct_size < offsetof(lms_options, max_workspace))
    return fail(LMS_ERR_ARG, "bad options size");
  // automatic tiles and seeds: the autotuned choice for this size class, if any
  lms_tuning tuned{0, 0, -1, 0, 0.0, 0, 0};
  const bool have_tuned = n >= 2 && n <= LMS_MAX_N &&
                          lms_host::get_tuning(kPathSingle, lms_host::size_class((int)n), &tuned);
  int tile_regs = opt ? opt->tile_regs : 0;
  int tile_batches = opt ? opt->tile_batches : 0;
  int bins_log2 = opt ? opt->bins_log2 : 0;
  if (have_tuned && tile_regs == 0) tile_regs = tuned.tile_regs;
  if (have_tuned && tile_batches == 0) tile_batches = tuned.tile_batches;
  if (have_tuned && bins_log2 == 0) bins_log2 = tuned.bins_log2;
  if (tile_batches < 0 || tile_batches > 64) return fail(LMS_ERR_ARG, "tile_batches must be in [0, 64]");
  if (bins_log2 != 0 && bins_log2 != -1 && (bins_log2 < 11 || bins_log2 > 15))
    return fail(LMS_ERR_ARG, "bins_log2 must be 0, -1 or in [11, 15]");
  Plan& p = S->p;
  lms_status st = make_plan(d_xy, n, h, &p, tile_regs);
  if (st != LMS_OK) return st;
  if (!d_out) return fail(LMS_ERR_ARG, "null result pointer");
  int seeds = (have_tuned && tuned.seed_pairs >= 0) ? tuned.seed_pairs : kDefaultSeeds;
  unsigned flags = 0;
  const double* d_seed_theta = nullptr;
  int64_t n_seed_theta = 0;
  int window_pairs = 0;
  if (opt) {
    flags = opt->flags;
    if (opt->seed_pairs < -1) return fail(LMS_ERR_ARG, "seed_pairs must be >= -1");
    if (opt->seed_pairs >= 0) seeds = opt->seed_pairs;
    d_seed_theta = opt->d_seed_theta;
    n_seed_theta = opt->n_seed_theta;
    if (n_seed_theta < 0 || (n_seed_theta > 0 && !d_seed_theta) || n_seed_theta > (1 << 24))
      return fail(LMS_ERR_ARG, "bad seed slope array");
    window_pairs = opt->window_pairs;
    if (window_pairs < 0 || window_pairs > (1 << 16))
      return fail(LMS_ERR_ARG, "window_pairs must be in [0, 65536]");
    if (opt->struct_size >= offsetof(lms_options, d_net_params) + sizeof(void*) &&
        opt->d_net_params) {
      if (n_seed_theta) return fail(LMS_ERR_ARG, "d_net_params and d_seed_theta are exclusive");
      S->net = opt->d_net_params;
      n_seed_theta = 1;  // the network's slope, computed on the device
    }
  }
  const long long pairs = (long long)p.n * (p.n - 1) / 2;
  const bool no_prune = (flags & LMS_F_NO_PRUNE) != 0;
  if (no_prune && pairs > kScreenCap)
    return fail(LMS_ERR_ARG, "LMS_F_NO_PRUNE supports at most 2^24 pairs");
  // window pairs need a seed line and a bound to tighten
  if (n_seed_theta == 0 || no_prune) window_pairs = 0;
  p.n_seeds = 1 + seeds + 2 * window_pairs;
  const long long screen_cap = std::min(pairs, kScreenCap);
  p.cap = p.n_seeds + screen_cap;
  if (p.cap > INT_MAX) return fail(LMS_ERR_ARG, "too many seeds");
  // slope-bin screen: at least n bins (its per-anchor list holds n / 2 partners)
  const bool use_bins = bins_log2 != -1;
  if (use_bins) {
    if (bins_log2 == 0) bins_log2 = default_bins_log2(p.n);
  }
  const int Pmax = p.n / 2;
  const int batches = (Pmax + 63) / 64;
  S->G = std::min(tile_batches > 0 ? tile_batches : 4, std::max(1, batches));
  S->ipa = (batches + S->G - 1) / S->G;
  S->n_items = (long long)p.n * S->ipa;
  S->xy = d_xy;
  S->out = d_out;
  S->flags = flags;
  S->seeds = seeds;
  S->window_pairs = window_pairs;
  S->bins_log2 = bins_log2;
  S->no_prune = no_prune;
  S->use_bins = use_bins;
  // The slope range costs two or three short launches and kGrid (2 kGrid)
  // exact windows; the anchors and points it drops pay for that above
  // kRangeMinN (kRefineMinN) points.
  // the tuned range choice applies when the flags leave it open
  const bool flags_range = (flags & (LMS_F_RANGE | LMS_F_NO_RANGE)) != 0;
  const bool force_range = (flags & LMS_F_RANGE) != 0 ||
                           (!flags_range && have_tuned && tuned.range > 0);
  const bool no_range = (flags & LMS_F_NO_RANGE) != 0 ||
                        (!flags_range && have_tuned && tuned.range < 0);
  S->range = use_bins && !no_prune && !no_range && (force_range || p.n > kRangeMinN);
  S->refine = S->range && (force_range || p.n > kRefineMinN);
  S->seed_theta = d_seed_theta;
  S->n_seed_theta = n_seed_theta;
  S->pairs = pairs;
  S->cand_cap = use_bins ? screen_cap : 0;
  // split re-evaluation slots: the usual number of survivors
  S->final_slots = split_slots(p.n, p.n > 4096 ? kFinalSlotsLarge : kFinalSlots);
  const long long tmp = (long long)S->final_slots * next_pow2(p.n);
  S->L = layout(p.n_pad, p.cap, n_seed_theta, S->cand_cap, tmp, S->net != nullptr);
  // A workspace limit shrinks the lists (order below).
  const uint64_t max_ws =
      opt && opt->struct_size >= offsetof(lms_options, max_workspace) + sizeof(uint64_t)
          ? opt->max_workspace : 0;
  if (max_ws && S->L.total > max_ws) {
    // The survivor list shrinks first to kKeepSurv slots (tens of survivors
    // are usual), then the pass list (its overflow only costs time: the
    // exhaustive FP32 screen runs), then the survivor list again (its
    // overflow is LMS_ERR_CAPACITY), each down to kMinList slots.
    const long long kMinList = 1024, kKeepSurv = 65536;
    const long long per_c = (long long)sizeof(uint2);
    const long long per_s = (long long)(sizeof(uint2) + sizeof(double4));
    auto relayout = [&]() {
      S->L = layout(p.n_pad, p.cap, n_seed_theta, S->cand_cap, tmp, S->net != nullptr);
    };
    auto shrink = [&](long long& slots, long long floor, long long per, long long base) {
      if (S->L.total <= max_ws || slots - base <= floor) return;
      const long long over = (long long)(S->L.total - max_ws);
      slots = base + std::max(floor, slots - base - (over + per - 1) / per - 64);
      relayout();
    };
    shrink(p.cap, kKeepSurv, per_s, p.n_seeds);
    shrink(S->cand_cap, kMinList, per_c, 0);
    shrink(p.cap, kMinList, per_s, p.n_seeds);
    if (S->L.total > max_ws)
      return fail(LMS_ERR_NOMEM, "max_workspace below the " + std::to_string(S->L.total) +
                                     " bytes this solve needs at the least");
  }
  return LMS_OK;
}

// Enqueues one solve on s (kernels only, so it can be captured in a graph).
lms_status enqueue_solve(const Setup& S, char* base, hipStream_t s, lms_host::StageEvents* prof) {
  const Plan& p = S.p;
  const Layout& L = S.L;
  const double* d_xy = S.xy;
  Ctx* ctx = (Ctx*)(base + L.ctx);
  float2* xy32 = (float2*)(base + L.xy32);
  uint2* entries = (uint2*)(base + L.entries);
  double4* res = (double4*)(base + L.res);
  double4* rec = (double4*)(base + L.rec);
  const int cu = lms_host::num_cu();
  const int seeds = S.seeds, window_pairs = S.window_pairs;
  const int64_t n_seed_theta = S.n_seed_theta;
  auto mark = [&]() { if (prof) prof->mark(); };
  const unsigned long long key = 0x5EEDull + (unsigned long long)p.n * 0x100000001ull;
  launch_prep(s, d_xy, p.n, p.h, p.n_pad, ctx, xy32, entries, p.n_seeds, seeds, key,
              S.use_bins ? bins_count(S.bins_log2) : 0u, (int)p.cap);
  // the seed network's slope, as the device seed slope
  const double* seed_theta = S.seed_theta;
  if (S.net) {
    double* th = (double*)(base + L.net);
    const lms_status st = lms_host::net_infer_enqueue(S.net, d_xy, nullptr, 1, p.n, kNetPoints,
                                                      th, nullptr, base + L.net + 256, s);
    if (st != LMS_OK) return st;
    seed_theta = th;
  }
  mark();
  // Seeds: exact FP64 widths of a few slopes set the screen's bound: the
  // device seed slopes, the extreme-x and random pairs, and with window pairs
  // two rounds of pairs drawn from the narrowest window found so far. Without
  // pruning the bound stays +inf and the screen keeps every pair whose
  // anchored window can hold h points at all.
  double* tmp = (double*)(base + L.sort_tmp);
  if (n_seed_theta > 0 && !S.no_prune) {
    if (p.n <= kSeedExactMax || S.final_slots <= 0)
      launch_eval(s, (int)std::min<int64_t>(n_seed_theta, 4 * cu), d_xy, p.n, p.h, seed_theta,
                  (int)n_seed_theta, nullptr, ctx, rec);
    else  // larger sets: the split sort (chunk sorts in registers, one merge)
      launch_recheck(s, p.n, (int)std::min<int64_t>(n_seed_theta, 4 * cu), d_xy, ctx, entries,
                     rec, 0, (int)n_seed_theta, 1, tmp,
                     (int)std::min<int64_t>(n_seed_theta, S.final_slots),
                     p.n > 4096 ? 64 : 32, seed_theta);
  }
  const int first_w = 1 + seeds;
  if (window_pairs)
    hipLaunchKernelGGL(k_window_pairs, dim3(1), dim3(kWinNT), 0, s, d_xy, ctx, rec,
                       (int)n_seed_theta, entries, first_w, window_pairs, key ^ 0xA1ull);
  // up to kSeedExactMax points one workgroup sorts a seed's intercepts
  // faster than the histogram levels take, and the window is exact
  auto seed_windows = [&](int grid, int begin, int end, int upd) {
    if (p.n <= kSeedExactMax)
      launch_recheck(s, p.n, grid, d_xy, ctx, entries, res, begin, end, upd, nullptr, 0, 0);
    else
      launch_seed_bounds(s, p.n, grid, d_xy, ctx, entries, res, begin, end, upd);
  };
  seed_windows(std::min(first_w + window_pairs, 4 * cu), 0, first_w + window_pairs,
               S.no_prune ? 0 : 1);
  if (window_pairs) {
    // second round: from the narrowest window of the first round's pairs
    hipLaunchKernelGGL(k_window_pairs, dim3(1), dim3(kWinNT), 0, s, d_xy, ctx, res + first_w,
                       window_pairs, entries, first_w + window_pairs, window_pairs, key ^ 0xA2ull);
    seed_windows(std::min(window_pairs, 4 * cu), first_w + window_pairs, p.n_seeds, 1);
  }
  // Slope range of the slope-bin screen: exact windows at kGrid slopes around
  // the best seed slope (they may lower W too), then the range, the key
  // buckets and the anchors it leaves.
  unsigned* perm = (unsigned*)(base + L.range);
  uint2* live = (uint2*)(perm + p.n_pad);
  double2* sxy = (double2*)(live + p.n_pad);
  if (S.range) {
    double* grid_theta = (double*)(base + L.grid);
    double4* grid_res = (double4*)(grid_theta + 2 * kGrid);
    hipLaunchKernelGGL(k_grid_slopes<256>, dim3(1), dim3(256), 0, s, ctx, res, p.n_seeds,
                       n_seed_theta > 0 ? rec : nullptr, (int)n_seed_theta, grid_theta);
    auto eval_grid = [&](double* th, double4* out) {
      if (p.n <= kSeedExactMax)
        launch_eval(s, kGrid, d_xy, p.n, p.h, th, kGrid, nullptr, ctx, out);
      else
        launch_recheck(s, p.n, kGrid, d_xy, ctx, entries, out, 0, kGrid, 1, tmp, kGrid, kGrid, th);
    };
    eval_grid(grid_theta, grid_res);
    if (S.refine) {
      hipLaunchKernelGGL(k_grid_refine, dim3(1), dim3(64), 0, s, ctx, grid_theta, grid_res);
      eval_grid(grid_theta + kGrid, grid_res + kGrid);
    }
    launch_range(s, p.n, cu, d_xy, ctx, grid_theta, grid_res, S.refine, perm, sxy, live);
  }
  mark();
  // Screen. With slope bins: per-anchor bin counts, then the FP32 test of the
  // pairs they pass, and the exhaustive FP32 screen only if their list could
  // overflow and did. Without: the exhaustive FP32 screen.
  hipError_t err = hipSuccess;
  if (S.use_bins) {
    uint2* cands = (uint2*)(base + L.cands);
    err = launch_bins(s, S.bins_log2, cu, p.n, d_xy, ctx, cands, (int)S.cand_cap, entries,
                      (int)p.cap, res, n_seed_theta > 0 && !S.no_prune ? rec : nullptr,
                      (int)n_seed_theta, perm, sxy, S.range ? live : nullptr);
    mark();
    // the exhaustive screen, should the list overflow, runs in the same launch
    if (err == hipSuccess)
      err = launch_list(s, p.R, p.lds, cu, d_xy, xy32, ctx, cands, (int)S.cand_cap, entries,
                        (int)p.cap, p.nq, S.G, S.ipa,
                        S.pairs > S.cand_cap ? (int)S.n_items : 0);
  } else {
    mark();  // no slope-bin stage
    err = launch_screen(s, p.R, p.lds, cu, d_xy, xy32, ctx, entries, (int)p.cap, S.G, S.ipa,
                        (int)S.n_items, p.nq);
  }
  if (err != hipSuccess)
    return fail(LMS_ERR_DEVICE, std::string("screen launch: ") + hipGetErrorString(err));
  mark();
  // survivors: usually few; their number is known only on the device
  launch_recheck(s, p.n, std::min(S.final_slots > 0 ? S.final_slots : 4 * cu, 4 * cu), d_xy, ctx,
                 entries, res, p.n_seeds, (int)p.cap, 0, tmp, S.final_slots,
                 p.n > 4096 ? 64 : 32);
  mark();
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinalNT), 0, s, ctx, entries, res, (int)p.cap,
                     S.out);
  mark();
  err = hipGetLastError();
  if (err != hipSuccess) return fail(LMS_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(err));
  return LMS_OK;
}

// Graph replay of single solves (LMS_F_GRAPH): one captured graph, with its
// own workspace, per (input, output, stream, problem and option values).
struct SolveKey {
  const void* xy;
  const void* out;
  const void* seed_theta;
  const void* net;
  void* stream;
  int64_t n_seed_theta;
  int n, h, seeds, window_pairs, bins_log2, R, G;
  unsigned flags;
  long long cand_cap, cap;
  bool operator<(const SolveKey& o) const {
    return std::tie(xy, out, seed_theta, net, stream, n_seed_theta, n, h, seeds, window_pairs,
                    bins_log2, R, G, flags, cand_cap, cap) <
           std::tie(o.xy, o.out, o.seed_theta, o.net, o.stream, o.n_seed_theta, o.n, o.h, o.seeds,
                    o.window_pairs, o.bins_log2, o.R, o.G, o.flags, o.cand_cap, o.cap);
  }
};
struct SolveGraph {
  char* base = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};
std::mutex g_smu;
std::map<SolveKey, SolveGraph> g_solves;

lms_status solve_graph(const Setup& S, hipStream_t s) {
  const SolveKey key{S.xy,       S.out,         S.seed_theta,  S.net,    (void*)s,
                     S.n_seed_theta, S.p.n,     S.p.h,         S.seeds,  S.window_pairs,
                     S.bins_log2, S.p.R,        S.G,           S.flags,  S.cand_cap,
                     S.p.cap};
  std::lock_guard<std::mutex> lk(g_smu);
  auto it = g_solves.find(key);
  if (it == g_solves.end()) {
    SolveGraph sg;
    if (hipMalloc(&sg.base, S.L.total) != hipSuccess) {
      (void)hipGetLastError();
      return fail(LMS_ERR_NOMEM, "hipMalloc of the graph workspace failed");
    }
    // capture on a private stream (the legacy null stream cannot be captured)
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
      (void)hipFree(sg.base);
      return fail(LMS_ERR_DEVICE, "hipStreamCreate failed");
    }
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipStreamDestroy(cs);
      (void)hipFree(sg.base);
      return fail(LMS_ERR_DEVICE, "hipStreamBeginCapture failed");
    }
    const lms_status st = enqueue_solve(S, sg.base, cs, nullptr);
    const hipError_t e = hipStreamEndCapture(cs, &sg.graph);
    (void)hipStreamDestroy(cs);
    if (st != LMS_OK || e != hipSuccess || !sg.graph ||
        hipGraphInstantiate(&sg.exec, sg.graph, nullptr, nullptr, 0) != hipSuccess) {
      if (sg.graph) (void)hipGraphDestroy(sg.graph);
      (void)hipFree(sg.base);
      (void)hipGetLastError();
      return st != LMS_OK ? st : fail(LMS_ERR_DEVICE, "capturing the solve graph failed");
    }
    it = g_solves.emplace(key, sg).first;
  }
  lms_host::StageEvents prof;
  prof.start(s);
  if (hipGraphLaunch(it->second.exec, s) != hipSuccess)
    return fail(LMS_ERR_DEVICE, "hipGraphLaunch failed");
  for (int k = 0; k < LMS_NSTAGES; ++k) prof.mark();  // the whole graph is stage 0
  prof.finish();
  return LMS_OK;
}

// ---------------------------------------------------------------- allocation-free solves

// lms_solve_noalloc's workspace: one file-scope device array, held by each
// GPU the library runs on until the process ends. Host code never passes the
// array's name to a kernel (in host code it is only a stand-in for the
// symbol); its device address is looked up once per device with
// hipGetSymbolAddress and kept here.
constexpr size_t kScratchBytes = size_t(LMS_NOALLOC_WORKSPACE);
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch;  // device -> device address of `scratch`

lms_status scratch_address(char** ptr) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(LMS_ERR_DEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LMS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e));
    it = g_scratch.emplace(dev, (char*)p).first;
  }
  *ptr = it->second;
  return LMS_OK;
}

void release_solves() {
  std::lock_guard<std::mutex> lk(g_smu);
  for (auto& kv : g_solves) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    if (kv.second.base) (void)hipFree(kv.second.base);
  }
  g_solves.clear();
}

}  // namespace

// ---------------------------------------------------------------- C ABI

extern "C" {

const char* lms_status_str(int s) {
  switch (s) {
    case LMS_OK: return "ok";
    case LMS_OK_DEGENERATE: return "ok (all x equal: slope set to 0)";
    case LMS_ERR_ARG: return "invalid argument";
    case LMS_ERR_NONFINITE: return "non-finite coordinate";
    case LMS_ERR_DEVICE: return "HIP device error";
    case LMS_ERR_NOMEM: return "out of device memory";
    case LMS_ERR_CAPACITY: return "survivor list overflow";
    default: return "unknown status";
  }
}

const char* lms_last_error(void) { return lms_host::last_error(); }

lms_status lms_solve(const double* d_xy, int64_t n, int64_t h, lms_result* d_out,
                     const lms_options* opt, void* stream) {
  lms_host::clear_error();
  Setup S;
  lms_status st = make_setup(d_xy, n, h, d_out, opt, &S);
  if (st != LMS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (S.flags & LMS_F_GRAPH) return solve_graph(S, s);
  char* base = nullptr;
  st = lms_host::get_workspace(0, stream, S.L.total, &base);
  if (st != LMS_OK) return st;
  lms_host::StageEvents prof;
  prof.start(s);
  st = enqueue_solve(S, base, s, &prof);
  prof.finish();
  return st;
}

lms_status lms_workspace_size(int64_t n, int64_t h, const lms_options* opt, uint64_t* bytes) {
  lms_host::clear_error();
  if (!bytes) return fail(LMS_ERR_ARG, "null pointer");
  Setup S;
  // the setup only reads the pointers' values: any non-null placeholder works
  static const double dummy_xy[2] = {0.0, 0.0};
  static lms_result dummy_out;
  const lms_status st = make_setup(dummy_xy, n, h, &dummy_out, opt, &S);
  if (st != LMS_OK) return st;
  *bytes = (uint64_t)S.L.total;
  return LMS_OK;
}

lms_status lms_solve_noalloc(const double* d_xy, int64_t n, int64_t h, lms_result* d_out,
                             const lms_options* opt, void* stream) {
  lms_host::clear_error();
  if (opt && opt->struct_size < offsetof(lms_options, max_workspace))
    return fail(LMS_ERR_ARG, "bad options size");
  if (opt && (opt->flags & LMS_F_GRAPH))
    return fail(LMS_ERR_ARG, "lms_solve_noalloc builds no graph of its own (the caller may "
                             "capture the stream)");
  // the solve's lists shrink to fit the static workspace (lms_solve's
  // max_workspace rule); the caller's limit, if smaller, still applies
  lms_options o;
  std::memset(&o, 0, sizeof(o));
  o.seed_pairs = -1;  // the defaults lms_solve takes for opt == NULL
  if (opt) std::memcpy(&o, opt, std::min<size_t>(opt->struct_size, sizeof(o)));
  o.struct_size = sizeof(o);
  if (o.max_workspace == 0 || o.max_workspace > kScratchBytes) o.max_workspace = kScratchBytes;
  Setup S;
  lms_status st = make_setup(d_xy, n, h, d_out, &o, &S);
  if (st == LMS_ERR_NOMEM)
    return fail(LMS_ERR_ARG, "this solve needs more than the " + std::to_string(kScratchBytes) +
                                 " bytes of lms_solve_noalloc's workspace");
  if (st != LMS_OK) return st;
  char* base = nullptr;
  st = scratch_address(&base);
  if (st != LMS_OK) return st;
  return enqueue_solve(S, base, (hipStream_t)stream, nullptr);
}

lms_status lms_autotune(const double* d_xy, int64_t n, int64_t h, int32_t reps, void* stream,
                        lms_tuning* out) {
  lms_host::clear_error();
  if (!d_xy || n < 2 || n > LMS_MAX_N || reps < 1 || reps > 100)
    return fail(LMS_ERR_ARG, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  lms_result* d_res = nullptr;
  if (hipMalloc(&d_res, sizeof(lms_result)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LMS_ERR_NOMEM, "hipMalloc failed");
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  lms_status st = LMS_OK;
  lms_result ref{}, got{};
  bool have_ref = false;
  // median time of `reps` solves with option set o; checks the line against
  // the defaults' (the first candidate)
  auto time_opts = [&](lms_options& o, double* ms) -> lms_status {
    lms_status r = lms_solve(d_xy, n, h, d_res, &o, stream);  // warm-up, sizes the workspace
    if (r != LMS_OK) return r;
    if (hipMemcpyAsync(&got, d_res, sizeof(got), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(LMS_ERR_DEVICE, "reading a tuning result failed");
    if (!have_ref) {
      ref = got;
      have_ref = true;
    } else if (got.width != ref.width || got.theta1 != ref.theta1 || got.z_lo != ref.z_lo ||
               got.z_hi != ref.z_hi || got.status != ref.status) {
      return fail(LMS_ERR_DEVICE, "a tuning candidate changed the result");
    }
    std::vector<float> t(reps);
    for (int k = 0; k < reps; ++k) {
      (void)hipEventRecord(e0, s);
      r = lms_solve(d_xy, n, h, d_res, &o, stream);
      (void)hipEventRecord(e1, s);
      if (r != LMS_OK) return r;
      if (hipEventSynchronize(e1) != hipSuccess) return fail(LMS_ERR_DEVICE, "event failed");
      (void)hipEventElapsedTime(&t[k], e0, e1);
    }
    std::sort(t.begin(), t.end());
    *ms = t[reps / 2];
    return LMS_OK;
  };
  auto base_opts = [&]() {
    lms_options o;
    std::memset(&o, 0, sizeof(o));
    o.struct_size = sizeof(o);
    return o;
  };
  // explicit defaults, so that a table entry from an earlier tuning does not
  // leak into the candidates
  lms_tuning best{pick_R((int)n), 4, kDefaultSeeds, default_bins_log2((int)n), 1e30, 0, 0};
  // bins per anchor down to n / 2 (below 2 n the screen takes its WIDE form)
  int min_bins = 11;
  while (min_bins < 15 && (1 << min_bins) < n / 2) ++min_bins;
  best.bins_log2 = std::max(best.bins_log2, min_bins);
  // 1. the screen's bins, the slope range and the seeds
  static const int kSeedsC[] = {kDefaultSeeds, 63, 255};
  static const int kRangeC[] = {0, 1, -1};
  for (int bl = min_bins; bl <= 15 && st == LMS_OK; ++bl)
    for (int rg : kRangeC)
      for (int sp : kSeedsC) {
        lms_options o = base_opts();
        o.seed_pairs = sp;
        o.bins_log2 = bl;
        o.tile_regs = best.tile_regs >= 64 ? 64 : best.tile_regs;
        o.tile_batches = best.tile_batches;
        o.flags = rg > 0 ? LMS_F_RANGE : (rg < 0 ? LMS_F_NO_RANGE : 0u);
        double ms = 0;
        st = time_opts(o, &ms);
        if (st != LMS_OK) break;
        if (ms < best.ms) {
          best.seed_pairs = sp;
          best.bins_log2 = bl;
          best.range = rg;
          best.ms = ms;
        }
      }
  // 2. the FP32 screen's tiles, with the choice of step 1
  const int auto_R = pick_R((int)n);
  static const int kRegs[] = {0, 32, 16};
  static const int kBatches[] = {1, 4};
  for (int r : kRegs) {
    if (st != LMS_OK) break;
    if (r != 0 && r >= auto_R) continue;  // only fewer register chunks than automatic
    for (int g : kBatches) {
      lms_options o = base_opts();
      o.seed_pairs = best.seed_pairs;
      o.bins_log2 = best.bins_log2;
      o.flags = best.range > 0 ? LMS_F_RANGE : (best.range < 0 ? LMS_F_NO_RANGE : 0u);
      o.tile_regs = r == 0 ? 64 : r;
      o.tile_batches = g;
      double ms = 0;
      st = time_opts(o, &ms);
      if (st != LMS_OK) break;
      if (ms < best.ms) {
        best.tile_regs = o.tile_regs;
        best.tile_batches = g;
        best.ms = ms;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(d_res);
  if (st != LMS_OK) return st;
  lms_host::set_tuning(kPathSingle, lms_host::size_class((int)n), best);
  if (out) *out = best;
  return LMS_OK;
}

lms_status lms_solve_host(const double* xy, int64_t n, int64_t h, lms_result* out,
                          const lms_options* opt) {
  lms_host::clear_error();
  if (!xy || !out) return fail(LMS_ERR_ARG, "null pointer");
  if (n < 2 || n > LMS_MAX_N) return fail(LMS_ERR_ARG, "n out of range");
  if (opt && opt->n_seed_theta > 0) return fail(LMS_ERR_ARG, "device seed slopes need lms_solve");
  hipStream_t s;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
    return fail(LMS_ERR_DEVICE, "hipStreamCreate failed");
  double* d_xy = nullptr;
  lms_result* d_out = nullptr;
  lms_status st = LMS_OK;
  if (hipMalloc(&d_xy, (size_t)n * 2 * sizeof(double)) != hipSuccess ||
      hipMalloc(&d_out, sizeof(lms_result)) != hipSuccess) {
    st = fail(LMS_ERR_NOMEM, "hipMalloc failed");
  }
  if (st == LMS_OK &&
      hipMemcpyAsync(d_xy, xy, (size_t)n * 2 * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
    st = fail(LMS_ERR_DEVICE, "hipMemcpy failed");
  if (st == LMS_OK) st = lms_solve(d_xy, n, h, d_out, opt, s);
  if (st == LMS_OK &&
      (hipMemcpyAsync(out, d_out, sizeof(lms_result), hipMemcpyDeviceToHost, s) != hipSuccess ||
       hipStreamSynchronize(s) != hipSuccess))
    st = fail(LMS_ERR_DEVICE, "result copy failed");
  if (st == LMS_OK && out->status < 0) st = (lms_status)out->status;
  (void)hipStreamSynchronize(s);
  lms_host::free_workspace(0, (void*)s);  // keyed by this temporary stream
  if (d_xy) (void)hipFree(d_xy);
  if (d_out) (void)hipFree(d_out);
  (void)hipStreamDestroy(s);
  return st;
}

lms_status lms_eval_slopes(const double* d_xy, int64_t n, int64_t h, const double* d_theta,
                           int64_t m, double* d_out, void* stream) {
  lms_host::clear_error();
  Plan p;
  lms_status st = make_plan(d_xy, n, h, &p);
  if (st != LMS_OK) return st;
  if (m < 0 || m > INT_MAX || (m > 0 && (!d_theta || !d_out)))
    return fail(LMS_ERR_ARG, "bad slope array");
  if (m == 0) return LMS_OK;
  launch_eval((hipStream_t)stream, (int)std::min<int64_t>(m, 8 * lms_host::num_cu()), d_xy, p.n, p.h,
              d_theta, (int)m, d_out, nullptr);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(LMS_ERR_DEVICE, hipGetErrorString(err));
  return LMS_OK;
}

lms_status lms_screen_pairs(const double* d_xy, int64_t n, int64_t h, double W,
                            const int32_t* d_pairs, int64_t m, int32_t* d_verdict, void* stream) {
  lms_host::clear_error();
  Plan p;
  lms_status st = make_plan(d_xy, n, h, &p);
  if (st != LMS_OK) return st;
  if (m < 0 || m > INT_MAX || (m > 0 && (!d_pairs || !d_verdict)))
    return fail(LMS_ERR_ARG, "bad pair array");
  if (!(W >= 0.0)) return fail(LMS_ERR_ARG, "W must be >= 0");
  if (m == 0) return LMS_OK;
  p.n_seeds = 1;
  p.cap = 1;
  const Layout L = layout(p.n_pad, p.cap);
  char* base = nullptr;
  st = lms_host::get_workspace(0, stream, L.total, &base);
  if (st != LMS_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  Ctx* ctx = (Ctx*)(base + L.ctx);
  float2* xy32 = (float2*)(base + L.xy32);
  uint2* entries = (uint2*)(base + L.entries);
  launch_prep(s, d_xy, p.n, p.h, p.n_pad, ctx, xy32, entries, 1, 0, 0ull, 0u, 0);
  hipError_t err = launch_pairs(s, p.R, p.lds, d_xy, xy32, ctx, W, d_pairs, (int)m, d_verdict, p.nq);
  if (err != hipSuccess) return fail(LMS_ERR_DEVICE, hipGetErrorString(err));
  return LMS_OK;
}

void lms_tuning_clear(void) { lms_host::clear_tuning(); }

void lms_profile_begin(void) { lms_host::profile_begin(); }

int64_t lms_profile_end(double* ms) { return lms_host::profile_end(ms); }

void lms_shutdown(void) {
  release_solves();
  lms_host::release_batches();
  lms_host::free_workspaces();
}

}  // extern "C"
