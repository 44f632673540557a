// Batched exact LMS: many independent point sets in one pass of persistent
// kernels, optionally captured in a hipGraph.
//
// Motivation: the paper follows a coarse Hough transform with one LMS fit
// per accumulator peak, on the points that voted for it (Section 5). That is
// many small, uneven problems. Launching one solve per problem leaves the GPU
// idle between tiny kernels. Here every stage covers all problems at once:
//
//   k_bprep     one block per problem: n, h, finiteness, centring, the padded
//               FP32 copy, seed pairs.
//   k_bwindow   FP64 windows of the seed pairs (per-problem width bound W_b),
//               later of the screen survivors that k_bmerge_* keep.
//   k_bscreen   persistent wavefronts over work items (problem, anchor), the
//               same band and split tests as the single-problem screen, with
//               the number of 64-point chunks of each problem as a runtime
//               bound. One launch per register class (up to 512, 1024, 2048
//               and 4096 points).
//   k_bmerge_*  survivors of one problem with bit-identical slopes share one
//               FP64 window: a hash set keeps the smallest pair per slope.
//   k_bselect   canonical minimum per problem, (width, theta, z_lo, pair), in
//               three passes of order-preserving u64 atomicMin over the
//               entries.
//   k_bfinal    one lms_result per problem.
//
// Every counter and key is initialised by a kernel (no memset nodes), so the
// whole sequence replays from a captured graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include <cstddef>

#include "lms.h"
#include "lms_device.h"
#include "lms_host.h"

namespace {

using namespace lms_dev;
using lms_host::fail;

constexpr int kBatchMaxN = 4096;
constexpr int kClasses = 4;
constexpr int kClassChunks[kClasses] = {8, 16, 32, 64};  // n <= 512, 1024, 2048, 4096
constexpr long long kBatchScreenCap = 1ll << 24;  // FP64 survivor slots
constexpr long long kBatchCandCap = 1ll << 26;    // slope-bin list slots per class
constexpr int kBatchSeeds = 31;   // default random seed pairs per problem
constexpr int kPathBatched = 1;   // tuning-table key of lms_solve_batched
constexpr int kSmallBinsLog2 = 12;  // default bins of the small classes' screen

// Per-problem state in device memory.
struct __align__(16) PMeta {
  int off, n, h, pad_off;
  int R, status, all_x_equal;
  unsigned overflow;  // a survivor of this problem found no list slot
  double xh, yh, xabs, yabs;
  unsigned long long wbound;
  unsigned long long best_w, best_th, best_lo, best_pair;
  double best_hi;
  unsigned long long vertical, survivors, evals, dir_evals, band_pass, bin_pass;
  double center;  // slope of the narrowest seed window (centre of the bin map)
  double pad2;
  double fx, fy;  // scales of the FP32 copy (powers of two; f32_scale)
};

struct __align__(16) BState {
  unsigned n_entries, overflow;
  unsigned next_item[kClasses];
  unsigned n_reps;
  unsigned cand_overflow;        // bit c: the slope-bin list of class c overflowed
  unsigned n_cands[kClasses];    // list slots reserved by the slope-bin screen, per class
};

// Slot of the hash set that merges survivors of equal slope: key (slope bits,
// problem), value the smallest pair key (lo << 16 | hi) seen with that key.
struct __align__(16) Slot {
  unsigned long long th;
  unsigned prob, pair;
};
constexpr unsigned kNoSlot = 0xFFFFFFFFu;
constexpr int kProbes = 64;

// Entry: problem id and the pair packed as lo | hi << 16 (n <= 4096).
__device__ __forceinline__ unsigned pack_pair(unsigned lo, unsigned hi) { return lo | (hi << 16); }
constexpr unsigned kInvalidPair = 0xFFFFFFFEu;

__device__ __forceinline__ double key_to_double(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  return __longlong_as_double((long long)b);
}

// ---------------------------------------------------------------- prep

__global__ __launch_bounds__(256) void k_bprep(const double* __restrict__ xy,
                                               const int64_t* __restrict__ offsets,
                                               const int* __restrict__ d_h, int B,
                                               const int* __restrict__ pad_off,
                                               const int* __restrict__ chunks, PMeta* meta,
                                               float2* __restrict__ xy32, uint2* __restrict__ entries,
                                               int S, BState* state, unsigned long long seed_key) {
  __shared__ double s_mn[256], s_mx[256], s_my[256], s_My[256];
  __shared__ int s_amn[256], s_amx[256], s_fin[256];
  const int b = blockIdx.x, t = threadIdx.x;
  if (b == 0 && t == 0) {
    BState st;
    memset(&st, 0, sizeof(st));
    st.n_entries = (unsigned)B * (unsigned)S;
    *state = st;
  }
  const int off = (int)offsets[b];
  const int n = (int)(offsets[b + 1] - offsets[b]);
  const int h = d_h ? d_h[b] : n / 2 + 1;
  double mnx = INFINITY, mxx = -INFINITY, mny = INFINITY, mxy = -INFINITY;
  int amn = INT_MAX, amx = INT_MAX, fin = 1;
  for (int k = t; k < n; k += blockDim.x) {
    const double x = xy[2 * (off + k)], y = xy[2 * (off + k) + 1];
    if (!isfinite(x) || !isfinite(y)) fin = 0;
    if (x < mnx) { mnx = x; amn = k; }
    if (x > mxx) { mxx = x; amx = k; }
    mny = fmin(mny, y);
    mxy = fmax(mxy, y);
  }
  s_mn[t] = mnx; s_mx[t] = mxx; s_my[t] = mny; s_My[t] = mxy;
  s_amn[t] = amn; s_amx[t] = amx; s_fin[t] = fin;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) {
      const int u = t + s;
      if (s_mn[u] < s_mn[t] || (s_mn[u] == s_mn[t] && s_amn[u] < s_amn[t])) {
        s_mn[t] = s_mn[u]; s_amn[t] = s_amn[u];
      }
      if (s_mx[u] > s_mx[t] || (s_mx[u] == s_mx[t] && s_amx[u] < s_amx[t])) {
        s_mx[t] = s_mx[u]; s_amx[t] = s_amx[u];
      }
      s_my[t] = fmin(s_my[t], s_my[u]);
      s_My[t] = fmax(s_My[t], s_My[u]);
      s_fin[t] &= s_fin[u];
    }
    __syncthreads();
  }
  const double minx = s_mn[0], maxx = s_mx[0], miny = s_my[0], maxy = s_My[0];
  int status = LMS_OK;
  if (n < 2 || n > kBatchMaxN || h < 2 || h > n) status = LMS_ERR_ARG;
  else if (!s_fin[0]) status = LMS_ERR_NONFINITE;
  const bool ok = status == LMS_OK;
  const double cx = minx + 0.5 * (maxx - minx), cy = miny + 0.5 * (maxy - miny);
  const int R = chunks[b];
  if (t == 0) {
    PMeta m;
    memset(&m, 0, sizeof(m));
    m.off = off; m.n = n; m.h = h; m.pad_off = pad_off[b]; m.R = R;
    m.status = status;
    m.all_x_equal = ok && (minx == maxx);
    if (ok) {
      m.xh = fmax(fabs(minx - cx), fabs(maxx - cx)) * (1.0 + 0x1p-40);
      m.yh = fmax(fabs(miny - cy), fabs(maxy - cy)) * (1.0 + 0x1p-40);
      m.fx = f32_scale(m.xh);
      m.fy = f32_scale(m.yh);
      m.xabs = fmax(fabs(minx), fabs(maxx));
      m.yabs = fmax(fabs(miny), fabs(maxy));
    }
    m.wbound = 0x7FF0000000000000ull;
    m.best_w = m.best_th = m.best_lo = m.best_pair = ~0ull;
    meta[b] = m;
  }
  const float qnan = __int_as_float(0x7FC00000);
  const int po = pad_off[b];
  // the scales thread 0 stored (same inputs, same operations)
  const double fx = f32_scale(fmax(fabs(minx - cx), fabs(maxx - cx)) * (1.0 + 0x1p-40));
  const double fy = f32_scale(fmax(fabs(miny - cy), fabs(maxy - cy)) * (1.0 + 0x1p-40));
  for (int k = t; k < 64 * R; k += blockDim.x) {
    float2 p = make_float2(qnan, qnan);
    if (ok && k < n)
      p = make_float2((float)((xy[2 * (off + k)] - cx) * fx),
                      (float)((xy[2 * (off + k) + 1] - cy) * fy));
    xy32[po + k] = p;
  }
  for (int e = t; e < S; e += blockDim.x) {
    unsigned code = kInvalidPair;
    if (ok && e == 0) {
      code = (minx == maxx) ? kDegenerate
                            : pack_pair((unsigned)min(s_amn[0], s_amx[0]),
                                        (unsigned)max(s_amn[0], s_amx[0]));
    } else if (ok && minx != maxx) {
      const unsigned long long r =
          mix64(seed_key + 0x9E3779B97F4A7C15ull * ((unsigned long long)b * 4096u + e + 1));
      const unsigned a = (unsigned)((r >> 32) % (unsigned long long)n);
      unsigned c = (unsigned)((r & 0xFFFFFFFFull) % (unsigned long long)(n - 1));
      if (c >= a) ++c;
      code = pack_pair(min(a, c), max(a, c));
    }
    entries[(size_t)b * S + e] = make_uint2((unsigned)b, code);
  }
}

// ---------------------------------------------------------------- FP64 windows

// FP64 window of each entry in [begin, end): pair slope, fma intercepts, a
// bitonic sort of next_pow2(n_b) values in LDS, narrowest window. Lowers the
// problem's best width key, and with update_bound also its screen bound.
// window_f64 of a set of up to NMAX <= 512 points by a one-wavefront block:
// the n2 (power of two) values are sorted in registers (sort_regs, no LDS
// pass and no barrier), the same network as window_f64_rt's, so the same
// result bit for bit.
template <int NMAX>
__device__ __forceinline__ void window_wave(const double* __restrict__ xy, int n, int h, int n2,
                                            double theta, double* z, double* w, double* lo,
                                            double* hi) {
  static_assert(NMAX <= 512, "at most 8 values per lane");
  if (n2 <= 64)
    window_f64<64, 64>(xy, n, h, theta, z, w, lo, hi);
  else if (n2 <= 128)
    window_f64<128, 64>(xy, n, h, theta, z, w, lo, hi);
  else if (NMAX >= 256 && n2 <= 256)
    window_f64<(NMAX >= 256 ? 256 : 64), 64>(xy, n, h, theta, z, w, lo, hi);
  else
    window_f64<NMAX, 64>(xy, n, h, theta, z, w, lo, hi);
}

template <int NMAX, int NT>
__global__ __launch_bounds__(NT) void k_bwindow(const double* __restrict__ xy, PMeta* meta,
                                                const uint2* __restrict__ entries,
                                                double4* __restrict__ res, int begin,
                                                const BState* state, int fixed_end, int cap,
                                                int update_bound,
                                                const unsigned* __restrict__ reps) {
  __shared__ double z[NMAX];
  // entries [begin, fixed_end), or the listed representatives
  const unsigned end = reps ? min(state->n_reps, (unsigned)cap)
                            : fixed_end >= 0 ? (unsigned)fixed_end
                                             : min(state->n_entries, (unsigned)cap);
  for (unsigned k = (reps ? 0u : (unsigned)begin) + blockIdx.x; k < end; k += gridDim.x) {
    const unsigned e = reps ? reps[k] : k;
    const uint2 en = entries[e];
    const PMeta m = meta[en.x];
    if (m.status != LMS_OK || en.y == kInvalidPair) {
      if (threadIdx.x == 0) res[e] = make_double4(INFINITY, NAN, NAN, NAN);
      continue;
    }
    double theta = 0.0;
    if (en.y != kDegenerate) {
      const int lo = m.off + (int)(en.y & 0xFFFFu), hi = m.off + (int)(en.y >> 16);
      const double xl = xy[2 * lo], xr = xy[2 * hi];
      if (xl == xr) {
        if (threadIdx.x == 0) res[e] = make_double4(INFINITY, NAN, NAN, NAN);
        continue;
      }
      theta = (xy[2 * hi + 1] - xy[2 * lo + 1]) / (xr - xl);
    }
    int n2 = 64;
    while (n2 < m.n) n2 <<= 1;
    double w, lo, hi;
    if constexpr (NT == 64)  // one wavefront: the sort runs in registers
      window_wave<NMAX>(xy + 2 * m.off, m.n, m.h, n2, theta, z, &w, &lo, &hi);
    else
      window_f64_rt<NMAX, NT>(xy + 2 * m.off, m.n, m.h, n2, theta, z, &w, &lo, &hi);
    if (threadIdx.x == 0) {
      res[e] = make_double4(w, theta, lo, hi);
      if (w == w) atomicMin(&meta[en.x].best_w, (unsigned long long)__double_as_longlong(w));
      if (update_bound && w == w)
        atomicMin(&meta[en.x].wbound, (unsigned long long)__double_as_longlong(
                                          width_bound(w, theta, m.xabs, m.yabs)));
    }
  }
}

// ---------------------------------------------------------------- screen

// Work item = (problem, anchor i): all partners j = (i + o) mod n, o = 1..P(i),
// in batches of 64. items[k] = (problem, anchor) of the k-th item of one
// register class, numbered problem by problem with the largest problems first.
// fallback = 1: runs only if the slope-bin list of this class overflowed,
// which has then already counted and listed the vertical and forced pairs.
template <int RMAX>
__global__ __launch_bounds__(256, 3) void k_bscreen(
    const double* __restrict__ xy, const float2* __restrict__ xy32, PMeta* meta,
    const uint2* __restrict__ items, int n_items, uint2* __restrict__ entries, int cap,
    BState* state, int cls, int fallback) {
  const int lane = threadIdx.x & 63;
  if (fallback && !((state->cand_overflow >> cls) & 1u)) return;
  for (;;) {
    int item = 0;
    if (lane == 0) item = (int)atomicAdd(&state->next_item[cls], 1u);
    item = __shfl(item, 0);
    if (item >= n_items) break;
    const uint2 it = items[item];
    const int b = __builtin_amdgcn_readfirstlane((int)it.x);
    const int i = __builtin_amdgcn_readfirstlane((int)it.y);
    const PMeta m = meta[b];
    if (m.status != LMS_OK || m.all_x_equal) continue;
    // per-problem scalars, made explicitly wave-uniform (SGPRs)
    const int n = __builtin_amdgcn_readfirstlane(m.n);
    const int h = __builtin_amdgcn_readfirstlane(m.h);
    const int Rb = __builtin_amdgcn_readfirstlane(m.R);
    const int poff = __builtin_amdgcn_readfirstlane(m.pad_off);
    const int goff = __builtin_amdgcn_readfirstlane(m.off);
    const float2* pts = xy32 + poff;
    const float2 pi = pts[i];
    const float2* src = pts;
    asm volatile("" : "+s"(src));
    float X[RMAX], Y[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) {
      if (r < Rb) {
        const float2 p = src[lane + 64 * r];
        X[r] = p.x - pi.x;
        Y[r] = p.y - pi.y;
      }
    }
    const int half = n >> 1;
    const int P = (n & 1) ? half : (i < half ? half : half - 1);
    const double* gxy = xy + 2 * goff;
    const double W = __longlong_as_double((long long)m.wbound);
    unsigned long long n_vert = 0, n_evals = 0, n_devals = 0, n_band = 0, n_keep = 0;
    for (int o0 = 1; o0 <= P; o0 += 64) {
      const int o = o0 + lane;
      const bool valid = o <= P;
      int j = i + (valid ? o : 1);
      if (j >= n) j -= n;
      const int lo = min(i, j), hi = max(i, j);
      const double xl = gxy[2 * lo], yl = gxy[2 * lo + 1];
      const double xr = gxy[2 * hi], yr = gxy[2 * hi + 1];
      const bool vert = valid && (xl == xr);
      const double th = (yr - yl) / (xr - xl);
      const ScreenScalars sc = screen_scalars(th, W, m.fx, m.fy, m.xh, m.yh);
      const bool force = valid && !vert && sc.force;
      const bool test = valid && !vert && !force;
      const float th32 = test ? sc.th32 : 0.0f;
      const float thr = test ? sc.thr : 0.0f;
      const float ta = test ? sc.ta : 0.0f;
      if (!fallback) n_vert += __popcll(__ballot(vert));
      unsigned long long msk = __ballot(test);
      // lanes whose pair is appended
      unsigned long long kept = fallback ? 0ull : __ballot(force);
      while (msk) {
        const int cl = __ffsll((long long)msk) - 1;
        msk &= msk - 1;
        const PairTest pt = test_pair_rt<RMAX>(X, Y, Rb, -lane_f(th32, cl), lane_f(thr, cl),
                                               lane_f(ta, cl), h);
        n_evals += (unsigned)pt.band_chunks;
        if (pt.split_chunks >= 0) {
          ++n_band;
          n_devals += (unsigned)pt.split_chunks;
        }
        if (pt.keep) kept |= 1ull << cl;
      }
      // one reservation per batch of 64 partners; each kept lane writes its
      // own entry
      if (kept) {
        const unsigned cnt = (unsigned)__popcll(kept);
        unsigned base = 0;
        if (lane == 0) {
          // no reservation once the list is full, so the counter never wraps
          const unsigned now = __hip_atomic_load(&state->n_entries, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
          base = now >= (unsigned)cap ? (unsigned)cap : atomicAdd(&state->n_entries, cnt);
        }
        base = __shfl(base, 0);
        if ((kept >> lane) & 1ull) {
          const unsigned idx = base + (unsigned)__popcll(kept & ((1ull << lane) - 1ull));
          if (idx < (unsigned)cap) {
            entries[idx] = make_uint2((unsigned)b, pack_pair(lo, hi));
          } else {
            atomicOr(&state->overflow, 1u);
            atomicOr(&meta[b].overflow, 1u);
          }
        }
        n_keep += cnt;
      }
    }
    if (lane == 0) {
      if (n_vert) atomicAdd(&meta[b].vertical, n_vert);
      if (n_keep) atomicAdd(&meta[b].survivors, n_keep);
      atomicAdd(&meta[b].evals, 64ull * n_evals);
      if (n_band) {
        atomicAdd(&meta[b].band_pass, n_band);
        atomicAdd(&meta[b].dir_evals, 64ull * n_devals);
      }
    }
  }
}

// ---------------------------------------------------------------- slope-bin screen

// Centre of each problem's bin map: the slope of its narrowest seed window.
__global__ __launch_bounds__(256) void k_bcenter(const double4* __restrict__ res, PMeta* meta,
                                                 int B, int S) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double bw = INFINITY, th = 0.0;
  for (int e = 0; e < S; ++e) {
    const double4 r = res[(size_t)b * S + e];
    if (r.x < bw) {
      bw = r.x;
      th = r.y;
    }
  }
  meta[b].center = th;
}

// One work item (problem b, anchor i) at a time per block, items taken
// round-robin (no shared counter): the two window intervals of every point of
// b in NB slope bins (see add_point_bins), their prefix sum, and each
// partner's bounds on its window counts from the bin of its slope. Passing
// pairs go to the class's list as (b, i | j << 16); a block reserves list
// slots kReserve at a time and marks the slots it leaves unused with
// kNoProblem. Forced slopes go straight to the FP64 entries.
constexpr unsigned kNoProblem = 0xFFFFFFFFu;
constexpr unsigned kReserve = 512;

template <int NB, int NT>
__global__ __launch_bounds__(NT) void k_bbins(const double* __restrict__ xy, PMeta* meta,
                                              const uint2* __restrict__ items, int n_items,
                                              uint2* __restrict__ cands, int cand_cap,
                                              uint2* __restrict__ entries, int cap, BState* state,
                                              int cls) {
  // NB + NT bins, an odd number per thread in the prefix sum, and one word
  // for the decrements past the last bin
  constexpr int NBINS = NB + NT;
  constexpr int kRLog = __builtin_ctz(NB) - 1;  // the map spans bins [3, NB + 3]
  static_assert((NB % NT) == 0 && ((NB / NT) & 1) == 0, "bins must be 2^k per thread");
  __shared__ __align__(16) unsigned bins[(NBINS + 4) & ~3];  // whole 16-byte words
  __shared__ unsigned short list[NB / 2];  // partner offsets o - 1 (P <= n / 2 <= NB / 2)
  __shared__ unsigned s_part[NT / 64 > 0 ? NT / 64 : 1];
  __shared__ unsigned s_all, s_cnt, s_next, s_end;
  const int t = threadIdx.x, lane = t & 63;
  if (t == 0) s_next = s_end = 0;  // reserved list slots [s_next, s_end)
  for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
    __syncthreads();  // the previous item's queries are done with the bins
    if (t == 0) {
      s_all = 0;
      s_cnt = 0;
    }
    for (int b = t; b < (NBINS + 4) / 4; b += NT) reinterpret_cast<uint4*>(bins)[b] = uint4{};
    __syncthreads();
    const uint2 it = items[item];
    const int b = __builtin_amdgcn_readfirstlane((int)it.x);
    const int i = __builtin_amdgcn_readfirstlane((int)it.y);
    const PMeta m = meta[b];
    if (m.status != LMS_OK || m.all_x_equal) continue;
    const int n = __builtin_amdgcn_readfirstlane(m.n);
    const int h = __builtin_amdgcn_readfirstlane(m.h);
    const double* gxy = xy + 2 * m.off;
    const double W = __longlong_as_double((long long)m.wbound);
    const double lim = W * (1.0 + 0x1p-50);
    const BinFrame F = bin_frame(m.center, m.xh, m.yh, W, NBINS);
    const double xi = gxy[2 * i], yi = gxy[2 * i + 1];
    const double2* pts = reinterpret_cast<const double2*>(gxy);
    unsigned all = 0;
    // the next point's load is issued before this point's work
    double2 nxt = t < n ? pts[t] : make_double2(0.0, 0.0);
    for (int k = t; k < n; k += NT) {
      const double2 cur = nxt;
      if (k + NT < n) nxt = pts[k + NT];
      add_point_bins<kRLog>(bins, cur.x - xi, cur.y - yi, W, lim, F, all);
    }
#pragma unroll
    for (int q = 32; q >= 1; q >>= 1) all += __shfl_xor(all, q);
    if (lane == 0) atomicAdd(&s_all, all);
    __syncthreads();
    scan_bins<NBINS, NT>(bins, s_part);
    __syncthreads();
    const unsigned pall = s_all;
    const int half = n >> 1;
    const int P = (n & 1) ? half : (i < half ? half : half - 1);
    unsigned long long n_vert = 0, n_forced = 0, n_pass = 0;  // per wavefront (uniform)
    const double th_lim = screen_th_lim(m.fx, m.fy, m.xh, m.yh);
    auto partner = [&](int o) { return i + o >= n ? i + o - n : i + o; };
    double2 pn = 1 + t <= P ? pts[partner(1 + t)] : make_double2(0.0, 0.0);
    for (int o0 = 1; o0 <= P; o0 += NT) {
      const int o = o0 + t;
      const bool valid = o <= P;
      const int j = partner(valid ? o : 1);
      const int lo = min(i, j), hi = max(i, j);
      // the pair's bin and FP64 hand-off as in k_bins
      const double2 pj = pn;  // the next partner's load goes out first
      if (o + NT <= P) pn = pts[partner(o + NT)];
      const double dx = pj.x - xi, dy = pj.y - yi, adx = fabs(dx);
      const bool vert = valid && dx == 0.0;
      const double r = recip(dx);
      const double th = dy * r;
      const bool ok = adx >= 0x1p-900 && adx <= 0x1p900 && fabs(th) < th_lim;
      const bool force = valid && !vert && !ok;
      const bool test = valid && !vert && ok;
      const bool pass = test && bins_pass(bins[slope_bin<kRLog>(dx, dy, r, F)], pall, h);
      const unsigned long long mf = __ballot(force), mp = __ballot(pass);
      n_vert += __popcll(__ballot(vert));
      n_forced += __popcll(mf);
      n_pass += __popcll(mp);
      if (mf) {
        unsigned base = 0;
        if (lane == 0) {
          const unsigned now = __hip_atomic_load(&state->n_entries, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
          base = now >= (unsigned)cap ? (unsigned)cap
                                      : atomicAdd(&state->n_entries, (unsigned)__popcll(mf));
        }
        base = __shfl(base, 0);
        if (force) {
          const unsigned idx = base + (unsigned)__popcll(mf & ((1ull << lane) - 1ull));
          if (idx < (unsigned)cap) {
            entries[idx] = make_uint2((unsigned)b, pack_pair(lo, hi));
          } else {
            atomicOr(&state->overflow, 1u);
            atomicOr(&meta[b].overflow, 1u);
          }
        }
      }
      if (mp) {
        unsigned base = 0;
        if (lane == 0) base = atomicAdd(&s_cnt, (unsigned)__popcll(mp));
        base = __shfl(base, 0);
        if (pass) list[base + __popcll(mp & ((1ull << lane) - 1ull))] = (unsigned short)(o - 1);
      }
    }
    if (lane == 0) {
      if (n_vert) atomicAdd(&meta[b].vertical, n_vert);
      if (n_forced) atomicAdd(&meta[b].survivors, n_forced);
      if (n_pass) atomicAdd(&meta[b].bin_pass, n_pass);
    }
    __syncthreads();
    const unsigned cnt = s_cnt;
    if (cnt) {
      unsigned first = s_next;
      if (s_end - first < cnt) {  // not enough reserved: mark the rest unused, reserve more
        for (unsigned q = first + t; q < s_end; q += NT)
          cands[q] = make_uint2(kNoProblem, 0u);
        __syncthreads();
        if (t == 0) {
          const unsigned want = cnt > kReserve ? cnt : kReserve;
          const unsigned now = __hip_atomic_load(&state->n_cands[cls], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
          const unsigned got = now >= (unsigned)cand_cap ? (unsigned)cand_cap
                                                         : atomicAdd(&state->n_cands[cls], want);
          s_next = got;
          s_end = got >= (unsigned)cand_cap ? got : min(got + want, (unsigned)cand_cap);
          if (s_end - s_next < cnt) atomicOr(&state->cand_overflow, 1u << cls);
        }
        __syncthreads();
        first = s_next;
      }
      const unsigned room = s_end - first;
      for (unsigned q = t; q < cnt && q < room; q += NT) {
        int j = i + 1 + (int)list[q];
        if (j >= n) j -= n;
        cands[first + q] = make_uint2((unsigned)b, (unsigned)i | ((unsigned)j << 16));
      }
      __syncthreads();
      if (t == 0) s_next = first + min(cnt, room);
    }
  }
  __syncthreads();
  for (unsigned q = s_next + t; q < s_end; q += NT) cands[q] = make_uint2(kNoProblem, 0u);
}

// The same screen with one work item per wavefront, for small problems
// (n <= 1024): the per-item steps (clear, insert, prefix sum, queries) are
// short, and the block-wide barriers between them left most of the time to
// latency. Here each wavefront owns a histogram of NB + 64 bins in LDS and
// runs its items with no block barrier; a wavefront's LDS operations execute
// in order, so only compiler reordering needs fencing. A wavefront takes
// chunks of kItemChunk consecutive items (mostly anchors of one problem),
// keeps the problem's points in registers while the problem lasts, and stores
// each point's query code in LDS during the insertion (add_point_bins_coded),
// so the queries read LDS only. Passes go to the class's list from a
// per-wavefront reservation window.
// Prefix sums of the NB + 64 bins by one wavefront, in two parts: lane l
// takes bins l S .. l S + S - 1 (S odd, so the lanes read distinct banks) and
// leaves their running sums in place; loff[l] gets the sum of the lanes before
// it. Bin q's prefix sum is then bins[q] + loff[q / S] (wave_bin_sum), which
// saves the second pass over the bins that adding the offsets would cost.
template <int NB>
__device__ __forceinline__ void wave_scan_bins(unsigned* bins, unsigned* loff) {
  constexpr int S = (NB + 64) / 64;
  static_assert(S * 64 == NB + 64 && (S & 1), "bins per lane must be odd");
  const int lane = threadIdx.x & 63;
  unsigned run = 0;
#pragma unroll
  for (int r = 0; r < S; ++r) {
    run += bins[lane * S + r];
    bins[lane * S + r] = run;
  }
  unsigned x = run;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    const unsigned y = __shfl_up(x, m);
    if (lane >= m) x += y;
  }
  loff[lane] = x - run;
}

template <int NB>
__device__ __forceinline__ unsigned wave_bin_sum(const unsigned* bins, const unsigned* loff,
                                                 unsigned q) {
  constexpr unsigned S = (NB + 64) / 64;
  return bins[q] + loff[q / S];
}

__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Lane l's value of v (uniform).
__device__ __forceinline__ double lane_d(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

constexpr int kItemChunk = 16;

template <int NB, int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_bbins_wave(
    const double* __restrict__ xy, PMeta* meta, const uint2* __restrict__ items, int n_items,
    uint2* __restrict__ cands, int cand_cap, uint2* __restrict__ entries, int cap, BState* state,
    int cls) {
  constexpr int NBINS = NB + 64;
  constexpr int kRLog = __builtin_ctz(NB) - 1;
  constexpr int kMaxN = 1024, RMAX = kMaxN / 64;
  constexpr unsigned kWaveReserve = 256;
  // (rows of whole 16-byte words, for the clearing stores)
  __shared__ __align__(16) unsigned s_bins[WAVES][(NBINS + 4) & ~3];
  __shared__ unsigned short s_list[WAVES][kMaxN / 2];
  __shared__ unsigned short s_code[WAVES][kMaxN];
  __shared__ unsigned s_loff[WAVES][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  unsigned* bins = s_bins[wv];
  unsigned* loff = s_loff[wv];
  unsigned short* list = s_list[wv];
  unsigned short* code = s_code[wv];
  unsigned w_next = 0, w_end = 0;  // this wavefront's reserved list slots (uniform)
  const int n_chunks = (n_items + kItemChunk - 1) / kItemChunk;
  const int stride = gridDim.x * WAVES;
  // the current problem (uniform): its metadata and points (lane l holds
  // points l + 64 r, r < R)
  int cur = -1, n = 0, h = 0, R = 0;
  bool skip = true;
  double W = 0.0, lim = 0.0, th_lim = 0.0;
  BinFrame F{0.0, 0.0, 0.0};
  double X[RMAX], Y[RMAX];
  for (int ch = blockIdx.x * WAVES + wv; ch < n_chunks; ch += stride) {
    const int i0 = ch * kItemChunk;
    const int cnt_items = min(kItemChunk, n_items - i0);
    const uint2 my = lane < cnt_items ? items[i0 + lane] : make_uint2(0u, 0u);
    for (int q = 0; q < cnt_items; ++q) {
      const int b = __builtin_amdgcn_readlane((int)my.x, q);
      const int i = __builtin_amdgcn_readlane((int)my.y, q);
      if (b != cur) {
        cur = b;
        const PMeta m = meta[b];
        skip = m.status != LMS_OK || m.all_x_equal;
        n = __builtin_amdgcn_readfirstlane(m.n);
        h = __builtin_amdgcn_readfirstlane(m.h);
        R = (n + 63) >> 6;
        W = __longlong_as_double((long long)m.wbound);
        lim = W * (1.0 + 0x1p-50);
        F = bin_frame(m.center, m.xh, m.yh, W, NBINS);
        th_lim = screen_th_lim(m.fx, m.fy, m.xh, m.yh);
        const double2* pts = reinterpret_cast<const double2*>(xy + 2 * m.off);
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
          if (r < R) {
            const double2 p = pts[min(lane + 64 * r, n - 1)];
            X[r] = p.x;
            Y[r] = p.y;
          }
        }
      }
      if (skip) continue;
      // the anchor, read from the lane that holds it
      const int ri = i >> 6, li = i & 63;
      double xi = 0.0, yi = 0.0;
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        if (r == ri) {
          xi = lane_d(X[r], li);
          yi = lane_d(Y[r], li);
        }
      }
      wave_fence();  // the previous item's queries are done with the bins and codes
      for (int q2 = lane; q2 < (NBINS + 4) / 4; q2 += 64)
        reinterpret_cast<uint4*>(bins)[q2] = uint4{};
      wave_fence();
      unsigned all = 0;
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        const int k = lane + 64 * r;
        if (r < R && k < n)
          add_point_bins_coded<kRLog>(bins, X[r] - xi, Y[r] - yi, W, lim, F, th_lim, &code[k],
                                      all);
      }
#pragma unroll
      for (int q2 = 32; q2 >= 1; q2 >>= 1) all += __shfl_xor(all, q2);
      wave_fence();
      wave_scan_bins<NB>(bins, loff);
      wave_fence();
      const unsigned pall = all;
      const int half = n >> 1;
      const int P = (n & 1) ? half : (i < half ? half : half - 1);
      unsigned long long n_vert = 0, n_forced = 0, n_pass = 0;  // uniform
      auto partner = [&](int o) { return i + o >= n ? i + o - n : i + o; };
      unsigned cnt = 0;  // passes listed so far (uniform)
      for (int o0 = 1; o0 <= P; o0 += 64) {
        const int o = o0 + lane;
        const bool valid = o <= P;
        const int j = partner(min(o, P));
        const unsigned cj = code[j];
        // read for every lane, with no branch (codes 0..2 read bins 0..2,
        // which no test uses)
        const unsigned pb = wave_bin_sum<NB>(bins, loff, cj);
        const unsigned long long mv = __ballot(valid);
        const unsigned long long mf = __ballot(cj == kCodeFP64) & mv;
        const unsigned long long mp = __ballot(bins_pass(pb, pall, h)) & __ballot(cj > kCodePass) & mv;
        const bool force = (mf >> lane) & 1ull, pass = (mp >> lane) & 1ull;
        n_vert += __popcll(__ballot(cj == kCodeVertical) & mv);
        n_forced += __popcll(mf);
        n_pass += __popcll(mp);
        if (mf) {
          unsigned base = 0;
          if (lane == 0) {
            const unsigned now = __hip_atomic_load(&state->n_entries, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            base = now >= (unsigned)cap ? (unsigned)cap
                                        : atomicAdd(&state->n_entries, (unsigned)__popcll(mf));
          }
          base = __shfl(base, 0);
          if (force) {
            const unsigned idx = base + (unsigned)__popcll(mf & ((1ull << lane) - 1ull));
            if (idx < (unsigned)cap) {
              entries[idx] = make_uint2((unsigned)b, pack_pair(min(i, j), max(i, j)));
            } else {
              atomicOr(&state->overflow, 1u);
              atomicOr(&meta[b].overflow, 1u);
            }
          }
        }
        if (pass) list[cnt + __popcll(mp & ((1ull << lane) - 1ull))] = (unsigned short)(o - 1);
        cnt += (unsigned)__popcll(mp);
      }
      if (lane == 0) {
        if (n_vert) atomicAdd(&meta[b].vertical, n_vert);
        if (n_forced) atomicAdd(&meta[b].survivors, n_forced);
        if (n_pass) atomicAdd(&meta[b].bin_pass, n_pass);
      }
      if (cnt) {
        wave_fence();  // the list entries are written
        if (w_end - w_next < cnt) {  // mark the rest unused, reserve more
          for (unsigned q2 = w_next + lane; q2 < w_end; q2 += 64u)
            cands[q2] = make_uint2(kNoProblem, 0u);
          const unsigned want = cnt > kWaveReserve ? cnt : kWaveReserve;
          unsigned got = 0;
          if (lane == 0) {
            const unsigned now = __hip_atomic_load(&state->n_cands[cls], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            got = now >= (unsigned)cand_cap ? (unsigned)cand_cap
                                            : atomicAdd(&state->n_cands[cls], want);
          }
          got = __shfl(got, 0);
          w_next = got;
          w_end = got >= (unsigned)cand_cap ? got : min(got + want, (unsigned)cand_cap);
          if (w_end - w_next < cnt && lane == 0) atomicOr(&state->cand_overflow, 1u << cls);
        }
        const unsigned room = w_end - w_next;
        for (unsigned q2 = lane; q2 < cnt && q2 < room; q2 += 64u) {
          int j = i + 1 + (int)list[q2];
          if (j >= n) j -= n;
          cands[w_next + q2] = make_uint2((unsigned)b, (unsigned)i | ((unsigned)j << 16));
        }
        w_next += min(cnt, room);
      }
    }
  }
  for (unsigned q = w_next + lane; q < w_end; q += 64u) cands[q] = make_uint2(kNoProblem, 0u);
}

// FP32 test of the listed pairs of one register class: a wavefront takes 64
// consecutive list entries and, for each distinct (problem, anchor) among
// them, loads that problem's points shifted by the anchor and runs the band
// and split tests on its pairs.
constexpr int kBListBlock = 32;
constexpr unsigned kEntryReserve = 256;

template <int RMAX>
__global__ __launch_bounds__(256, 3) void k_bscreen_list(
    const double* __restrict__ xy, const float2* __restrict__ xy32, PMeta* meta,
    const uint2* __restrict__ cands, int cand_cap, uint2* __restrict__ entries, int cap,
    BState* state, int cls) {
  const int lane = threadIdx.x & 63;
  if ((state->cand_overflow >> cls) & 1u) return;
  const unsigned total = min(state->n_cands[cls], (unsigned)cand_cap);
  const unsigned n_blocks = (total + kBListBlock - 1u) / kBListBlock;
  const unsigned n_waves = gridDim.x * (blockDim.x / 64u);
  const unsigned w0 = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / 64u) +
                                                     threadIdx.x / 64u);
  // Per-problem counters accumulate while consecutive groups share a problem;
  // survivor slots are reserved kEntryReserve at a time per wavefront, and
  // slots left unused are marked kInvalidPair.
  int cur = -1;
  unsigned long long a_evals = 0, a_devals = 0, a_band = 0, a_keep = 0;
  unsigned e_next = 0, e_end = 0;
  auto flush_counts = [&]() {
    if (cur >= 0 && lane == 0) {
      if (a_keep) atomicAdd(&meta[cur].survivors, a_keep);
      if (a_evals) atomicAdd(&meta[cur].evals, 64ull * a_evals);
      if (a_band) {
        atomicAdd(&meta[cur].band_pass, a_band);
        atomicAdd(&meta[cur].dir_evals, 64ull * a_devals);
      }
    }
    a_evals = a_devals = a_band = a_keep = 0;
  };
  for (unsigned blk = w0; blk < n_blocks; blk += n_waves) {
    const unsigned e = blk * kBListBlock + (unsigned)lane;
    uint2 cd = make_uint2(0u, 0u);
    bool valid = false;
    if (lane < kBListBlock && e < total) {
      cd = cands[e];
      valid = cd.x != kNoProblem;
    }
    const int cb = (int)cd.x, ci = (int)(cd.y & 0xFFFFu), cj = (int)(cd.y >> 16);
    unsigned long long todo = __ballot(valid);
    while (todo) {
      const int l0 = __ffsll((long long)todo) - 1;
      const int b = lane_i(cb, l0), i = lane_i(ci, l0);
      const unsigned long long mine = __ballot(valid && cb == b && ci == i) & todo;
      todo &= ~mine;
      const PMeta m = meta[b];
      const int h = __builtin_amdgcn_readfirstlane(m.h);
      const int Rb = __builtin_amdgcn_readfirstlane(m.R);
      const int poff = __builtin_amdgcn_readfirstlane(m.pad_off);
      const float2* pts = xy32 + poff;
      const float2 pi = pts[i];
      const float2* src = pts;
      asm volatile("" : "+s"(src));
      float X[RMAX], Y[RMAX];
#pragma unroll
      for (int r = 0; r < RMAX; ++r) {
        if (r < Rb) {
          const float2 p = src[lane + 64 * r];
          X[r] = p.x - pi.x;
          Y[r] = p.y - pi.y;
        }
      }
      const bool me = (mine >> lane) & 1ull;
      const int j = me ? cj : (i == 0 ? 1 : 0);
      const int lo = min(i, j), hi = max(i, j);
      const double* gxy = xy + 2 * m.off;
      const double xl = gxy[2 * lo], yl = gxy[2 * lo + 1];
      const double xr = gxy[2 * hi], yr = gxy[2 * hi + 1];
      const double th = (yr - yl) / (xr - xl);
      const double W = __longlong_as_double((long long)m.wbound);
      const ScreenScalars sc = screen_scalars(th, W, m.fx, m.fy, m.xh, m.yh);
      const float th32 = me ? sc.th32 : 0.0f;
      const float thr = me ? sc.thr : 0.0f;
      const float ta = me ? sc.ta : 0.0f;
      if (b != cur) {
        flush_counts();
        cur = b;
      }
      unsigned long long kept = 0;
      unsigned long long msk = mine;
      while (msk) {
        const int cl = __ffsll((long long)msk) - 1;
        msk &= msk - 1;
        const PairTest pt = test_pair_rt<RMAX>(X, Y, Rb, -lane_f(th32, cl), lane_f(thr, cl),
                                               lane_f(ta, cl), h);
        a_evals += (unsigned)pt.band_chunks;
        if (pt.split_chunks >= 0) {
          ++a_band;
          a_devals += (unsigned)pt.split_chunks;
        }
        if (pt.keep) kept |= 1ull << cl;
      }
      if (kept) {
        const unsigned cnt = (unsigned)__popcll(kept);
        a_keep += cnt;
        if (e_end - e_next < cnt) {
          for (unsigned q = e_next + (unsigned)lane; q < e_end; q += 64u)
            entries[q] = make_uint2(0u, kInvalidPair);
          unsigned got = 0;
          const unsigned want = cnt > kEntryReserve ? cnt : kEntryReserve;
          if (lane == 0) {
            const unsigned now = __hip_atomic_load(&state->n_entries, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            got = now >= (unsigned)cap ? (unsigned)cap : atomicAdd(&state->n_entries, want);
          }
          got = __shfl(got, 0);
          e_next = got;
          e_end = got >= (unsigned)cap ? got : min(got + want, (unsigned)cap);
          if (e_end - e_next < cnt && lane == 0) {
            atomicOr(&state->overflow, 1u);
            atomicOr(&meta[b].overflow, 1u);
          }
        }
        if ((kept >> lane) & 1ull) {
          const unsigned idx = e_next + (unsigned)__popcll(kept & ((1ull << lane) - 1ull));
          if (idx < e_end) entries[idx] = make_uint2((unsigned)b, pack_pair(lo, hi));
        }
        e_next = min(e_next + cnt, e_end);
      }
    }
  }
  flush_counts();
  for (unsigned q = e_next + (unsigned)lane; q < e_end; q += 64u)
    entries[q] = make_uint2(0u, kInvalidPair);
}

// The same tests for problems up to 512 points with one listed pair per lane:
// a wavefront takes 64 consecutive list entries and, for each problem among
// them, stages the problem's FP32 points in LDS and streams them to every
// lane (broadcast reads). Each lane evaluates its own pair's residuals
// d = fma(-theta32, x_k - x_i, y_k - y_i) (the same operations as
// test_pair_rt, so the same decisions) and counts, in its own registers,
// the points above ta and thr and below -ta and -thr: then
// B = n - #(d > thr) - #(d < -thr), P = #(d > ta) - #(d > thr) and
// N = #(d < -ta) - #(d < -thr), and the pair survives iff B >= h and
// (P <= B - h or N <= B - h). No ballot or scalar count per point: the
// lanes-as-points kernel spent twice as many scalar as vector instructions.
constexpr int kLanesMaxN = 512;

template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void k_bscreen_lanes(
    const double* __restrict__ xy, const float2* __restrict__ xy32, PMeta* meta,
    const uint2* __restrict__ cands, int cand_cap, uint2* __restrict__ entries, int cap,
    BState* state, int cls) {
  __shared__ float2 s_pts[WAVES][kLanesMaxN];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if ((state->cand_overflow >> cls) & 1u) return;
  float2* pts = s_pts[wv];
  const unsigned total = min(state->n_cands[cls], (unsigned)cand_cap);
  const unsigned n_blocks = (total + 63u) / 64u;
  const unsigned n_waves = gridDim.x * WAVES;
  unsigned e_next = 0, e_end = 0;  // reserved survivor slots (uniform)
  for (unsigned blk = blockIdx.x * WAVES + wv; blk < n_blocks; blk += n_waves) {
    const unsigned e = blk * 64u + (unsigned)lane;
    uint2 cd = make_uint2(0u, 0u);
    bool valid = false;
    if (e < total) {
      cd = cands[e];
      valid = cd.x != kNoProblem;
    }
    const int cb = (int)cd.x, ci = (int)(cd.y & 0xFFFFu), cj = (int)(cd.y >> 16);
    unsigned long long todo = __ballot(valid);
    while (todo) {
      const int l0 = __ffsll((long long)todo) - 1;
      const int b = lane_i(cb, l0);
      const unsigned long long mine = __ballot(valid && cb == b) & todo;
      todo &= ~mine;
      const bool me = (mine >> lane) & 1ull;
      const PMeta m = meta[b];
      const int n = __builtin_amdgcn_readfirstlane(m.n);
      const int h = __builtin_amdgcn_readfirstlane(m.h);
      const int Rb = __builtin_amdgcn_readfirstlane(m.R);
      const int poff = __builtin_amdgcn_readfirstlane(m.pad_off);
      wave_fence();  // the previous problem's reads of pts are done
      for (int k = lane; k < n; k += 64) pts[k] = xy32[poff + k];
      wave_fence();
      // this lane's pair: FP64 slope, FP32 test scalars, anchor
      const int i = me ? ci : 0, j = me ? cj : 1;
      const int lo = min(i, j), hi = max(i, j);
      const double* gxy = xy + 2 * m.off;
      const double th = (gxy[2 * hi + 1] - gxy[2 * lo + 1]) / (gxy[2 * hi] - gxy[2 * lo]);
      const double W = __longlong_as_double((long long)m.wbound);
      const ScreenScalars sc = screen_scalars(th, W, m.fx, m.fy, m.xh, m.yh);
      const float nth = me ? -sc.th32 : 0.0f;
      const float thr = sc.thr, ta = sc.ta;
      const float2 pi = pts[i];
      int gt_ta = 0, gt_thr = 0, lt_ta = 0, lt_thr = 0;
      int k = 0;
      for (; k + 4 <= n; k += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float2 p = pts[k + u];
          const float d = fmaf(nth, p.x - pi.x, p.y - pi.y);
          gt_ta += d > ta;
          gt_thr += d > thr;
          lt_ta += d < -ta;
          lt_thr += d < -thr;
        }
      }
      for (; k < n; ++k) {
        const float2 p = pts[k];
        const float d = fmaf(nth, p.x - pi.x, p.y - pi.y);
        gt_ta += d > ta;
        gt_thr += d > thr;
        lt_ta += d < -ta;
        lt_thr += d < -thr;
      }
      const int B = n - gt_thr - lt_thr;
      const bool band = me && B >= h;
      const bool keep = band && (gt_ta - gt_thr <= B - h || lt_ta - lt_thr <= B - h);
      const unsigned long long kept = __ballot(keep);
      const unsigned long long nb = (unsigned long long)__popcll(__ballot(band));
      if (lane == 0) {
        const unsigned long long np = (unsigned long long)__popcll(mine);
        atomicAdd(&meta[b].evals, 64ull * (unsigned long long)Rb * np);
        if (nb) {
          atomicAdd(&meta[b].band_pass, nb);
          atomicAdd(&meta[b].dir_evals, 64ull * (unsigned long long)Rb * nb);
        }
        if (kept) atomicAdd(&meta[b].survivors, (unsigned long long)__popcll(kept));
      }
      if (kept) {
        const unsigned cnt = (unsigned)__popcll(kept);
        if (e_end - e_next < cnt) {
          for (unsigned q = e_next + (unsigned)lane; q < e_end; q += 64u)
            entries[q] = make_uint2(0u, kInvalidPair);
          unsigned got = 0;
          const unsigned want = cnt > kEntryReserve ? cnt : kEntryReserve;
          if (lane == 0) {
            const unsigned now = __hip_atomic_load(&state->n_entries, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            got = now >= (unsigned)cap ? (unsigned)cap : atomicAdd(&state->n_entries, want);
          }
          got = __shfl(got, 0);
          e_next = got;
          e_end = got >= (unsigned)cap ? got : min(got + want, (unsigned)cap);
          if (e_end - e_next < cnt && lane == 0) {
            atomicOr(&state->overflow, 1u);
            atomicOr(&meta[b].overflow, 1u);
          }
        }
        if (keep) {
          const unsigned idx = e_next + (unsigned)__popcll(kept & ((1ull << lane) - 1ull));
          if (idx < e_end) entries[idx] = make_uint2((unsigned)b, pack_pair(lo, hi));
        }
        e_next = min(e_next + cnt, e_end);
      }
    }
  }
  for (unsigned q = e_next + (unsigned)lane; q < e_end; q += 64u)
    entries[q] = make_uint2(0u, kInvalidPair);
}

// ---------------------------------------------------------------- merge of equal slopes

// Survivors of one problem with bit-identical FP64 slopes have identical
// intercepts z_k = fma(-theta, x_k, y_k), hence the same window, so the
// canonical order (width, theta, z_lo, pair) among them is decided by the pair
// alone. Only the smallest pair of each (problem, slope) needs its FP64
// window; the others are marked as not evaluated. Integer data (pixel
// coordinates) gives thousands of survivors on a few slopes.
__global__ __launch_bounds__(256) void k_bmerge_clear(Slot* __restrict__ tab, unsigned size) {
  for (unsigned k = blockIdx.x * blockDim.x + threadIdx.x; k < size; k += gridDim.x * blockDim.x) {
    Slot sl;
    sl.th = ~0ull;
    sl.prob = kNoSlot;
    sl.pair = kNoSlot;
    tab[k] = sl;
  }
}

__device__ __forceinline__ unsigned pair_key(unsigned code) {
  return ((code & 0xFFFFu) << 16) | (code >> 16);  // (lo, hi) in lexicographic order
}

// Inserts every screen survivor e in [begin, end) into the set and records its
// slot (kNoSlot: not merged, evaluated on its own).
__global__ __launch_bounds__(256) void k_bmerge_insert(const double* __restrict__ xy,
                                                       const PMeta* __restrict__ meta,
                                                       const uint2* __restrict__ entries,
                                                       const BState* state, int begin, int cap,
                                                       Slot* __restrict__ tab, unsigned size,
                                                       unsigned* __restrict__ slot_of) {
  const unsigned end = min(state->n_entries, (unsigned)cap);
  for (unsigned e = begin + blockIdx.x * blockDim.x + threadIdx.x; e < end;
       e += gridDim.x * blockDim.x) {
    const uint2 en = entries[e];
    unsigned slot = kNoSlot;
    if (en.y != kDegenerate && en.y != kInvalidPair) {
      const int off = meta[en.x].off;
      const int lo = off + (int)(en.y & 0xFFFFu), hi = off + (int)(en.y >> 16);
      const double xl = xy[2 * lo], xr = xy[2 * hi];
      if (xl != xr) {
        // the same expression as the window kernel, hence the same bits
        const double theta = (xy[2 * hi + 1] - xy[2 * lo + 1]) / (xr - xl);
        const unsigned long long key = (unsigned long long)__double_as_longlong(theta);
        const unsigned pk = pair_key(en.y);
        unsigned s = (unsigned)mix64(key ^ (0x9E3779B97F4A7C15ull * (en.x + 1ull))) & (size - 1);
        for (int q = 0; q < kProbes; ++q, s = (s + 1) & (size - 1)) {
          const unsigned long long t = atomicCAS(&tab[s].th, ~0ull, key);
          if (t != ~0ull && t != key) continue;
          const unsigned pb = atomicCAS(&tab[s].prob, kNoSlot, en.x);
          if (pb != kNoSlot && pb != en.x) continue;
          atomicMin(&tab[s].pair, pk);
          slot = s;
          break;
        }
      }
    }
    slot_of[e] = slot;
  }
}

// Lists the survivors whose window is evaluated: those not merged and the
// smallest pair of each slot. The others get an infinite width.
__global__ __launch_bounds__(256) void k_bmerge_mark(const uint2* __restrict__ entries,
                                                     BState* state, int begin, int cap,
                                                     const Slot* __restrict__ tab,
                                                     const unsigned* __restrict__ slot_of,
                                                     unsigned* __restrict__ reps,
                                                     double4* __restrict__ res) {
  const unsigned end = min(state->n_entries, (unsigned)cap);
  const int lane = threadIdx.x & 63;
  const unsigned stride = gridDim.x * blockDim.x;
  // whole wavefronts step together so that the ballot sees every lane
  for (unsigned w0 = begin + blockIdx.x * blockDim.x + (threadIdx.x & ~63u); w0 < end;
       w0 += stride) {
    const unsigned e = w0 + lane;
    bool rep = false;
    if (e < end) {
      const unsigned code = entries[e].y;
      const unsigned s = slot_of[e];
      rep = code != kInvalidPair && (s == kNoSlot || tab[s].pair == pair_key(code));
      if (!rep) res[e] = make_double4(INFINITY, NAN, NAN, NAN);
    }
    const unsigned long long mask = __ballot(rep);
    if (!mask) continue;
    unsigned base = 0;
    if (lane == 0) base = atomicAdd(&state->n_reps, (unsigned)__popcll(mask));
    base = __shfl(base, 0);
    if (rep) reps[base + (unsigned)__popcll(mask & ((1ull << lane) - 1ull))] = e;
  }
}

// ---------------------------------------------------------------- selection

// pass 1: slope key among the narrowest; pass 2: z_lo key; pass 3: pair key
// and the window's upper end.
__global__ __launch_bounds__(256) void k_bselect(const uint2* __restrict__ entries,
                                                 const double4* __restrict__ res, PMeta* meta,
                                                 const BState* state, int cap, int pass) {
  const unsigned end = min(state->n_entries, (unsigned)cap);
  for (unsigned e = blockIdx.x * blockDim.x + threadIdx.x; e < end; e += gridDim.x * blockDim.x) {
    const double4 r = res[e];
    if (!(r.x < INFINITY)) continue;
    const uint2 en = entries[e];
    PMeta* m = &meta[en.x];
    if ((unsigned long long)__double_as_longlong(r.x) != m->best_w) continue;
    const unsigned long long kth = order_key(r.y);
    if (pass == 1) { atomicMin(&m->best_th, kth); continue; }
    if (kth != m->best_th) continue;
    const unsigned long long klo = order_key(r.z);
    if (pass == 2) { atomicMin(&m->best_lo, klo); continue; }
    if (klo != m->best_lo) continue;
    const unsigned long long kp =
        en.y == kDegenerate ? ~0ull - 1
                            : ((unsigned long long)(en.y & 0xFFFFu) << 32) | (en.y >> 16);
    atomicMin(&m->best_pair, kp);
    m->best_hi = r.w;  // equal slope => identical sorted intercepts => same window
  }
}

__global__ __launch_bounds__(256) void k_bfinal(const PMeta* __restrict__ meta, int B,
                                                const BState* state, lms_result* out, int bins) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const PMeta m = meta[b];
  lms_result o;
  memset(&o, 0, sizeof(o));
  o.h = m.h;
  int st = m.status;
  if (st >= 0 && m.overflow) st = LMS_ERR_CAPACITY;  // re-solved by the host
  if (st >= 0 && m.best_w == ~0ull) st = LMS_ERR_DEVICE;
  if (st >= 0 && m.all_x_equal) st = LMS_OK_DEGENERATE;
  o.status = st;
  const unsigned long long pairs =
      m.n >= 2 ? (unsigned long long)m.n * (unsigned long long)(m.n - 1) / 2 : 0;
  if (st < 0) {
    o.theta1 = o.theta2 = o.half_width = o.width = o.z_lo = o.z_hi = NAN;
    o.pair_i = o.pair_j = -1;
  } else {
    o.width = __longlong_as_double((long long)m.best_w);
    o.half_width = 0.5 * o.width;
    o.theta1 = key_to_double(m.best_th);
    o.z_lo = key_to_double(m.best_lo);
    o.z_hi = m.best_hi;
    o.theta2 = 0.5 * (o.z_lo + o.z_hi);
    if (m.best_pair >= ~0ull - 1) {
      o.pair_i = o.pair_j = -1;
    } else {
      o.pair_i = (int)(m.best_pair >> 32);
      o.pair_j = (int)(m.best_pair & 0xFFFFFFFFull);
    }
  }
  o.vertical = m.all_x_equal ? pairs : m.vertical;
  o.candidates = pairs - o.vertical;
  o.survivors = m.survivors;
  o.point_evals = m.evals;
  o.dir_evals = m.dir_evals;
  o.band_pass = m.band_pass;
  o.bin_pass = m.bin_pass;
  // the class's bins: the per-wavefront screen's below 1024 points
  o.bins = bins ? (m.R <= kClassChunks[1] ? (unsigned)bins : 8192u + 256u) : 0u;
  out[b] = o;
}

// ---------------------------------------------------------------- host side

// Host-side plan of a batch: per-problem padding and register class, and the
// work order of each class. Cached by the content of the offsets.
struct BPlan {
  int B = 0, S = 0, max_n = 0;
  int small_log2 = kSmallBinsLog2;  // bins of the per-wavefront screen (classes 0, 1)
  long long pad_total = 0, pairs = 0, cap = 0;
  bool may_overflow = false;  // more pairs than survivor slots: check after the pass
  int n_probs[kClasses] = {};
  int n_items[kClasses] = {};
  long long pairs_c[kClasses] = {};   // pairs per register class
  long long cand_cap[kClasses] = {};  // slope-bin list slots per class
  size_t cand_off[kClasses] = {};     // first slot of each class's list
  // device arrays inside the workspace
  size_t o_meta = 0, o_state = 0, o_pad = 0, o_chunks = 0, o_items = 0, o_xy32 = 0,
         o_entries = 0, o_res = 0, o_tab = 0, o_slot = 0, o_reps = 0, o_cands = 0, total = 0;
  size_t items_off[kClasses] = {};  // first item of each class in the item table
  unsigned tab_size = 0;            // slots of the equal-slope set (power of two)
  std::vector<int> h_pad, h_chunks;
  std::vector<unsigned> h_items;  // (problem, anchor) per work item
};

size_t up256(size_t v) { return (v + 255) & ~size_t(255); }

void layout_batch(BPlan* P);

lms_status plan_batch(const int64_t* h_off, int B, int S, uint64_t max_ws, BPlan* P) {
  P->B = B;
  P->S = S;
  P->h_pad.assign(B, 0);
  P->h_chunks.assign(B, 1);
  std::vector<std::vector<int>> cls(kClasses);
  long long pad = 0;
  for (int b = 0; b < B; ++b) {
    const long long n = h_off[b + 1] - h_off[b];
    if (n < 0) return fail(LMS_ERR_ARG, "offsets must be non-decreasing");
    if (n > kBatchMaxN)
      return fail(LMS_ERR_ARG, "batched problems hold at most 4096 points; use lms_solve");
    const int R = (int)std::max<long long>(1, (n + 63) / 64);
    P->h_chunks[b] = R;
    P->h_pad[b] = (int)pad;
    pad += 64ll * R;
    P->max_n = std::max<int>(P->max_n, (int)n);
    P->pairs += n * (n - 1) / 2;
    if (n >= 2) {
      int c = 0;
      while (R > kClassChunks[c]) ++c;
      cls[c].push_back(b);
      P->pairs_c[c] += n * (n - 1) / 2;
    }
  }
  if (h_off[0] < 0) return fail(LMS_ERR_ARG, "offsets must be >= 0");
  // the kernels index points and padded chunks with 32-bit offsets
  if (h_off[B] > (1ll << 30) || pad > (1ll << 30))
    return fail(LMS_ERR_ARG, "a batch holds at most 2^30 points");
  P->pad_total = pad;
  P->h_items.clear();
  for (int c = 0; c < kClasses; ++c) {
    auto& v = cls[c];
    // largest problems first: the tail of the persistent loop is small items
    std::stable_sort(v.begin(), v.end(), [&](int a, int b) {
      return (h_off[a + 1] - h_off[a]) > (h_off[b + 1] - h_off[b]);
    });
    P->items_off[c] = P->h_items.size() / 2;
    long long items = 0;
    for (int b : v) {
      const long long n = h_off[b + 1] - h_off[b];
      for (long long i = 0; i < n; ++i) {
        P->h_items.push_back((unsigned)b);
        P->h_items.push_back((unsigned)i);
      }
      items += n;
    }
    if (items > INT_MAX) return fail(LMS_ERR_ARG, "batch too large");
    P->n_probs[c] = (int)v.size();
    P->n_items[c] = (int)items;
  }
  const long long seeds = (long long)B * S;
  // slack for the survivor slots each wavefront reserves ahead
  P->cap = seeds + std::min<long long>(P->pairs, kBatchScreenCap) + (1ll << 20);
  if (P->cap > INT_MAX) return fail(LMS_ERR_ARG, "batch too large");
  for (int c = 0; c < kClasses; ++c)
    // slack for the slots each block reserves ahead and may leave unused
    P->cand_cap[c] = P->pairs_c[c] ? std::min<long long>(P->pairs_c[c] + (1ll << 20), kBatchCandCap)
                                   : 0;
  layout_batch(P);
  if (max_ws && P->total > max_ws) {
    // a workspace limit shrinks the pass lists (an overflowing class runs the
    // exhaustive screen instead), then the survivor list (its problems that
    // lose survivors are re-solved on their own)
    const long long kMinList = 4096;
    for (int c = 0; c < kClasses && P->total > max_ws; ++c) {
      if (P->cand_cap[c] <= kMinList) continue;
      const long long over = (long long)(P->total - max_ws);
      P->cand_cap[c] = std::max(kMinList, P->cand_cap[c] - (over + 7) / 8 - 64);
      layout_batch(P);
    }
    while (P->total > max_ws && P->cap - seeds > kMinList) {
      // entries, windows, slot and representative per survivor, and the
      // equal-slope set (about two slots per survivor)
      const long long per = (long long)(sizeof(uint2) + sizeof(double4) + 2 * sizeof(unsigned) +
                                        2 * sizeof(Slot));
      const long long over = (long long)(P->total - max_ws);
      P->cap = seeds + std::max(kMinList, P->cap - seeds - (over + per - 1) / per - 64);
      layout_batch(P);
    }
    if (P->total > max_ws)
      return fail(LMS_ERR_NOMEM, "max_workspace below the " + std::to_string(P->total) +
                                     " bytes this batch needs at the least");
  }
  // every pair could survive in the worst case; beyond the list's slots the
  // host checks for problems that lost survivors after the pass
  P->may_overflow = P->pairs + (1ll << 20) > P->cap - seeds;
  return LMS_OK;
}

// Offsets of the device arrays of a plan in its buffer (P->total: the size).
void layout_batch(BPlan* P) {
  const long long seeds = (long long)P->B * P->S;
  size_t o = 0;
  P->o_state = o; o += up256(sizeof(BState));
  P->o_meta = o; o += up256((size_t)P->B * sizeof(PMeta));
  P->o_pad = o; o += up256((size_t)P->B * sizeof(int));
  P->o_chunks = o; o += up256((size_t)P->B * sizeof(int));
  P->o_items = o; o += up256(P->h_items.size() * sizeof(unsigned) + 8);
  P->o_xy32 = o; o += up256((size_t)P->pad_total * sizeof(float2));
  P->o_entries = o; o += up256((size_t)P->cap * sizeof(uint2));
  P->o_res = o; o += up256((size_t)P->cap * sizeof(double4));
  // equal-slope set: at least twice the screen's entry capacity, at most 2^23
  // slots (128 MiB); survivors that find no slot are evaluated on their own
  unsigned ts = 256;
  while (ts < (1u << 23) && (long long)ts < 2 * (P->cap - seeds)) ts <<= 1;
  P->tab_size = ts;
  P->o_tab = o; o += up256((size_t)ts * sizeof(Slot));
  P->o_slot = o; o += up256((size_t)P->cap * sizeof(unsigned));
  P->o_reps = o; o += up256((size_t)P->cap * sizeof(unsigned));
  long long cands = 0;
  for (int c = 0; c < kClasses; ++c) {
    P->cand_off[c] = (size_t)cands;
    cands += P->cand_cap[c];
  }
  P->o_cands = o; o += up256((size_t)cands * sizeof(uint2));
  P->total = o;
}

template <int NMAX>
void launch_bwindow(hipStream_t s, int grid, const double* xy, PMeta* meta, const uint2* e,
                    double4* res, int begin, const BState* st, int fixed_end, int cap, int upd,
                    const unsigned* reps) {
  // up to 512 points one wavefront per window (twice the blocks)
  constexpr int NT = NMAX <= 512 ? 64 : (NMAX >= 2048 ? 512 : 256);
  hipLaunchKernelGGL((k_bwindow<NMAX, NT>), dim3(NT == 64 ? 2 * grid : grid), dim3(NT), 0, s, xy,
                     meta, e, res, begin, st, fixed_end, cap, upd, reps);
}

void launch_bwindow_n(hipStream_t s, int max_n, int grid, const double* xy, PMeta* meta,
                      const uint2* e, double4* res, int begin, const BState* st, int fixed_end,
                      int cap, int upd, const unsigned* reps) {
  if (max_n <= 256) launch_bwindow<256>(s, grid, xy, meta, e, res, begin, st, fixed_end, cap, upd, reps);
  else if (max_n <= 512) launch_bwindow<512>(s, grid, xy, meta, e, res, begin, st, fixed_end, cap, upd, reps);
  else if (max_n <= 1024) launch_bwindow<1024>(s, grid, xy, meta, e, res, begin, st, fixed_end, cap, upd, reps);
  else launch_bwindow<4096>(s, grid, xy, meta, e, res, begin, st, fixed_end, cap, upd, reps);
}

struct BatchKey {
  const void* xy;
  const void* off;
  const void* h;
  const void* out;
  void* stream;
  int B, S;
  bool bins;
  uint64_t max_ws;
  int small_log2;
  bool operator<(const BatchKey& o) const {
    return std::tie(xy, off, h, out, stream, B, S, bins, max_ws, small_log2) <
           std::tie(o.xy, o.off, o.h, o.out, o.stream, o.B, o.S, o.bins, o.max_ws, o.small_log2);
  }
};

// A plan with its own device buffer (plan arrays, state, FP32 copy, entries)
// and, once captured, its graph.
struct BatchCache {
  std::vector<int64_t> offsets;  // the offsets the plan was made for
  BPlan plan;
  char* base = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (base) (void)hipFree(base);
    exec = nullptr;
    graph = nullptr;
    base = nullptr;
  }
};

std::mutex g_bmu;
std::map<BatchKey, BatchCache> g_batches;

// Resident 256-thread blocks per CU of the screen kernel of class c.
int bscreen_blocks_per_cu(int c) {
  static int cached[kClasses] = {};
  if (cached[c] == 0) {
    const void* f = c == 0   ? (const void*)k_bscreen<8>
                    : c == 1 ? (const void*)k_bscreen<16>
                    : c == 2 ? (const void*)k_bscreen<32>
                             : (const void*)k_bscreen<64>;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 256, 0) != hipSuccess || nb < 1) {
      (void)hipGetLastError();
      nb = 3;
    }
    cached[c] = nb;
  }
  return cached[c];
}

void launch_bscreen(hipStream_t s, int c, int cu, const double* xy, const float2* xy32,
                    PMeta* meta, const uint2* it, int n_items, uint2* entries, int cap,
                    BState* state, int fallback) {
  // persistent blocks: as many as fit on the chip at once
  const int grid = std::max(1, std::min((n_items + 3) / 4, bscreen_blocks_per_cu(c) * cu));
  switch (c) {
    case 0:
      hipLaunchKernelGGL((k_bscreen<8>), dim3(grid), dim3(256), 0, s, xy, xy32, meta, it, n_items,
                         entries, cap, state, c, fallback);
      break;
    case 1:
      hipLaunchKernelGGL((k_bscreen<16>), dim3(grid), dim3(256), 0, s, xy, xy32, meta, it, n_items,
                         entries, cap, state, c, fallback);
      break;
    case 2:
      hipLaunchKernelGGL((k_bscreen<32>), dim3(grid), dim3(256), 0, s, xy, xy32, meta, it, n_items,
                         entries, cap, state, c, fallback);
      break;
    default:
      hipLaunchKernelGGL((k_bscreen<64>), dim3(grid), dim3(256), 0, s, xy, xy32, meta, it, n_items,
                         entries, cap, state, c, fallback);
      break;
  }
}

// Slope bins per class: 4096 up to 1024 points (pixel data with many tied
// slopes needs about 8 bins per point to keep the bounds within a few counts
// of exact), 8192 above; four wavefronts per item.
template <int NB, int NT>
void launch_bbins_nb(hipStream_t s, int c, int cu, const double* xy, PMeta* meta,
                     const uint2* it, int n_items, uint2* cands, int cand_cap, uint2* entries,
                     int cap, BState* state) {
  static int resident = 0;
  if (resident == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_bbins<NB, NT>, NT, 0) !=
            hipSuccess || nb < 1) {
      (void)hipGetLastError();
      nb = 1;
    }
    resident = nb;
  }
  const int grid = std::max(1, std::min(n_items, resident * cu));
  hipLaunchKernelGGL((k_bbins<NB, NT>), dim3(grid), dim3(NT), 0, s, xy, meta, it, n_items, cands,
                     cand_cap, entries, cap, state, c);
}

// One item per wavefront (classes 0 and 1, n <= 1024): WAVES wavefronts per
// block, each with its own histogram.
template <int NB, int WAVES>
void launch_bbins_wave(hipStream_t s, int c, int cu, const double* xy, PMeta* meta,
                       const uint2* it, int n_items, uint2* cands, int cand_cap, uint2* entries,
                       int cap, BState* state) {
  static int resident = 0;
  if (resident == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_bbins_wave<NB, WAVES>,
                                                     64 * WAVES, 0) != hipSuccess || nb < 1) {
      (void)hipGetLastError();
      nb = 1;
    }
    resident = nb;
  }
  const int grid = std::max(1, std::min((n_items + WAVES - 1) / WAVES, resident * cu));
  hipLaunchKernelGGL((k_bbins_wave<NB, WAVES>), dim3(grid), dim3(64 * WAVES), 0, s, xy, meta, it,
                     n_items, cands, cand_cap, entries, cap, state, c);
}

// Bins of the small classes' per-wavefront screen (2^small_log2 nominal).
int small_class_bins(int small_log2) { return 1 << small_log2; }

void launch_bbins(hipStream_t s, int c, int cu, int small_log2, const double* xy, PMeta* meta,
                  const uint2* it, int n_items, uint2* cands, int cand_cap, uint2* entries,
                  int cap, BState* state) {
  if (c <= 1) {
    if (small_log2 <= 11)
      launch_bbins_wave<2048, 4>(s, c, cu, xy, meta, it, n_items, cands, cand_cap, entries, cap,
                                 state);
    else
      launch_bbins_wave<4096, 2>(s, c, cu, xy, meta, it, n_items, cands, cand_cap, entries, cap,
                                 state);
    return;
  }
  launch_bbins_nb<8192, 256>(s, c, cu, xy, meta, it, n_items, cands, cand_cap, entries, cap,
                             state);
}

template <int RMAX>
void launch_bscreen_list_r(hipStream_t s, int c, int cu, const double* xy, const float2* xy32,
                           PMeta* meta, const uint2* cands, int cand_cap, uint2* entries, int cap,
                           BState* state) {
  static int resident = 0;
  if (resident == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_bscreen_list<RMAX>, 256,
                                                     0) != hipSuccess || nb < 1) {
      (void)hipGetLastError();
      nb = 1;
    }
    resident = nb;
  }
  hipLaunchKernelGGL((k_bscreen_list<RMAX>), dim3(resident * cu), dim3(256), 0, s, xy, xy32, meta,
                     cands, cand_cap, entries, cap, state, c);
}

// Problems up to 512 points (class 0): one pair per lane (k_bscreen_lanes).
void launch_bscreen_lanes(hipStream_t s, int c, int cu, const double* xy, const float2* xy32,
                          PMeta* meta, const uint2* cands, int cand_cap, uint2* entries, int cap,
                          BState* state) {
  constexpr int kWaves = 4;
  static int resident = 0;
  if (resident == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_bscreen_lanes<kWaves>,
                                                     64 * kWaves, 0) != hipSuccess || nb < 1) {
      (void)hipGetLastError();
      nb = 1;
    }
    resident = nb;
  }
  hipLaunchKernelGGL((k_bscreen_lanes<kWaves>), dim3(resident * cu), dim3(64 * kWaves), 0, s, xy,
                     xy32, meta, cands, cand_cap, entries, cap, state, c);
}

void launch_bscreen_list(hipStream_t s, int c, int cu, const double* xy, const float2* xy32,
                         PMeta* meta, const uint2* cands, int cand_cap, uint2* entries, int cap,
                         BState* state) {
  static_assert(kClassChunks[0] * 64 <= kLanesMaxN, "class 0 fits the lanes kernel");
  switch (c) {
    case 0: launch_bscreen_lanes(s, c, cu, xy, xy32, meta, cands, cand_cap, entries, cap, state); break;
    case 1: launch_bscreen_list_r<16>(s, c, cu, xy, xy32, meta, cands, cand_cap, entries, cap, state); break;
    case 2: launch_bscreen_list_r<32>(s, c, cu, xy, xy32, meta, cands, cand_cap, entries, cap, state); break;
    default: launch_bscreen_list_r<64>(s, c, cu, xy, xy32, meta, cands, cand_cap, entries, cap, state); break;
  }
}

// Enqueues the whole batched pipeline on s (capturable: kernels only).
lms_status enqueue_batch(const BPlan& P, char* base, const double* d_xy, const int64_t* d_off,
                         const int32_t* d_h, lms_result* d_out, hipStream_t s,
                         lms_host::StageEvents* prof, bool bins) {
  PMeta* meta = (PMeta*)(base + P.o_meta);
  BState* state = (BState*)(base + P.o_state);
  const int* pad = (const int*)(base + P.o_pad);
  const int* chunks = (const int*)(base + P.o_chunks);
  const uint2* items = (const uint2*)(base + P.o_items);
  Slot* tab = (Slot*)(base + P.o_tab);
  unsigned* slot_of = (unsigned*)(base + P.o_slot);
  unsigned* reps = (unsigned*)(base + P.o_reps);
  float2* xy32 = (float2*)(base + P.o_xy32);
  uint2* entries = (uint2*)(base + P.o_entries);
  double4* res = (double4*)(base + P.o_res);
  const int cu = lms_host::num_cu();
  const int cap = (int)P.cap;
  const int seeds = P.B * P.S;
  hipLaunchKernelGGL(k_bprep, dim3(P.B), dim3(256), 0, s, d_xy, d_off, d_h, P.B, pad, chunks,
                     meta, xy32, entries, P.S, state, 0xBA7C4ull);
  if (prof) prof->mark();
  launch_bwindow_n(s, P.max_n, std::min(seeds, 16 * cu), d_xy, meta, entries, res, 0, state,
                   seeds, cap, 1, nullptr);
  if (prof) prof->mark();
  hipLaunchKernelGGL(k_bmerge_clear, dim3(std::min<unsigned>(P.tab_size / 256, 8u * cu)), dim3(256), 0,
                     s, tab, P.tab_size);
  hipLaunchKernelGGL(k_bcenter, dim3((P.B + 255) / 256), dim3(256), 0, s, res, meta, P.B, P.S);
  uint2* cands = (uint2*)(base + P.o_cands);
  if (bins) {
    for (int c = 0; c < kClasses; ++c)
      if (P.n_items[c])
        launch_bbins(s, c, cu, P.small_log2, d_xy, meta, items + P.items_off[c], P.n_items[c],
                     cands + P.cand_off[c], (int)P.cand_cap[c], entries, cap, state);
  }
  if (prof) prof->mark();
  for (int c = 0; c < kClasses; ++c) {
    if (P.n_items[c] == 0) continue;
    const uint2* it = items + P.items_off[c];
    if (bins) {
      launch_bscreen_list(s, c, cu, d_xy, xy32, meta, cands + P.cand_off[c], (int)P.cand_cap[c],
                          entries, cap, state);
      // The exhaustive screen, in case the class's list overflowed (blocks
      // reserve slots ahead, so even a list sized for every pair can); it
      // returns at once otherwise.
      launch_bscreen(s, c, cu, d_xy, xy32, meta, it, P.n_items[c], entries, cap, state, 1);
    } else {
      launch_bscreen(s, c, cu, d_xy, xy32, meta, it, P.n_items[c], entries, cap, state, 0);
    }
  }
  if (prof) prof->mark();
  hipLaunchKernelGGL(k_bmerge_insert, dim3(16 * cu), dim3(256), 0, s, d_xy, meta, entries, state,
                     seeds, cap, tab, P.tab_size, slot_of);
  hipLaunchKernelGGL(k_bmerge_mark, dim3(16 * cu), dim3(256), 0, s, entries, state, seeds, cap,
                     tab, slot_of, reps, res);
  launch_bwindow_n(s, P.max_n, 16 * cu, d_xy, meta, entries, res, seeds, state, -1, cap, 0, reps);
  if (prof) prof->mark();
  for (int pass = 1; pass <= 3; ++pass)
    hipLaunchKernelGGL(k_bselect, dim3(4 * cu), dim3(256), 0, s, entries, res, meta, state, cap,
                       pass);
  hipLaunchKernelGGL(k_bfinal, dim3((P.B + 255) / 256), dim3(256), 0, s, meta, P.B, state, d_out,
                     bins ? small_class_bins(P.small_log2) + 64 : 0);
  if (prof) prof->mark();
  const hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(LMS_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(err));
  return LMS_OK;
}

// After a pass whose survivor list could overflow: wait for it, and solve
// again, one by one with lms_solve, the problems that lost survivors (status
// LMS_ERR_CAPACITY). lms_solve's own list holds every pair of a problem of
// up to kBatchMaxN points, so each gets its exact answer.
lms_status resolve_overflowed(const BatchCache& bc, const double* d_xy,
                              const std::vector<int64_t>& off, const int32_t* d_h,
                              lms_result* d_out, const lms_options* opt, hipStream_t s) {
  const int B = bc.plan.B;
  BState hs;
  if (hipMemcpyAsync(&hs, bc.base + bc.plan.o_state, sizeof(BState), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(LMS_ERR_DEVICE, "reading the batch state failed");
  if (!hs.overflow) return LMS_OK;
  std::vector<lms_result> res(B);
  std::vector<int32_t> hh(d_h ? B : 0);
  if (hipMemcpyAsync(res.data(), d_out, (size_t)B * sizeof(lms_result), hipMemcpyDeviceToHost,
                     s) != hipSuccess ||
      (d_h && hipMemcpyAsync(hh.data(), d_h, (size_t)B * sizeof(int32_t), hipMemcpyDeviceToHost,
                             s) != hipSuccess) ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(LMS_ERR_DEVICE, "reading the batch results failed");
  lms_options o;
  std::memset(&o, 0, sizeof(o));
  o.struct_size = sizeof(o);
  o.seed_pairs = -1;
  if (opt && opt->bins_log2 == -1) o.bins_log2 = -1;
  for (int b = 0; b < B; ++b) {
    if (res[b].status != LMS_ERR_CAPACITY) continue;
    const lms_status st = lms_solve(d_xy + 2 * off[b], off[b + 1] - off[b], d_h ? hh[b] : 0,
                                    d_out + b, &o, (void*)s);
    if (st != LMS_OK) return st;
  }
  return LMS_OK;
}

}  // namespace

extern "C" {

lms_status lms_solve_batched(const double* d_xy, const int64_t* d_offsets,
                             const int64_t* h_offsets, int64_t B, const int32_t* d_h,
                             lms_result* d_out, const lms_options* opt, void* stream) {
  lms_host::clear_error();
  if (!d_xy || !d_offsets || !d_out) return fail(LMS_ERR_ARG, "null pointer");
  if (B < 1 || B > (1 << 24)) return fail(LMS_ERR_ARG, "B must be in [1, 2^24]");
  if (opt && opt->struct_size < offsetof(lms_options, max_workspace))
    return fail(LMS_ERR_ARG, "bad options size");
  unsigned flags = opt ? opt->flags : 0u;
  const uint64_t max_ws =
      opt && opt->struct_size >= offsetof(lms_options, max_workspace) + sizeof(uint64_t)
          ? opt->max_workspace : 0;
  if (opt && opt->seed_pairs < -1) return fail(LMS_ERR_ARG, "seed_pairs must be >= -1");
  hipStream_t s = (hipStream_t)stream;
  std::vector<int64_t> off((size_t)B + 1);
  if (h_offsets) {
    std::memcpy(off.data(), h_offsets, off.size() * sizeof(int64_t));
  } else {
    if (hipMemcpyAsync(off.data(), d_offsets, off.size() * sizeof(int64_t), hipMemcpyDeviceToHost,
                       s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(LMS_ERR_DEVICE, "copying the offsets to the host failed");
  }
  // the tuning table's choice for this size class, where the options leave
  // the seeds or the small classes' bins open
  lms_tuning tuned;
  bool have_tuned = false;
  if (!(opt && opt->seed_pairs >= 0 && opt->bins_log2 != 0)) {
    long long mx = 0;
    for (int64_t b = 0; b < B; ++b) mx = std::max<long long>(mx, off[b + 1] - off[b]);
    have_tuned = mx <= kBatchMaxN &&
                 lms_host::get_tuning(kPathBatched, lms_host::size_class((int)std::max(2ll, mx)),
                                      &tuned);
  }
  int seed_pairs = kBatchSeeds;
  if (opt && opt->seed_pairs >= 0)
    seed_pairs = std::min(opt->seed_pairs, 1 << 16);
  else if (have_tuned && tuned.seed_pairs >= 0)
    seed_pairs = tuned.seed_pairs;
  const int S = 1 + seed_pairs;
  // slope-bin first screen unless bins_log2 = -1; 11 or 12 set the bins of
  // the per-wavefront screen of problems up to 1024 points (default 12)
  const bool bins = !(opt && opt->bins_log2 == -1);
  int small_log2 = kSmallBinsLog2;
  if (opt && opt->bins_log2 > 0) {
    if (opt->bins_log2 != 11 && opt->bins_log2 != 12)
      return fail(LMS_ERR_ARG, "lms_solve_batched: bins_log2 must be 0, -1, 11 or 12");
    small_log2 = opt->bins_log2;
  } else if (!(opt && opt->bins_log2 == -1) && have_tuned &&
             (tuned.bins_log2 == 11 || tuned.bins_log2 == 12)) {
    small_log2 = tuned.bins_log2;
  }
  const BatchKey key{d_xy, d_offsets, d_h, d_out, stream, (int)B, S, bins, max_ws, small_log2};
  std::lock_guard<std::mutex> lk(g_bmu);
  BatchCache& bc = g_batches[key];
  const bool same = bc.plan.B == (int)B && bc.offsets == off;
  if (!same) {
    // work queued with the old plan may still use its buffer
    if (bc.base && hipStreamSynchronize(s) != hipSuccess)
      return fail(LMS_ERR_DEVICE, "hipStreamSynchronize failed");
    bc.release();
    BPlan P;
    lms_status st = plan_batch(off.data(), (int)B, S, max_ws, &P);
    P.small_log2 = small_log2;
    if (st != LMS_OK) { g_batches.erase(key); return st; }
    char* base = nullptr;
    if (hipMalloc(&base, P.total) != hipSuccess) {
      (void)hipGetLastError();
      g_batches.erase(key);
      return fail(LMS_ERR_NOMEM, "hipMalloc of the batch buffer failed");
    }
    // plan arrays: staged once, synchronously, outside any graph
    if (hipMemcpy(base + P.o_pad, P.h_pad.data(), P.h_pad.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + P.o_chunks, P.h_chunks.data(), P.h_chunks.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        (!P.h_items.empty() && hipMemcpy(base + P.o_items, P.h_items.data(), P.h_items.size() * sizeof(unsigned), hipMemcpyHostToDevice) != hipSuccess)) {
      (void)hipFree(base);
      g_batches.erase(key);
      return fail(LMS_ERR_DEVICE, "uploading the batch plan failed");
    }
    bc.offsets = off;
    bc.plan = std::move(P);
    bc.base = base;
  }
  if (flags & LMS_F_GRAPH) {
    if (!bc.exec) {
      // Capture on a private stream (the legacy null stream cannot be
      // captured); the graph is then launched on the caller's stream.
      hipStream_t cs = nullptr;
      if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        return fail(LMS_ERR_DEVICE, "hipStreamCreate failed");
      if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return fail(LMS_ERR_DEVICE, "hipStreamBeginCapture failed");
      }
      const lms_status st =
          enqueue_batch(bc.plan, bc.base, d_xy, d_offsets, d_h, d_out, cs, nullptr, bins);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(cs, &g);
      (void)hipStreamDestroy(cs);
      if (st != LMS_OK) { if (g) (void)hipGraphDestroy(g); return st; }
      if (e != hipSuccess || !g) return fail(LMS_ERR_DEVICE, "hipStreamEndCapture failed");
      if (hipGraphInstantiate(&bc.exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(LMS_ERR_DEVICE, "hipGraphInstantiate failed");
      }
      bc.graph = g;
    }
    lms_host::StageEvents prof;
    prof.start(s);
    if (hipGraphLaunch(bc.exec, s) != hipSuccess) return fail(LMS_ERR_DEVICE, "hipGraphLaunch failed");
    for (int k = 0; k < LMS_NSTAGES; ++k) prof.mark();  // the whole graph is stage 0
    prof.finish();
    return bc.plan.may_overflow ? resolve_overflowed(bc, d_xy, off, d_h, d_out, opt, s) : LMS_OK;
  }
  lms_host::StageEvents prof;
  prof.start(s);
  const lms_status st = enqueue_batch(bc.plan, bc.base, d_xy, d_offsets, d_h, d_out, s, &prof, bins);
  prof.finish();
  if (st != LMS_OK || !bc.plan.may_overflow) return st;
  return resolve_overflowed(bc, d_xy, off, d_h, d_out, opt, s);
}

lms_status lms_autotune_batched(const double* d_xy, const int64_t* d_offsets,
                                const int64_t* h_offsets, int64_t B, const int32_t* d_h,
                                lms_result* d_out, int32_t reps, void* stream, lms_tuning* out) {
  lms_host::clear_error();
  if (!h_offsets || B < 1 || reps < 1 || reps > 100) return fail(LMS_ERR_ARG, "bad arguments");
  long long mx = 0;
  for (int64_t b = 0; b < B; ++b) mx = std::max<long long>(mx, h_offsets[b + 1] - h_offsets[b]);
  if (mx > kBatchMaxN) return fail(LMS_ERR_ARG, "problems hold at most 4096 points");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  // Candidates: the random seed pairs per problem and the bins of the small
  // classes' per-wavefront screen. A candidate counts only if every problem
  // gets the default settings' status and width, bit for bit (integer data
  // may tie between lines of equal width).
  static const int kSeeds[] = {15, 31, 63};
  static const int kSmall[] = {12, 11};
  const size_t bytes = (size_t)B * sizeof(lms_result);
  std::vector<lms_result> ref((size_t)B), cur((size_t)B);
  auto run = [&](int sp, int sl) {
    lms_options o;
    std::memset(&o, 0, sizeof(o));
    o.struct_size = sizeof(o);
    o.seed_pairs = sp;
    o.bins_log2 = sl;
    return lms_solve_batched(d_xy, d_offsets, h_offsets, B, d_h, d_out, &o, stream);
  };
  auto fetch = [&](std::vector<lms_result>& v) {
    if (hipMemcpyAsync(v.data(), d_out, bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(LMS_ERR_DEVICE, "reading the batch results failed");
    return LMS_OK;
  };
  lms_tuning best{0, 0, kBatchSeeds, 0, 1e30, 0, 0};
  lms_status st = run(kBatchSeeds, kSmallBinsLog2);
  if (st == LMS_OK) st = fetch(ref);
  for (int sp : kSeeds) {
    for (int sl : kSmall) {
      if (st != LMS_OK) break;
      if (sl != kSmallBinsLog2 && mx > 1024) continue;  // no small-class problem
      st = run(sp, sl);
      if (st == LMS_OK) st = fetch(cur);
      if (st != LMS_OK) break;
      bool same = true;
      for (int64_t b = 0; b < B && same; ++b)
        same = cur[b].status == ref[b].status &&
               std::memcmp(&cur[b].width, &ref[b].width, sizeof(double)) == 0;
      if (!same) continue;
      std::vector<float> t(reps);
      for (int k = 0; k < reps && st == LMS_OK; ++k) {
        (void)hipEventRecord(e0, s);
        st = run(sp, sl);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) st = fail(LMS_ERR_DEVICE, "event failed");
        (void)hipEventElapsedTime(&t[k], e0, e1);
      }
      if (st != LMS_OK) break;
      std::sort(t.begin(), t.end());
      if (t[reps / 2] < best.ms) best = {0, 0, sp, sl, t[reps / 2], 0, 0};
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != LMS_OK) return st;
  lms_host::set_tuning(kPathBatched, lms_host::size_class((int)std::max(2ll, mx)), best);
  if (out) *out = best;
  return LMS_OK;
}

}  // extern "C"

namespace lms_host {

void release_batches() {
  std::lock_guard<std::mutex> lk(g_bmu);
  for (auto& kv : g_batches) kv.second.release();
  g_batches.clear();
}

}  // namespace lms_host
