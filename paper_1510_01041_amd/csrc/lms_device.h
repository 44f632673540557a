// Device-side building blocks shared by the single-problem and batched LMS
// kernels (gfx950). See lms.hip for the method and the pipeline.
#ifndef LMS_DEVICE_H
#define LMS_DEVICE_H
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

namespace lms_dev {

constexpr unsigned kDegenerate = 0xFFFFFFFFu;  // entry code: slope 0, all x equal

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Smallest float >= v (v finite and >= 0 here; +inf stays +inf).
__device__ __forceinline__ float f32_up(double v) {
  float f = (float)v;
  if ((double)f < v) f = nextafterf(f, INFINITY);
  return f;
}

__device__ __forceinline__ float lane_f(float v, int c) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), c));
}
__device__ __forceinline__ int lane_i(int v, int c) { return __builtin_amdgcn_readlane(v, c); }

// Upper bound on the exact width at slope theta given its FP64 width w:
// every z carries at most one rounding of |z| <= yabs + |theta| xabs.
__device__ __forceinline__ double width_bound(double w, double theta, double xabs,
                                              double yabs) {
  const double zmax = yabs + fabs(theta) * xabs;
  return (w + 4.0 * 0x1p-53 * zmax) * (1.0 + 0x1p-50);
}

// Bound on |d_fp32 - d_exact| for every anchored residual at slope theta
// (centred FP32 coordinates, FP32 slope, one FMA; see the derivation above
// the screen kernel).
__device__ __forceinline__ double tau_bound(double theta, double xh, double yh) {
  return 0x1p-24 * (6.25 * yh + 8.25 * fabs(theta) * xh);
}

// Order-preserving map of a non-NaN double to u64 (for atomicMin keys).
__device__ __forceinline__ unsigned long long order_key(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// ---------------------------------------------------------------- FP64 window

// Narrowest window of h consecutive values of z_k = fma(-theta, x_k, y_k),
// k < n, computed by the whole block; z is an LDS array of N2 >= n doubles.
// Same operation sequence as the reference: fma, full sort, subtraction, and
// the lowest window among equally narrow ones.
template <int NMAX, int NT>
__device__ void window_f64_rt(const double* __restrict__ xy, int n, int h, int n2, double theta,
                              double* z, unsigned long long* s_w, int* s_s, double* width,
                              double* z_lo, double* z_hi) {
  const int t = threadIdx.x;
  for (int k = t; k < n2; k += NT)
    z[k] = (k < n) ? fma(-theta, xy[2 * k], xy[2 * k + 1]) : INFINITY;
  if (t == 0) { *s_w = ~0ull; *s_s = INT_MAX; }
  __syncthreads();
  for (int k = 2; k <= n2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int q = t; q < n2 / 2; q += NT) {
        const int a = 2 * q - (q & (j - 1));
        const int b = a + j;
        const double va = z[a], vb = z[b];
        const bool up = (a & k) == 0;
        if ((va > vb) == up) { z[a] = vb; z[b] = va; }
      }
      __syncthreads();
    }
  }
  double bw = INFINITY;
  int bs = INT_MAX;
  for (int s = t; s + h <= n; s += NT) {
    const double w = z[s + h - 1] - z[s];
    if (w < bw) { bw = w; bs = s; }
  }
  const unsigned long long bwb = (unsigned long long)__double_as_longlong(bw);
  atomicMin(s_w, bwb);
  __syncthreads();
  if (bs != INT_MAX && bwb == *s_w) atomicMin(s_s, bs);
  __syncthreads();
  // No window compares below +inf only if the slope or the data overflow to
  // NaN; report NaN and read window 0, which always exists.
  const int s = (*s_s == INT_MAX) ? 0 : *s_s;
  *width = (*s_s == INT_MAX) ? NAN : __longlong_as_double((long long)*s_w);
  *z_lo = z[s];
  *z_hi = z[s + h - 1];
  __syncthreads();
}

// Narrowest window and its ends from z[0..N2), sorted, by the whole block
// (the scan of window_f64_rt).
template <int NT>
__device__ __forceinline__ void window_scan(const double* z, int n, int h, unsigned long long* s_w,
                                            int* s_s, double* width, double* z_lo,
                                            double* z_hi) {
  const int t = threadIdx.x;
  double bw = INFINITY;
  int bs = INT_MAX;
  for (int s = t; s + h <= n; s += NT) {
    const double w = z[s + h - 1] - z[s];
    if (w < bw) { bw = w; bs = s; }
  }
  const unsigned long long bwb = (unsigned long long)__double_as_longlong(bw);
  atomicMin(s_w, bwb);
  __syncthreads();
  if (bs != INT_MAX && bwb == *s_w) atomicMin(s_s, bs);
  __syncthreads();
  const int s = (*s_s == INT_MAX) ? 0 : *s_s;
  *width = (*s_s == INT_MAX) ? NAN : __longlong_as_double((long long)*s_w);
  *z_lo = z[s];
  *z_hi = z[s + h - 1];
  __syncthreads();
}

// Narrowest window of h consecutive values of z_k = fma(-theta, x_k, y_k),
// k < n, computed by the whole block; z is an LDS array of N2 >= n doubles.
// Same operation sequence as the reference: fma, full sort, subtraction, and
// the lowest window among equally narrow ones.
//
// With N2 >= NT the sort runs in registers: value g = (wave * E + r) * 64 +
// lane (E = N2 / NT) sits in register r of that lane. A bitonic stage with
// partner distance j < 64 exchanges across lanes (wavefront shuffles), one
// with 64 <= j < 64 E within a thread, and one with j >= 64 E through LDS
// (two barriers). It is the same network with the same compare-and-swap rule
// as window_f64_rt's LDS sort, so the sorted sequence is identical (also for
// NaN and signed zeros).
template <int N2, int NT>
__device__ __forceinline__ void window_f64(const double* __restrict__ xy, int n, int h,
                                           double theta, double* z, unsigned long long* s_w,
                                           int* s_s, double* width, double* z_lo, double* z_hi) {
  if constexpr (N2 < NT) {
    window_f64_rt<N2, NT>(xy, n, h, N2, theta, z, s_w, s_s, width, z_lo, z_hi);
  } else {
    constexpr int E = N2 / NT;
    static_assert(N2 % NT == 0 && NT % 64 == 0, "block must tile the sort");
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int g = (wave * E + r) * 64 + lane;
      v[r] = g < n ? fma(-theta, xy[2 * g], xy[2 * g + 1]) : INFINITY;
    }
    if (t == 0) { *s_w = ~0ull; *s_s = INT_MAX; }
#pragma unroll
    for (int k = 2; k <= N2; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        if (j < 64) {
#pragma unroll
          for (int r = 0; r < E; ++r) {
            const int g = (wave * E + r) * 64 + lane;
            const double p = __shfl_xor(v[r], j);
            const bool up = (g & k) == 0;
            // pair (a, b) = (lower, upper) index; swap iff (a > b) == up
            const bool sw = (g & j) == 0 ? ((v[r] > p) == up) : ((p > v[r]) == up);
            v[r] = sw ? p : v[r];
          }
        } else if (j < 64 * E) {
          const int d = j / 64;
#pragma unroll
          for (int r = 0; r < E; ++r) {
            if ((r & d) == 0) {
              const int g = (wave * E + r) * 64 + lane;
              const bool up = (g & k) == 0;
              const double a = v[r], b = v[r | d];
              const bool sw = (a > b) == up;
              v[r] = sw ? b : a;
              v[r | d] = sw ? a : b;
            }
          }
        } else {
#pragma unroll
          for (int r = 0; r < E; ++r) z[(wave * E + r) * 64 + lane] = v[r];
          __syncthreads();
#pragma unroll
          for (int r = 0; r < E; ++r) {
            const int g = (wave * E + r) * 64 + lane;
            const double p = z[g ^ j];
            const bool up = (g & k) == 0;
            const bool sw = (g & j) == 0 ? ((v[r] > p) == up) : ((p > v[r]) == up);
            v[r] = sw ? p : v[r];
          }
          __syncthreads();
        }
      }
    }
#pragma unroll
    for (int r = 0; r < E; ++r) z[(wave * E + r) * 64 + lane] = v[r];
    __syncthreads();
    window_scan<NT>(z, n, h, s_w, s_s, width, z_lo, z_hi);
  }
}

// ---------------------------------------------------------------- slope bins
//
// Anchor i, point k, Dx = x_k - x_i, Dy = y_k - y_i (exact reals). The anchored
// residual d_k(theta) = Dy - theta Dx lies in the upper window [0, W] for theta
// in one closed interval and in the lower window [-W, 0] for theta in the
// adjacent one; both end at the slope of (i, k). Counted over k at a partner's
// slope, they give the pair's window counts U and D. Bins are uniform in
// u = theta / (1 + |theta|); a bin holds U in its low and D in its high 16
// bits, so one u32 difference array and one prefix sum serve both.

// Bin of slope t: bins are uniform in u = t' / (1 + |t'|), t' = (t - tc) * sc.
// The centre tc is the slope of the narrowest seed window and sc a magnified
// x/y aspect ratio: every pair that can pass has a slope near the optimum, so
// the map spends its resolution there (any monotone map is sound). The map is
// evaluated in FP32 with the hardware reciprocal: its error, below 4e-7 in u,
// is far below one bin (2 / NB >= 6e-5), so the computed bin is within one of
// the exact map's bin. t is finite or +-inf here.
template <int NB>
__device__ __forceinline__ int ubin(double t, double tc, float sc) {
  float f = (float)(t - tc) * sc;
  f = fminf(fmaxf(f, -1e30f), 1e30f);
  const float u = f * __builtin_amdgcn_rcpf(1.0f + fabsf(f));
  const int b = (int)floorf(fmaf(u, 0.5f * NB, 0.5f * NB));
  return b < 0 ? 0 : (b > NB - 1 ? NB - 1 : b);
}

// Prefix sums use one padding word per S = NB / NT bins so that each thread's
// S consecutive bins sit in distinct banks across a wavefront.
template <int NB, int NT>
__device__ __forceinline__ int bin_addr(int b) {
  return b + b / (NB / NT);
}

// Adds point (dx, dy)'s two window intervals to the difference array. Ends
// e = (Dy + c) / Dx, c in {-W, 0, W}, are formed as (Dy + c) * (1 / Dx): one
// rounding each of Dx, Dy, the sum, the reciprocal and the product give
// |e - e_exact| <= d = 2^-50 (2 |Dy| + W) / |Dx|. The bin coordinate moves by
// at most (NB / 2) sc per unit of slope, so d shifts it by at most a quarter
// bin whenever |Dx| >= 2^-47 (2 |Dy| + W) NB sc; the check uses 2^-46. Then
// the end's rounding, the FP32 bin map (at the ends and at the partner's
// slope) and the partner slope's rounding together move bin coordinates by
// less than one bin, so the two-bin margin keeps every exact slope of the
// interval inside the bins it adds to. A point failing the check, or with
// Dx = 0 and in a window, is counted in that window at every slope
// (returned packed: 1 = upper window, 65536 = lower window), which can only
// raise the bounds. nbsc = 2^-46 NB sc.
template <int NB, int NT>
__device__ __forceinline__ unsigned add_point_bins(unsigned* bins, double dx, double dy, double W,
                                                   double lim, double tc, float sc, double nbsc) {
  const double adx = fabs(dx), ady = fabs(dy);
  if (dx == 0.0)
    return (dy >= 0.0 && dy <= lim ? 1u : 0u) + (dy <= 0.0 && dy >= -lim ? 65536u : 0u);
  if (!(adx >= (2.0 * ady + W) * nbsc)) return 1u + 65536u;  // also W = inf
  const double inv = 1.0 / dx;
  const int b0 = ubin<NB>((dy - W) * inv, tc, sc);
  const int b1 = ubin<NB>(dy * inv, tc, sc);
  const int b2 = ubin<NB>((dy + W) * inv, tc, sc);
  // dx > 0: upper window on [e0, e1], lower on [e1, e2]; dx < 0: reversed
  const int ul = (dx > 0.0 ? b0 : b1) - 2, uh = (dx > 0.0 ? b1 : b0) + 2;
  const int dl = (dx > 0.0 ? b1 : b2) - 2, dh = (dx > 0.0 ? b2 : b1) + 2;
  atomicAdd(&bins[bin_addr<NB, NT>(ul < 0 ? 0 : ul)], 1u);
  if (uh + 1 < NB) atomicAdd(&bins[bin_addr<NB, NT>(uh + 1)], 0xFFFFFFFFu);
  atomicAdd(&bins[bin_addr<NB, NT>(dl < 0 ? 0 : dl)], 65536u);
  if (dh + 1 < NB) atomicAdd(&bins[bin_addr<NB, NT>(dh + 1)], 0xFFFF0000u);
  return 0u;
}

// Scale of the bin map: the x/y aspect ratio times kBinMag, in FP32, kept
// finite and positive. With the map centred on a slope within a few degrees
// of the optimum, a magnification of 16 leaves of the order of 1e-5 of the
// pairs of a 4096-point set above the bound, against 5e-3 unmagnified.
constexpr double kBinMag = 16.0;
__device__ __forceinline__ float bin_scale(double xh, double yh) {
  const double r = yh > 0.0 ? kBinMag * xh / yh : 1.0;
  return (float)fmin(fmax(r, 1e-30), 1e30);
}

// Slope of the narrowest of the candidate windows (width, theta, z_lo, z_hi)
// in a[0..ma) and b[0..mb), by the NT threads of the block (ties by the low
// bits of the width, then the index); 0 if none is finite. Ends with a
// barrier.
template <int NT>
__device__ __forceinline__ double best_slope(const double4* __restrict__ a, int ma,
                                             const double4* __restrict__ b, int mb,
                                             unsigned long long* s_key, double* s_th) {
  const int t = threadIdx.x;
  if (t == 0) *s_key = ~0ull;
  __syncthreads();
  unsigned long long key = ~0ull;
  for (int e = t; e < ma + mb; e += NT) {
    const double w = e < ma ? a[e].x : b[e - ma].x;
    if (w < INFINITY) {  // finite (NaN compares false)
      const unsigned long long k = ((unsigned long long)__double_as_longlong(w) & ~0xFFFFFull) |
                                   (unsigned long long)(e & 0xFFFFF);
      key = k < key ? k : key;
    }
  }
  atomicMin(s_key, key);
  __syncthreads();
  if (t == 0) {
    const int e = (int)(*s_key & 0xFFFFF);
    *s_th = *s_key == ~0ull ? 0.0 : (e < ma ? a[e].y : b[e - ma].y);
  }
  __syncthreads();
  return *s_th;
}

// In-place prefix sum of the NB-bin difference array by the NT threads of the
// block (all must call; ends with the sums in LDS, before a barrier). Modular
// u32 arithmetic is exact: every true sum U + 65536 D is below 2^31.
template <int NB, int NT>
__device__ __forceinline__ void scan_bins(unsigned* bins, unsigned* part) {
  constexpr int S = NB / NT;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  unsigned v[S];
  unsigned run = 0;
#pragma unroll
  for (int r = 0; r < S; ++r) {
    run += bins[t * (S + 1) + r];
    v[r] = run;
  }
  unsigned x = run;  // inclusive scan of the thread totals within the wavefront
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    const unsigned y = __shfl_up(x, m);
    if (lane >= m) x += y;
  }
  if (NT > 64) {
    if (lane == 63) part[wave] = x;
    __syncthreads();
  }
  unsigned off = x - run;
  for (int w = 0; w < wave; ++w) off += part[w];
#pragma unroll
  for (int r = 0; r < S; ++r) bins[t * (S + 1) + r] = v[r] + off;
}

// A pair passes when its bin bounds U or D (plus the every-slope points) at h.
__device__ __forceinline__ bool bins_pass(unsigned pb, unsigned pall, int h) {
  return (int)((pb & 0xFFFFu) + (pall & 0xFFFFu)) >= h || (int)((pb >> 16) + (pall >> 16)) >= h;
}

// ---------------------------------------------------------------- FP32 screen

// Error bound tau. With u = 2^-24, centred coordinates a_k = x_k - cx (exact),
// |x32_k - a_k| <= u|a_k| (1 + 2^-29) and the same for y. For a pair (i, j)
// at exact slope theta the anchored residual is d_k = (y_k - y_i) -
// theta (x_k - x_i). The kernel evaluates either
//   (registers) d = fl(fma(-theta32, fl(x32_k - x32_i), fl(y32_k - y32_i))), or
//   (LDS)       d = fl(fl(fma(-theta32, x32_k, y32_k)) - fl(fma(-theta32, x32_i, y32_i))),
// with |theta32 - theta| <= u|theta| (1 + 2^-28). Summing the input, shift,
// slope and FMA roundings gives, for both forms and to first order,
//   |d - d_k| <= u (6 Yh + 8 |theta| Xh),
// where Xh, Yh bound |x - cx| and |y - cy|. tau_bound adds a 4 % margin for the
// higher-order terms. If the exact anchored window [0, W] (or [-W, 0]) holds h
// points, their FP32 residuals lie in [-tau, W + tau] (or [-W - tau, tau]).

// Screen test of one pair (uniform across the wavefront).
//  Band test: B = #{|d| <= thr}, thr = W + tau. A pair whose anchored window
//  of width <= W holds h points has B >= h; misses beyond 64*chunks - h reject
//  it at once.
//  Split test: with N = #{-thr <= d < -ta} and P = #{ta < d <= thr}, the
//  one-sided counts are up = B - N and dn = B - P, so the pair survives iff
//  N <= B - h or P <= B - h. Both counts only grow, so the pair is rejected as
//  soon as both exceed B - h, usually within a few chunks.
// Outcome of one pair's test: keep flag and the 64-point chunks evaluated by
// the band and split passes (-1 split chunks: the band test rejected).
struct PairTest {
  int keep, band_chunks, split_chunks;
};

template <int R, bool LDS_PART>
__device__ __forceinline__ PairTest test_pair(const float (&X)[R], const float (&Y)[R],
                                              const float2* __restrict__ lds, int nq, float nth,
                                              float thr, float ta, float nc, int h) {
  const int lane = threadIdx.x & 63;
  const int total = R + (LDS_PART ? nq : 0);  // chunks of 64 points (padding never hits)
  // misses allowed before the pair is certainly rejected
  const int budget = 64 * total - h;
  int miss = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float d = fmaf(nth, X[r], Y[r]);
    miss += __popcll(__ballot(!(fabsf(d) <= thr)));
    if ((r & 7) == 7 || r == R - 1) {
      if (miss > budget) return {0, r + 1, -1};
    }
  }
  if (LDS_PART) {
    for (int q = 0; q < nq; ++q) {
      const float2 p = lds[q * 64 + lane];
      const float d = fmaf(nth, p.x, p.y) + nc;
      miss += __popcll(__ballot(!(fabsf(d) <= thr)));
      if (((q & 7) == 7 || q == nq - 1) && miss > budget) return {0, R + q + 1, -1};
    }
  }
  const int slack = budget - miss;  // B - h >= 0
  // The slope goes through an opaque copy so that the compiler recomputes the
  // residuals instead of keeping all R of them live from the band test.
  asm volatile("" : "+v"(nth));
  int below = 0, above = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float d = fmaf(nth, X[r], Y[r]);
    above += __popcll(__ballot(d > ta && d <= thr));
    below += __popcll(__ballot(d < -ta && d >= -thr));
    if (above > slack && below > slack) return {0, total, r + 1};
  }
  if (LDS_PART) {
    for (int q = 0; q < nq; ++q) {
      const float2 p = lds[q * 64 + lane];
      const float d = fmaf(nth, p.x, p.y) + nc;
      above += __popcll(__ballot(d > ta && d <= thr));
      below += __popcll(__ballot(d < -ta && d >= -thr));
      if (above > slack && below > slack) return {0, total, R + q + 1};
    }
  }
  return {1, total, total};
}

// Rest of one pair's test after its band count over chunks [0, start) came
// to `miss` (start a multiple of 8 within the register chunks, or a chunk
// index past them): the remaining band chunks, then the split test. Same
// checkpoints and outcome as test_pair<R, LDS_PART>.
template <int R, bool LDS_PART>
__device__ __forceinline__ PairTest finish_pair(const float (&X)[R], const float (&Y)[R],
                                                const float2* __restrict__ lds, int nq,
                                                float nth, float thr, float ta, float nc,
                                                int start, int miss, int h) {
  const int lane = threadIdx.x & 63;
  const int total = R + (LDS_PART ? nq : 0);
  const int budget = 64 * total - h;
#pragma unroll
  for (int b = 0; b < R; b += 8) {
    if (b >= start) {
#pragma unroll
      for (int r = b; r < b + 8 && r < R; ++r) {
        const float d = fmaf(nth, X[r], Y[r]);
        miss += __popcll(__ballot(!(fabsf(d) <= thr)));
      }
      if (miss > budget) return {0, b + 8 < R ? b + 8 : R, -1};
    }
  }
  if (LDS_PART) {
    for (int q = start > R ? start - R : 0; q < nq; ++q) {
      const float2 p = lds[q * 64 + lane];
      const float d = fmaf(nth, p.x, p.y) + nc;
      miss += __popcll(__ballot(!(fabsf(d) <= thr)));
      if (((q & 7) == 7 || q == nq - 1) && miss > budget) return {0, R + q + 1, -1};
    }
  }
  const int slack = budget - miss;
  asm volatile("" : "+v"(nth));
  int below = 0, above = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const float d = fmaf(nth, X[r], Y[r]);
    above += __popcll(__ballot(d > ta && d <= thr));
    below += __popcll(__ballot(d < -ta && d >= -thr));
    if (above > slack && below > slack) return {0, total, r + 1};
  }
  if (LDS_PART) {
    for (int q = 0; q < nq; ++q) {
      const float2 p = lds[q * 64 + lane];
      const float d = fmaf(nth, p.x, p.y) + nc;
      above += __popcll(__ballot(d > ta && d <= thr));
      below += __popcll(__ballot(d < -ta && d >= -thr));
      if (above > slack && below > slack) return {0, total, R + q + 1};
    }
  }
  return {1, total, total};
}

// Two pairs tested together. Their band counts run in lockstep over the same
// points (registers, then LDS), so each chunk issues two independent
// compare-and-count chains and each LDS read serves both; at the first
// checkpoint where either pair is rejected, each pair still open finishes
// alone. The outcomes equal two calls of test_pair<R, LDS_PART>.
struct PairTest2 {
  PairTest a, b;
};

template <int R, bool LDS_PART>
__device__ __forceinline__ PairTest2 test_pair2(const float (&X)[R], const float (&Y)[R],
                                                const float2* __restrict__ lds, int nq,
                                                float nth_a, float thr_a, float ta_a, float nc_a,
                                                float nth_b, float thr_b, float ta_b, float nc_b,
                                                int h) {
  const int lane = threadIdx.x & 63;
  const int total = R + (LDS_PART ? nq : 0);
  const int budget = 64 * total - h;
  int ma = 0, mb = 0, e = total;
  bool open = true;
#pragma unroll
  for (int b = 0; b < R; b += 8) {
#pragma unroll
    for (int r = b; r < b + 8 && r < R; ++r) {
      const float da = fmaf(nth_a, X[r], Y[r]);
      const float db = fmaf(nth_b, X[r], Y[r]);
      ma += __popcll(__ballot(!(fabsf(da) <= thr_a)));
      mb += __popcll(__ballot(!(fabsf(db) <= thr_b)));
    }
    if (ma > budget || mb > budget) {
      e = b + 8 < R ? b + 8 : R;
      open = false;
      break;
    }
  }
  if (LDS_PART && open) {
    for (int q = 0; q < nq; ++q) {
      const float2 p = lds[q * 64 + lane];
      const float da = fmaf(nth_a, p.x, p.y) + nc_a;
      const float db = fmaf(nth_b, p.x, p.y) + nc_b;
      ma += __popcll(__ballot(!(fabsf(da) <= thr_a)));
      mb += __popcll(__ballot(!(fabsf(db) <= thr_b)));
      if (((q & 7) == 7 || q == nq - 1) && (ma > budget || mb > budget)) {
        e = R + q + 1;
        break;
      }
    }
  }
  PairTest2 out;
  out.a = {0, e, -1};
  out.b = {0, e, -1};
  // One copy of the single-pair code serves both (k = 0: pair a, 1: pair b).
#pragma nounroll
  for (int k = 0; k < 2; ++k) {
    const int miss = k ? mb : ma;
    if (miss > budget) continue;
    const PairTest t = finish_pair<R, LDS_PART>(X, Y, lds, nq, k ? nth_b : nth_a,
                                                k ? thr_b : thr_a, k ? ta_b : ta_a,
                                                k ? nc_b : nc_a, e, miss, h);
    if (k) out.b = t;
    else out.a = t;
  }
  return out;
}

// test_pair for points held in registers only, with the number of 64-point
// chunks Rb <= RMAX known at run time (batched problems of different sizes).
template <int RMAX>
__device__ __forceinline__ PairTest test_pair_rt(const float (&X)[RMAX], const float (&Y)[RMAX],
                                                 int Rb, float nth, float thr, float ta, int h) {
  const int budget = 64 * Rb - h;
  int miss = 0;
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    if (r < Rb) {
      const float d = fmaf(nth, X[r], Y[r]);
      miss += __popcll(__ballot(!(fabsf(d) <= thr)));
      if (((r & 7) == 7 || r == Rb - 1) && miss > budget) return {0, r + 1, -1};
    }
  }
  const int slack = budget - miss;
  asm volatile("" : "+v"(nth));
  int below = 0, above = 0;
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    if (r < Rb) {
      const float d = fmaf(nth, X[r], Y[r]);
      above += __popcll(__ballot(d > ta && d <= thr));
      below += __popcll(__ballot(d < -ta && d >= -thr));
      if (above > slack && below > slack) return {0, Rb, r + 1};
    }
  }
  return {1, Rb, Rb};
}

// ---------------------------------------------------------------- canonical order

struct Best {
  double w, th, lo, hi;
  unsigned a, b;
};

__device__ __forceinline__ bool better(const Best& p, const Best& q) {
  if (p.w != q.w) return p.w < q.w;
  if (p.th != q.th) return p.th < q.th;
  if (p.lo != q.lo) return p.lo < q.lo;
  if (p.a != q.a) return p.a < q.a;
  return p.b < q.b;
}

}  // namespace lms_dev

#endif
