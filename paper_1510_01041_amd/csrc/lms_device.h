// Device-side building blocks shared by the single-problem and batched LMS
// kernels (gfx950). See lms.hip for the method and the pipeline.
#ifndef LMS_DEVICE_H
#define LMS_DEVICE_H
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <type_traits>

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

// Scale of one coordinate's FP32 copy: 2^-e, e the exponent of h (the
// centred half-range), so that the scaled centred values lie in (-2, 2) and
// fit FP32 whatever the input's magnitude (2^+-200 coordinates overflow or
// underflow FP32 otherwise); 1 for h = 0. Powers of two scale exactly.
__device__ __forceinline__ double f32_scale(double h) {
  if (!(h > 0.0) || !(h < INFINITY)) return 1.0;
  int e = ilogb(h);
  e = e < -1000 ? -1000 : (e > 1000 ? 1000 : e);
  return ldexp(1.0, -e);
}

// The FP32 test's scalars for a pair of FP64 slope th under the width bound
// W, in the frame of the FP32 copy (x scaled by fx, y by fy, both powers of
// two): there the slope is th fy / fx, the bound W fy, and tau is taken on the
// scaled half-ranges, so every residual and threshold is the input frame's
// times fy exactly. force: the pair skips the FP32 test (its slope or bound is
// too large for it) and goes to the FP64 recheck.
struct ScreenScalars {
  float th32, thr, ta;
  bool force;
};
__device__ __forceinline__ ScreenScalars screen_scalars(double th, double W, double fx, double fy,
                                                        double xh, double yh) {
  const double ths = th * (fy / fx);
  const double tau = tau_bound(ths, xh * fx, yh * fy);
  ScreenScalars r;
  r.force = !(fabs(ths) < 1e30 && tau < 1e30);
  r.th32 = (float)ths;
  r.thr = f32_up(W * fy + tau);
  r.ta = f32_up(tau);
  return r;
}

// The largest |th| (input frame) whose FP32 test bound stays below 1e29;
// steeper pairs go to the FP64 recheck. tau is affine in |th|; half the solved
// limit covers the roundings.
__device__ __forceinline__ double screen_th_lim(double fx, double fy, double xh, double yh) {
  const double xs = xh * fx, ys = yh * fy;
  const double tau0 = tau_bound(0.0, xs, ys), tau1 = tau_bound(1.0, xs, ys) - tau0;
  const double lim = tau0 < 1e29 ? fmin(1e29, 0.5 * (1e29 - tau0) / tau1) : 0.0;
  return lim * (fx / fy);
}

// Lanes of the wavefront (among the active ones) whose predicate holds: the
// compare mask itself, without materialising the predicate as an integer.
__device__ __forceinline__ unsigned long long lane_mask(bool p) {
  return __builtin_amdgcn_ballot_w64(p);
}

// A wavefront-uniform double moved to scalar registers (it must be uniform):
// frees the two vector registers a loop would otherwise hold it in.
__device__ __forceinline__ double uniform(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Point k of n (clamped to n - 1), loaded with no branch around the load, so
// that the loads of an unrolled loop are all in flight together (a load under
// a lane mask is waited for on its own).
__device__ __forceinline__ double2 point_clamped(const double* __restrict__ xy, int k, int n) {
  return reinterpret_cast<const double2*>(xy)[(unsigned)min(k, n - 1)];
}

// Order-preserving map of a non-NaN double to u64 (for atomicMin keys).
__device__ __forceinline__ unsigned long long order_key(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// ---------------------------------------------------------------- FP64 window

// Lexicographic minimum of the (w, s) pairs of the NT threads of the block,
// w compared as doubles (equal widths, signed zeros included, go to the lower
// s); every thread gets it. A thread without a candidate holds (+inf,
// INT_MAX), and NaN never wins. Wavefront shuffles, then one LDS slot per
// wavefront: no contended atomics. Ends with a barrier.
template <int NT>
__device__ __forceinline__ void block_argmin(double& w, int& s) {
  __shared__ double red_w[NT / 64];
  __shared__ int red_s[NT / 64];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const double ow = __shfl_xor(w, m);
    const int os = __shfl_xor(s, m);
    if (ow < w || (ow == w && os < s)) { w = ow; s = os; }
  }
  if (NT > 64) {
    if ((threadIdx.x & 63) == 0) { red_w[threadIdx.x >> 6] = w; red_s[threadIdx.x >> 6] = s; }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) {
      const double ow = red_w[k];
      const int os = red_s[k];
      if (ow < w || (ow == w && os < s)) { w = ow; s = os; }
    }
  }
  __syncthreads();
}

// Block-wide minimum and maximum of the NT threads' values (every thread gets
// both). Ends with a barrier.
template <int NT>
__device__ __forceinline__ void block_min_max(double& mn, double& mx) {
  __shared__ double red_mn[NT / 64], red_mx[NT / 64];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, m));
    mx = fmax(mx, __shfl_xor(mx, m));
  }
  if (NT > 64) {
    if ((threadIdx.x & 63) == 0) { red_mn[threadIdx.x >> 6] = mn; red_mx[threadIdx.x >> 6] = mx; }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) { mn = fmin(mn, red_mn[k]); mx = fmax(mx, red_mx[k]); }
  }
  __syncthreads();
}

// Narrowest window and its ends from the sorted values z[at(0..n)], by the
// whole block (`at` maps a rank to its LDS slot): the smallest z_{s+h-1} - z_s,
// the lowest s among equally narrow windows. No window compares below +inf
// only if the slope or the data overflow to NaN; then the width is NaN and
// window 0, which always exists, is read. Ends with a barrier.
template <int NT, class At>
__device__ __forceinline__ void window_scan_at(const double* z, At at, int n, int h,
                                               double* width, double* z_lo, double* z_hi) {
  double bw = INFINITY;
  int bs = INT_MAX;
  for (int s = threadIdx.x; s + h <= n; s += NT) {
    const double w = z[at(s + h - 1)] - z[at(s)];
    if (w < bw) { bw = w; bs = s; }
  }
  block_argmin<NT>(bw, bs);
  const int s = bs == INT_MAX ? 0 : bs;
  *width = bs == INT_MAX ? NAN : bw;
  *z_lo = z[at(s)];
  *z_hi = z[at(s + h - 1)];
  __syncthreads();
}

template <int NT>
__device__ __forceinline__ void window_scan(const double* z, int n, int h, double* width,
                                            double* z_lo, double* z_hi) {
  window_scan_at<NT>(z, [](int k) { return k; }, n, h, width, z_lo, z_hi);
}

// Narrowest window of h consecutive values of z_k = fma(-theta, x_k, y_k),
// k < n, computed by the whole block; z is an LDS array of N2 >= n doubles.
// Same operation sequence as the reference: fma, full sort, subtraction, and
// the lowest window among equally narrow ones.
template <int NMAX, int NT>
__device__ void window_f64_rt(const double* __restrict__ xy, int n, int h, int n2, double theta,
                              double* z, double* width, double* z_lo, double* z_hi) {
  const int t = threadIdx.x;
  for (int k = t; k < n2; k += NT)
    z[k] = (k < n) ? fma(-theta, xy[2 * k], xy[2 * k + 1]) : INFINITY;
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
  window_scan<NT>(z, n, h, width, z_lo, z_hi);
}

// Lane l's partner value v[l ^ J] for a partner distance J < 64, with every
// lane of the wavefront active. J = 1, 2 are quad permutes; J = 4, 8 compose
// two row permutes (half-row mirror then quad reversal gives l ^ 4, row
// mirror then half-row mirror gives l ^ 8). These move data within the VALU
// (DPP) instead of through the LDS crossbar as a permute does (J = 16, 32).
template <int J>
__device__ __forceinline__ int xor_lanes_i32(int x) {
  constexpr int kQuadXor1 = 0xB1, kQuadXor2 = 0x4E, kQuadReverse = 0x1B;
  constexpr int kRowMirror = 0x140, kRowHalfMirror = 0x141;
  if constexpr (J == 1) return __builtin_amdgcn_update_dpp(0, x, kQuadXor1, 0xF, 0xF, false);
  else if constexpr (J == 2) return __builtin_amdgcn_update_dpp(0, x, kQuadXor2, 0xF, 0xF, false);
  else if constexpr (J == 4)
    return __builtin_amdgcn_update_dpp(
        0, __builtin_amdgcn_update_dpp(0, x, kRowHalfMirror, 0xF, 0xF, false), kQuadReverse, 0xF,
        0xF, false);
  else if constexpr (J == 8)
    return __builtin_amdgcn_update_dpp(
        0, __builtin_amdgcn_update_dpp(0, x, kRowMirror, 0xF, 0xF, false), kRowHalfMirror, 0xF,
        0xF, false);
  else return __shfl_xor(x, J);
}

template <int J>
__device__ __forceinline__ double xor_lanes(double v) {
  if constexpr (J <= 8) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)xor_lanes_i32<J>((int)(unsigned)b);
    const unsigned hi = (unsigned)xor_lanes_i32<J>((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
  } else {
    return __shfl_xor(v, J);
  }
}

// Bitonic sort of N2 values held by the NT threads of the block: value
// g = (wave * E + r) * 64 + lane (E = N2 / NT) sits in v[r] of that lane. A
// stage with partner distance j < 64 exchanges across lanes (wavefront
// shuffles), one with 64 <= j < 64 E within a thread, and one with j >= 64 E
// through z (N2 doubles of LDS, two barriers). It is the same network with the
// same compare-and-swap rule as window_f64_rt's LDS sort, so the sorted
// sequence is identical (also for NaN and signed zeros).
template <int N2, int NT>
__device__ __forceinline__ void sort_regs(double (&v)[N2 / NT], double* z) {
  constexpr int E = N2 / NT;
  static_assert(N2 % NT == 0 && NT % 64 == 0, "block must tile the sort");
  // NT = 64: one wavefront sorts on its own (any wavefront of the block)
  const int t = threadIdx.x, lane = t & 63, wave = NT == 64 ? 0 : t >> 6;
  // a stage with partner distance J < 64: the exchange across lanes
  auto lane_stage = [&](auto jc, int k) {
    constexpr int J = decltype(jc)::value;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int g = (wave * E + r) * 64 + lane;
      const double p = xor_lanes<J>(v[r]);
      const bool up = (g & k) == 0;
      // pair (a, b) = (lower, upper) index; swap iff (a > b) == up
      const bool sw = (g & J) == 0 ? ((v[r] > p) == up) : ((p > v[r]) == up);
      v[r] = sw ? p : v[r];
    }
  };
#pragma unroll
  for (int k = 2; k <= N2; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j < 64) {
        switch (j) {
          case 1: lane_stage(std::integral_constant<int, 1>{}, k); break;
          case 2: lane_stage(std::integral_constant<int, 2>{}, k); break;
          case 4: lane_stage(std::integral_constant<int, 4>{}, k); break;
          case 8: lane_stage(std::integral_constant<int, 8>{}, k); break;
          case 16: lane_stage(std::integral_constant<int, 16>{}, k); break;
          default: lane_stage(std::integral_constant<int, 32>{}, k); break;
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
}

// Narrowest window of h consecutive values of z_k = fma(-theta, x_k, y_k),
// k < n, computed by the whole block; z is an LDS array of N2 >= n doubles.
// Same operation sequence as the reference: fma, full sort, subtraction, and
// the lowest window among equally narrow ones. With N2 >= NT the values are
// sorted in registers (sort_regs).
template <int N2, int NT>
__device__ __forceinline__ void window_f64(const double* __restrict__ xy, int n, int h,
                                           double theta, double* z, double* width, double* z_lo,
                                           double* z_hi) {
  if constexpr (N2 < NT) {
    window_f64_rt<N2, NT>(xy, n, h, N2, theta, z, width, z_lo, z_hi);
  } else {
    constexpr int E = N2 / NT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int g = (wave * E + r) * 64 + lane;
      const double2 p = point_clamped(xy, g, n);
      v[r] = g < n ? fma(-theta, p.x, p.y) : INFINITY;
    }
    sort_regs<N2, NT>(v, z);
#pragma unroll
    for (int r = 0; r < E; ++r) z[(wave * E + r) * 64 + lane] = v[r];
    __syncthreads();
    window_scan<NT>(z, n, h, width, z_lo, z_hi);
  }
}

// LDS slot of rank k in merge_runs' layout: one pad word every 16 values, so
// that the lanes of a wavefront, whose merge positions lie about E / 2 apart,
// fall in different banks.
__device__ __forceinline__ int merge_slot(int k) { return k + (k >> 4); }

// z holds NP values in merge_slot layout (NP + NP / 16 doubles), as sorted runs
// of length L (a power of two dividing NP); merges them pairwise, stably (on
// ties the lower run first), until they are sorted. In each round thread t
// writes the E = NP / NT outputs from rank t E on: a binary search on the
// merge path finds how many of the outputs before it come from the lower run,
// then E merge steps follow. The sorted values equal those of any other sort
// of the same data, up to the order of values that compare equal (signed
// zeros) or unordered (NaN). Each round ends with a barrier.
template <int NP, int NT>
__device__ __forceinline__ void merge_runs(double* z, int L) {
  constexpr int E = NP / NT;
  static_assert(NP % NT == 0, "block must tile the merge");
  const int o = threadIdx.x * E;
  for (; L < NP; L <<= 1) {
    const int a0 = o & ~(2 * L - 1), b0 = a0 + L;  // ranks of the two runs
    const int d = o - a0;  // outputs of this pair of runs before o
    // smallest i whose A[i] comes after B[d - 1 - i]: all reads in [0, L)
    int lo = d > L ? d - L : 0, hi = d < L ? d : L;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (z[merge_slot(a0 + mid)] <= z[merge_slot(b0 + d - 1 - mid)]) lo = mid + 1; else hi = mid;
    }
    int ia = lo, ib = d - lo;
    double out[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const double a = z[merge_slot(a0 + (ia < L ? ia : L - 1))];
      const double b = z[merge_slot(b0 + (ib < L ? ib : L - 1))];
      const bool ta = ib >= L || (ia < L && a <= b);
      out[r] = ta ? a : b;
      ia += ta ? 1 : 0;
      ib += ta ? 0 : 1;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) z[merge_slot(o + r)] = out[r];
    __syncthreads();
  }
}

// ---------------------------------------------------------------- slope bins
//
// Anchor i, point k, Dx = x_k - x_i, Dy = y_k - y_i (exact reals). The anchored
// residual d_k(theta) = Dy - theta Dx lies in the upper window [0, W] for theta
// in one closed interval and in the lower window [-W, 0] for theta in the
// adjacent one; both end at the slope of (i, k). Counted over k at a partner's
// slope, they give the pair's window counts U and D. Bins cover the slopes
// through a compact monotone map (fbin); a bin holds U in its low and D in its
// high 16 bits, so one u32 difference array and one prefix sum serve both.

// Bin of f, a slope's offset from the map's centre in units of 1 / sc. The
// bins are uniform in u(f) = sign(f) (1 - r(|f| + 1)) over [-1, 1], where
// r(g) is the reciprocal of g read off its bit pattern (the high word of the
// FP64 g subtracted, as one saturating integer, from that of 2^1023; adding
// RLOG to the exponent gives R r(g), R = 2^RLOG, in the same step): exact at
// powers of two, within 12.5 % of 1 / g between them, piecewise linear,
// decreasing, and 0 from g = 2^1023 on (also for +inf and NaN). So u is
// monotone with |du/df| <= 1/2 and |f du/df| <= 1 and, like f / (1 + |f|),
// spends half of the bins on |f| < 1, where the optimum's neighbours are. The
// bin coordinate R + 3 + R u spans [3, 2R + 3], so the two-bin margins stay
// inside [0, 2R + 6] with no clamp. Each step is monotone; dropping the low
// word of g (relative 2^-20) and the roundings move the coordinate by less
// than 2^-4 for R <= 2^15.
template <int RLOG>
__device__ __forceinline__ int fbin(double f) {
  constexpr double R = (double)(1 << RLOG), C = R + 3.0;
  const double g = fabs(f) + 1.0;
  const unsigned hi = __builtin_elementwise_sub_sat(
      0x7FE00000u + ((unsigned)RLOG << 20),
      (unsigned)((unsigned long long)__double_as_longlong(g) >> 32));
  const double v = __longlong_as_double((long long)((unsigned long long)hi << 32));  // R r(g)
  return (int)(C + copysign(R - v, f));
}

// Reciprocal of d for 2^-900 <= |d| <= 2^900: the hardware estimate and one
// Newton step, relative error below 2^-40.
__device__ __forceinline__ double recip(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  return fma(r, fma(-d, r, 1.0), r);
}

// The map's frame, uniform over a block: a slope theta has offset
// f = (theta - tc) sc. The centre tc is the slope of the narrowest seed
// window (0 if |tc| sc > 2^20) and sc = kBinMag x-range / y-range, in
// [2^-100, 2^100]: every pair that can pass has a slope near the optimum, so
// the map spends its resolution there (any monotone map is sound). A point
// with |Dx| < q |Dy| + 2^-900, or |Dx| > 2^900, counts in both windows at
// every slope; q is infinite when W is (then every point does).
constexpr double kBinMag = 32.0;
struct BinFrame {
  double tc, sc, q;
};
__device__ __forceinline__ BinFrame bin_frame(double tc, double xh, double yh, double W, int nb) {
  BinFrame F;
  const double r = yh > 0.0 ? kBinMag * xh / yh : 1.0;
  F.sc = fmin(fmax(r, 0x1p-100), 0x1p100);
  F.tc = fabs(tc) * F.sc <= 0x1p20 ? tc : 0.0;
  F.q = W < INFINITY ? 0x1p-46 * nb * F.sc : INFINITY;
  return F;
}

// Bin of the slope of the pair (anchor, partner) at offset (dx, dy), with
// r = recip(dx): f = fma(-tc, dx, dy) (sc r). Identical to the middle bin
// add_point_bins computes for that partner.
template <int RLOG>
__device__ __forceinline__ int slope_bin(double dx, double dy, double r, const BinFrame& F) {
  return fbin<RLOG>(fma(-F.tc, dx, dy) * (F.sc * r));
}

// Adds point (dx, dy)'s two window intervals to the difference array of the
// bins of fbin<RLOG> (2^(RLOG+1) + 7 words at least). In
// offset units the ends are f_c = (a + c) s, c in {-W, 0, W}, with
// a = fma(-tc, Dx, Dy) and s = sc recip(Dx). Against the exact
// (Dy + c - tc Dx) sc / Dx, the roundings of Dx, Dy, a, the sum, s and the
// product leave a relative error below 2^-44 and an absolute one below
// 2^-52 (|Dy / Dx| + |tc|) sc. As |f du/df| <= 1 and |du/df| <= 1/2, they move
// the bin coordinate by less than R 2^-44 + (R / 2) 2^-52 (2^46 / NB + 2^20)
// < 2^-7 when |Dx| >= q |Dy| (NB >= 2R the bins of the frame's q). With the map's own error (below 2^-4), every
// computed bin (ends here, a pair's slope_bin) is within one of the exact
// map's bin, so the two-bin margins keep every exact slope of an interval
// inside the bins it adds to. A point outside the check's range, or with
// Dx = 0 and in a window, is counted in that window at every slope (added to
// `all`, packed: 1 = upper window, 65536 = lower window), which can only
// raise the bounds. Only those rare cases touch `all`.
template <int RLOG>
__device__ __forceinline__ void add_point_bins(unsigned* bins, double dx, double dy, double W,
                                               double lim, const BinFrame& F, unsigned& all) {
  const double adx = fabs(dx), ady = fabs(dy);
  if (dx == 0.0) {
    all += (dy >= 0.0 && dy <= lim ? 1u : 0u) + (dy <= 0.0 && dy >= -lim ? 65536u : 0u);
    return;
  }
  if (!(adx >= fma(ady, F.q, 0x1p-900)) || adx > 0x1p900) {
    all += 1u + 65536u;
    return;
  }
  const double s = F.sc * recip(dx);
  const double a = fma(-F.tc, dx, dy);
  const int b0 = fbin<RLOG>((a - W) * s), b1 = fbin<RLOG>(a * s), b2 = fbin<RLOG>((a + W) * s);
  // dx > 0: upper window on [f_-W, f_0], lower on [f_0, f_W]; dx < 0: reversed
  atomicAdd(&bins[min(b0, b1) - 2], 1u);
  atomicAdd(&bins[max(b0, b1) + 3], 0xFFFFFFFFu);
  atomicAdd(&bins[min(b1, b2) - 2], 65536u);
  atomicAdd(&bins[max(b1, b2) + 3], 0xFFFF0000u);
}

// add_point_bins, and the point's code for the queries of this anchor's
// pairs: kCodeVertical (Dx = 0), kCodeFP64 (|Dx| outside [2^-900, 2^900], or
// a slope of magnitude th_lim or more: the pair goes to the FP64 entries),
// else the bin of the pair's slope (slope_bin, >= 3). The bin is taken for
// far points too: its error is relative (below 2^-44), so it is within one
// of the exact bin whatever the far-point check says.
constexpr unsigned short kCodeVertical = 0, kCodeFP64 = 1, kCodePass = 2;
template <int RLOG>
__device__ __forceinline__ void add_point_bins_coded(unsigned* bins, double dx, double dy,
                                                     double W, double lim, const BinFrame& F,
                                                     double th_lim, unsigned short* code,
                                                     unsigned& all) {
  const double adx = fabs(dx), ady = fabs(dy);
  if (dx == 0.0) {
    *code = kCodeVertical;
    all += (dy >= 0.0 && dy <= lim ? 1u : 0u) + (dy <= 0.0 && dy >= -lim ? 65536u : 0u);
    return;
  }
  if (!(adx >= 0x1p-900) || adx > 0x1p900) {
    *code = kCodeFP64;
    all += 1u + 65536u;
    return;
  }
  const double r = recip(dx);
  const double s = F.sc * r;
  const double a = fma(-F.tc, dx, dy);
  const int b1 = fbin<RLOG>(a * s);
  *code = fabs(dy * r) < th_lim ? (unsigned short)b1 : kCodeFP64;
  if (!(adx >= fma(ady, F.q, 0x1p-900))) {
    all += 1u + 65536u;
    return;
  }
  const int b0 = fbin<RLOG>((a - W) * s), b2 = fbin<RLOG>((a + W) * s);
  atomicAdd(&bins[min(b0, b1) - 2], 1u);
  atomicAdd(&bins[max(b0, b1) + 3], 0xFFFFFFFFu);
  atomicAdd(&bins[min(b1, b2) - 2], 65536u);
  atomicAdd(&bins[max(b1, b2) + 3], 0xFFFF0000u);
}

// Slope of the narrowest of the candidate windows (width, theta, z_lo, z_hi)
// in a[0..ma) and b[0..mb), by z_hi - z_lo (the width of an exact window, the
// bound of a seed's), by the NT threads of the block (ties to the lower
// index); 0 if none is finite. Ends with a barrier.
template <int NT>
__device__ __forceinline__ double best_slope(const double4* __restrict__ a, int ma,
                                             const double4* __restrict__ b, int mb) {
  double bw = INFINITY;
  int be = INT_MAX;
  for (int e = threadIdx.x; e < ma + mb; e += NT) {
    const double4 r = e < ma ? a[e] : b[e - ma];
    const double w = r.w - r.z;
    if (w < bw) { bw = w; be = e; }  // finite only (NaN compares false)
  }
  block_argmin<NT>(bw, be);
  return be == INT_MAX ? 0.0 : (be < ma ? a[be].y : b[be - ma].y);
}

// In-place prefix sum of the NB-bin difference array by the NT threads of the
// block (all must call; ends with the sums in LDS, before a barrier). Thread t
// takes bins t S .. t S + S - 1, S = NB / NT odd, so that the lanes of a
// wavefront read distinct banks. Modular u32 arithmetic is exact: every true
// sum U + 65536 D is below 2^31.
template <int NB, int NT>
__device__ __forceinline__ void scan_bins(unsigned* bins, unsigned* part) {
  constexpr int S = NB / NT;
  static_assert(S * NT == NB && (S & 1), "bins per thread must be odd");
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  unsigned v[S];
  unsigned run = 0;
#pragma unroll
  for (int r = 0; r < S; ++r) {
    run += bins[t * S + r];
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
  for (int r = 0; r < S; ++r) bins[t * S + r] = v[r] + off;
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
