// Line detection by a coarse Hough transform followed by one exact LMS fit
// per accumulator peak (Section 5): the accumulator only finds the points of
// each putative line; the LMS fit of those points gives the line, so up to
// half of a cell's points may be noise or belong to another structure.
//
//   k_hough_clear  zero the accumulator (a fill kernel, no memset node)
//   k_hough_vote   every edge pixel votes once per angle bin:
//                  rho = x cos(theta_b) + y sin(theta_b) (two products and a
//                  sum in FP64, no contraction), bin floor((rho - rho_min) /
//                  d_rho); one thread per (pixel, angle), angles fastest so
//                  that the lanes of a wavefront hit different rows
//   k_hough_peaks  one workgroup: cells that are local maxima of their 3x3
//                  neighbourhood (plateaus broken by cell index) with enough
//                  votes, keyed (votes, -index); the max_lines largest keys by
//                  an 8-pass radix select, then sorted, strongest first
//   k_hough_count  one workgroup per peak: its supporting pixels, those whose
//                  vote at the peak's angle fell in the peak's rho bin
//   k_hough_gather one workgroup per peak: the supporting pixels in pixel
//                  order; a set larger than max_support keeps the max_support
//                  pixels with the smallest SplitMix64 keys (random sampling
//                  of a cell's points, Section 5); a steep line's set is
//                  stored transposed, (y, x), so that its fit x = a y + b is
//                  well conditioned
//   then lms_solve_batched on the sets.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "lms.h"
#include "lms_device.h"
#include "lms_host.h"

namespace {

using lms_dev::mix64;
using lms_host::fail;

constexpr int kNT = 1024;
constexpr int kWorkspaceTag = 5;
constexpr unsigned long long kGamma = 0x9E3779B97F4A7C15ull;
constexpr double kDegToRad = 0.017453292519943295;  // pi / 180, rounded to double

struct Grid {
  int n_theta, n_rho;
  double rho_min, d_rho;
};

__device__ __forceinline__ int rho_bin(int x, int y, double c, double s, const Grid& g) {
  const double rho = __dadd_rn(__dmul_rn((double)x, c), __dmul_rn((double)y, s));
  return (int)floor(__ddiv_rn(rho - g.rho_min, g.d_rho));
}

__global__ void k_hough_clear(int* __restrict__ acc, long long cells) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < cells;
       k += (long long)gridDim.x * blockDim.x)
    acc[k] = 0;
}

__global__ __launch_bounds__(256) void k_hough_vote(const int* __restrict__ pix, long long N,
                                                    const double2* __restrict__ trig, Grid g,
                                                    int* __restrict__ acc) {
  const long long total = N * g.n_theta;
  for (long long k = blockIdx.x * 256ll + threadIdx.x; k < total; k += (long long)gridDim.x * 256) {
    const long long p = k / g.n_theta;
    const int b = (int)(k - p * g.n_theta);
    const double2 cs = trig[b];
    const int r = rho_bin(pix[2 * p], pix[2 * p + 1], cs.x, cs.y, g);
    if (r >= 0 && r < g.n_rho) atomicAdd(&acc[(long long)b * g.n_rho + r], 1);
  }
}

// key of a cell: (votes << 32) | (~index), 0 if not a peak
__device__ __forceinline__ unsigned long long peak_key(const int* __restrict__ acc, const Grid& g,
                                                       int cell, int min_votes) {
  const int b = cell / g.n_rho, r = cell - b * g.n_rho;
  const int v = acc[cell];
  if (v < min_votes) return 0ull;
  for (int db = -1; db <= 1; ++db)
    for (int dr = -1; dr <= 1; ++dr) {
      if (!db && !dr) continue;
      const int bb = b + db, rr = r + dr;
      if (bb < 0 || bb >= g.n_theta || rr < 0 || rr >= g.n_rho) continue;
      const int nb = bb * g.n_rho + rr;
      const int u = acc[nb];
      // strictly above earlier cells, at least as high as later ones
      if (u > v || (u == v && nb < cell)) return 0ull;
    }
  return ((unsigned long long)(unsigned)v << 32) | (unsigned)(~(unsigned)cell);
}

// One workgroup: the K = max_lines largest peak keys, strongest first, as
// cell indices in peaks[0..*n_peaks).
__global__ __launch_bounds__(kNT) void k_hough_peaks(const int* __restrict__ acc, Grid g,
                                                     int min_votes, int K,
                                                     int* __restrict__ peaks,
                                                     int* __restrict__ n_peaks) {
  __shared__ unsigned hist[256];
  __shared__ unsigned long long s_prefix;
  __shared__ unsigned s_rank, s_total, s_cnt;
  __shared__ unsigned long long sel[kNT];
  const int t = threadIdx.x;
  const int cells = g.n_theta * g.n_rho;
  if (t == 0) {
    s_total = 0;
    s_cnt = 0;
  }
  __syncthreads();
  unsigned mine = 0;
  for (int c = t; c < cells; c += kNT) mine += peak_key(acc, g, c, min_votes) != 0ull;
  atomicAdd(&s_total, mine);
  __syncthreads();
  const unsigned total = s_total;
  const unsigned take = min(total, (unsigned)K);
  unsigned long long T = 1ull;  // threshold key: take every key >= T
  if (take > 0 && take < total) {
    // the take-th largest key: radix select on the complemented keys
    if (t == 0) {
      s_prefix = 0;
      s_rank = take;
    }
    for (int pass = 0; pass < 8; ++pass) {
      const int shift = 56 - 8 * pass;
      for (int d = t; d < 256; d += kNT) hist[d] = 0;
      __syncthreads();
      const unsigned long long prefix = s_prefix;
      const unsigned long long hmask = pass == 0 ? 0ull : ~0ull << (shift + 8);
      for (int c = t; c < cells; c += kNT) {
        const unsigned long long k = peak_key(acc, g, c, min_votes);
        if (!k) continue;
        const unsigned long long ck = ~k;
        if ((ck & hmask) == prefix) atomicAdd(&hist[(ck >> shift) & 0xFF], 1u);
      }
      __syncthreads();
      if (t == 0) {
        unsigned r = s_rank, d = 0;
        while (hist[d] < r) r -= hist[d++];
        s_rank = r;
        s_prefix = prefix | ((unsigned long long)d << shift);
      }
      __syncthreads();
    }
    T = ~s_prefix;  // keys are distinct (they hold the cell index)
  }
  // collect the selected keys (at most K <= kNT), then sort them descending
  for (int c = t; c < cells; c += kNT) {
    const unsigned long long k = peak_key(acc, g, c, min_votes);
    if (k && k >= T) {
      const unsigned slot = atomicAdd(&s_cnt, 1u);
      if (slot < (unsigned)kNT) sel[slot] = k;
    }
  }
  __syncthreads();
  const unsigned cnt = min(s_cnt, (unsigned)kNT);
  for (unsigned k = cnt + t; k < (unsigned)kNT; k += kNT) sel[k] = 0ull;
  __syncthreads();
  // bitonic sort, descending, kNT keys by kNT/2 threads
  for (int size = 2; size <= kNT; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (t < kNT / 2) {
        const int lo = 2 * t - (t & (stride - 1)), hi = lo + stride;
        const bool desc = (lo & size) == 0;
        const unsigned long long a = sel[lo], b = sel[hi];
        if ((a < b) == desc && a != b) {
          sel[lo] = b;
          sel[hi] = a;
        }
      }
      __syncthreads();
    }
  if (t < (int)cnt) {
    peaks[t] = (int)(~(unsigned)(sel[t] & 0xFFFFFFFFull));
    peaks[K + t] = (int)(sel[t] >> 32);  // votes
  }
  if (t == 0) *n_peaks = (int)cnt;
}

__device__ __forceinline__ bool supports(const int* __restrict__ pix, long long p,
                                         const double2* __restrict__ trig, const Grid& g, int b,
                                         int r) {
  const double2 cs = trig[b];
  return rho_bin(pix[2 * p], pix[2 * p + 1], cs.x, cs.y, g) == r;
}

__global__ __launch_bounds__(kNT) void k_hough_count(const int* __restrict__ pix, long long N,
                                                     const double2* __restrict__ trig, Grid g,
                                                     const int* __restrict__ peaks,
                                                     const int* __restrict__ n_peaks,
                                                     int* __restrict__ counts) {
  __shared__ unsigned s_n;
  const int k = blockIdx.x;
  if (k >= *n_peaks) return;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  const int cell = peaks[k], b = cell / g.n_rho, r = cell - b * g.n_rho;
  unsigned mine = 0;
  for (long long p = threadIdx.x; p < N; p += kNT) mine += supports(pix, p, trig, g, b, r);
  atomicAdd(&s_n, mine);
  __syncthreads();
  if (threadIdx.x == 0) counts[k] = (int)s_n;
}

__device__ __forceinline__ unsigned long long sample_key(unsigned long long seed, long long p) {
  return mix64(seed + (unsigned long long)(p + 1) * kGamma);
}

// One workgroup per peak: its supporting pixels in pixel order into
// xy[off[k] ..), sampled down to off[k+1] - off[k] points when there are more.
__global__ __launch_bounds__(kNT) void k_hough_gather(const int* __restrict__ pix, long long N,
                                                      const double2* __restrict__ trig, Grid g,
                                                      const int* __restrict__ peaks,
                                                      const int* __restrict__ counts,
                                                      const int64_t* __restrict__ off,
                                                      unsigned long long seed,
                                                      double* __restrict__ xy) {
  __shared__ unsigned hist[256];
  __shared__ unsigned long long s_prefix;
  __shared__ unsigned s_rank;
  __shared__ unsigned wave_tot[kNT / 64];
  const int k = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int cell = peaks[k], b = cell / g.n_rho, r = cell - b * g.n_rho;
  const unsigned m = (unsigned)(off[k + 1] - off[k]);
  const bool sampled = (unsigned)counts[k] > m;
  // a steep line (normal within 45 degrees of the x axis) is fitted as x(y)
  const bool steep = fabs(trig[b].x) > fabs(trig[b].y);
  unsigned long long T = ~0ull;
  unsigned need_eq = UINT_MAX;
  if (sampled) {
    if (t == 0) {
      s_prefix = 0;
      s_rank = m;
    }
    for (int pass = 0; pass < 8; ++pass) {
      const int shift = 56 - 8 * pass;
      for (int d = t; d < 256; d += kNT) hist[d] = 0;
      __syncthreads();
      const unsigned long long prefix = s_prefix;
      const unsigned long long hmask = pass == 0 ? 0ull : ~0ull << (shift + 8);
      for (long long p = t; p < N; p += kNT) {
        if (!supports(pix, p, trig, g, b, r)) continue;
        const unsigned long long key = sample_key(seed, p);
        if ((key & hmask) == prefix) atomicAdd(&hist[(key >> shift) & 0xFF], 1u);
      }
      __syncthreads();
      if (t == 0) {
        unsigned rr = s_rank, d = 0;
        while (hist[d] < rr) rr -= hist[d++];
        s_rank = rr;
        s_prefix = prefix | ((unsigned long long)d << shift);
      }
      __syncthreads();
    }
    T = s_prefix;
    need_eq = s_rank;
  }
  unsigned base = 0, eq_base = 0;
  double* out = xy + 2 * off[k];
  for (long long p0 = 0; p0 < N; p0 += kNT) {
    const long long p = p0 + t;
    const bool sup = p < N && supports(pix, p, trig, g, b, r);
    const unsigned long long key = sup && sampled ? sample_key(seed, p) : 0ull;
    const bool lt = sup && (!sampled || key < T), eq = sup && sampled && key == T;
    const unsigned long long eqm = __ballot(eq);
    if (lane == 0) wave_tot[wv] = __popcll(eqm);
    __syncthreads();
    unsigned eq_rank = eq_base + __popcll(eqm & ((1ull << lane) - 1)), eq_round = 0;
    for (int w = 0; w < kNT / 64; ++w) {
      if (w < wv) eq_rank += wave_tot[w];
      eq_round += wave_tot[w];
    }
    __syncthreads();
    const bool take = lt || (eq && eq_rank < need_eq);
    const unsigned long long tm = __ballot(take);
    if (lane == 0) wave_tot[wv] = __popcll(tm);
    __syncthreads();
    unsigned pos = base + __popcll(tm & ((1ull << lane) - 1)), round = 0;
    for (int w = 0; w < kNT / 64; ++w) {
      if (w < wv) pos += wave_tot[w];
      round += wave_tot[w];
    }
    if (take && pos < m) {
      const double x = (double)pix[2 * p], y = (double)pix[2 * p + 1];
      out[2 * pos] = steep ? y : x;
      out[2 * pos + 1] = steep ? x : y;
    }
    base += round;
    eq_base += eq_round;
    __syncthreads();
  }
}

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

extern "C" lms_status lms_detect_lines(const int32_t* d_pix, int64_t N,
                                       const lms_hough_params* prm, int32_t* d_acc,
                                       lms_line* lines, int32_t* n_lines, void* stream) {
  lms_host::clear_error();
  if (!prm || !lines || !n_lines || (N > 0 && !d_pix)) return fail(LMS_ERR_ARG, "null pointer");
  if (prm->struct_size < sizeof(lms_hough_params)) return fail(LMS_ERR_ARG, "bad params size");
  const lms_hough_params p = *prm;
  if (N < 0 || N > (1ll << 30)) return fail(LMS_ERR_ARG, "N must be in [0, 2^30]");
  if (p.width < 1 || p.height < 1 || p.width > (1 << 20) || p.height > (1 << 20))
    return fail(LMS_ERR_ARG, "image size must be in [1, 2^20]");
  if (!(p.d_rho >= 0.25) || !(p.d_theta_deg > 0.0) || !(p.d_theta_deg <= 180.0))
    return fail(LMS_ERR_ARG, "d_rho must be >= 0.25 and d_theta_deg in (0, 180]");
  if (p.max_lines < 1 || p.max_lines > LMS_HOUGH_MAX_LINES)
    return fail(LMS_ERR_ARG, "max_lines must be in [1, " + std::to_string(LMS_HOUGH_MAX_LINES) + "]");
  if (p.min_votes < 2) return fail(LMS_ERR_ARG, "min_votes must be >= 2");
  if (p.max_support < 2 || p.max_support > LMS_BATCH_MAX_N)
    return fail(LMS_ERR_ARG, "max_support must be in [2, LMS_BATCH_MAX_N]");
  Grid g;
  g.n_theta = (int)std::ceil(180.0 / p.d_theta_deg);
  g.rho_min = -(double)(p.width - 1);
  g.d_rho = p.d_rho;
  g.n_rho = (int)std::floor((double)(2 * (p.width - 1) + (p.height - 1)) / p.d_rho) + 1;
  const long long cells = (long long)g.n_theta * g.n_rho;
  if (cells > (1ll << 28)) return fail(LMS_ERR_ARG, "accumulator too large");
  // angle table on the host: theta_b = b * (d_theta * pi / 180)
  std::vector<double2> trig(g.n_theta);
  const double step = p.d_theta_deg * kDegToRad;
  for (int b = 0; b < g.n_theta; ++b) {
    const double th = (double)b * step;
    trig[b] = make_double2(std::cos(th), std::sin(th));
  }
  const int K = p.max_lines;
  hipStream_t s = (hipStream_t)stream;
  const size_t o_trig = 0;
  const size_t o_acc = o_trig + up256(g.n_theta * sizeof(double2));
  const size_t o_peaks = o_acc + (d_acc ? 0 : up256((size_t)cells * sizeof(int)));
  const size_t o_counts = o_peaks + up256((2 * K + 1) * sizeof(int));
  const size_t o_off = o_counts + up256(K * sizeof(int));
  const size_t o_xy = o_off + up256((K + 1) * sizeof(long long));
  const size_t o_res = o_xy + up256((size_t)K * p.max_support * 2 * sizeof(double));
  const size_t total = o_res + up256(K * sizeof(lms_result));
  char* base = nullptr;
  lms_status st = lms_host::get_workspace(kWorkspaceTag, stream, total, &base);
  if (st != LMS_OK) return st;
  double2* d_trig = (double2*)(base + o_trig);
  int* acc = d_acc ? d_acc : (int*)(base + o_acc);
  int* d_peaks = (int*)(base + o_peaks);
  int* d_npk = d_peaks + 2 * K;  // cells [0, K), votes [K, 2K), count
  int* d_counts = (int*)(base + o_counts);
  int64_t* d_off = (int64_t*)(base + o_off);
  double* d_sets = (double*)(base + o_xy);
  lms_result* d_res = (lms_result*)(base + o_res);
  auto dev_fail = [&](hipError_t e, const char* what) {
    return fail(LMS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e = hipMemcpyAsync(d_trig, trig.data(), g.n_theta * sizeof(double2),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return dev_fail(e, "trig copy");
  const int cu = lms_host::num_cu();
  hipLaunchKernelGGL(k_hough_clear, dim3((unsigned)std::min<long long>((cells + 255) / 256, 8 * cu)),
                     dim3(256), 0, s, acc, cells);
  if (N > 0) {
    const long long work = N * g.n_theta;
    hipLaunchKernelGGL(k_hough_vote, dim3((unsigned)std::min<long long>((work + 255) / 256, 16 * cu)),
                       dim3(256), 0, s, (const int*)d_pix, (long long)N, d_trig, g, acc);
  }
  hipLaunchKernelGGL(k_hough_peaks, dim3(1), dim3(kNT), 0, s, acc, g, p.min_votes, K, d_peaks,
                     d_npk);
  hipLaunchKernelGGL(k_hough_count, dim3(K), dim3(kNT), 0, s, (const int*)d_pix, (long long)N,
                     d_trig, g, d_peaks, d_npk, d_counts);
  e = hipGetLastError();
  if (e != hipSuccess) return dev_fail(e, "launch");
  // the sizes of the supporting sets decide the batch's plan: one sync
  std::vector<int> h_peaks(2 * K + 1), h_counts(K);
  e = hipMemcpyAsync(h_peaks.data(), d_peaks, (2 * K + 1) * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h_counts.data(), d_counts, K * sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(e, "peak readback");
  const int np = h_peaks[2 * K];
  std::vector<int64_t> h_off(np + 1, 0);
  for (int k = 0; k < np; ++k) h_off[k + 1] = h_off[k] + std::min(h_counts[k], p.max_support);
  *n_lines = np;
  if (np == 0) return LMS_OK;
  e = hipMemcpyAsync(d_off, h_off.data(), (np + 1) * sizeof(long long), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return dev_fail(e, "offset copy");
  hipLaunchKernelGGL(k_hough_gather, dim3(np), dim3(kNT), 0, s, (const int*)d_pix, (long long)N,
                     d_trig, g, d_peaks, d_counts, d_off, (unsigned long long)p.seed, d_sets);
  e = hipGetLastError();
  if (e != hipSuccess) return dev_fail(e, "launch");
  // a cell with fewer than two points gets LMS_ERR_ARG in its own result
  st = lms_solve_batched(d_sets, d_off, h_off.data(), np, nullptr, d_res, nullptr, stream);
  if (st != LMS_OK) return st;
  std::vector<lms_result> res(np);
  e = hipMemcpyAsync(res.data(), d_res, np * sizeof(lms_result), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return dev_fail(e, "result readback");
  for (int k = 0; k < np; ++k) {
    lms_line& L = lines[k];
    std::memset(&L, 0, sizeof(L));
    L.theta_bin = h_peaks[k] / g.n_rho;
    L.rho_bin = h_peaks[k] - L.theta_bin * g.n_rho;
    L.votes = h_peaks[K + k];
    L.support = h_counts[k];
    L.fitted = (int32_t)(h_off[k + 1] - h_off[k]);
    L.transposed = std::fabs(trig[L.theta_bin].x) > std::fabs(trig[L.theta_bin].y);
    L.result = res[k];
  }
  return LMS_OK;
}
