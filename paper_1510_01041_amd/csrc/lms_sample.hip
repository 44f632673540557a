// Random sampling of a large point set before the exact search (Section 5:
// the LMS step of the line detector can be sped up by randomly sampling the
// feature points that voted for a Hough cell). The answer is approximate: it
// is the exact LMS line of the sample, not of the whole set.
//
// The sample is the m points with the smallest keys, key_k = SplitMix64's
// (k+1)-th output for the state `seed` (Steele, Lea and Flood, OOPSLA 2014):
// mix64(seed + (k + 1) * 0x9E3779B97F4A7C15). That is a uniform draw of m of
// the n points without replacement, the same on every device for a seed.
//
//   k_sample  one workgroup: the m-th smallest key by an 8-pass radix select
//             (keys recomputed per pass, nothing stored), then the sample
//             gathered in index order (points below the threshold key, and
//             the first of those equal to it).
//   lms_solve on the gathered points (any of its options), then
//   k_unmap   the result's pair indices taken back to the input's numbering.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <string>

#include "lms.h"
#include "lms_device.h"
#include "lms_host.h"

namespace {

using lms_dev::mix64;
using lms_host::fail;

constexpr int kNT = 1024;
constexpr int kWorkspaceTag = 4;
constexpr unsigned long long kGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ unsigned long long sample_key(unsigned long long seed, long long k) {
  return mix64(seed + (unsigned long long)(k + 1) * kGamma);
}

__global__ __launch_bounds__(kNT) void k_sample(const double* __restrict__ xy, long long n,
                                                int m, unsigned long long seed,
                                                double* __restrict__ sxy, int* __restrict__ sidx) {
  __shared__ unsigned hist[256];
  __shared__ unsigned long long s_prefix;
  __shared__ unsigned s_rank;
  __shared__ unsigned wave_tot[kNT / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (t == 0) {
    s_prefix = 0;
    s_rank = (unsigned)m;  // 1-based rank of the threshold key among the keys
  }
  // radix select, most significant byte first
  for (int pass = 0; pass < 8; ++pass) {
    const int shift = 56 - 8 * pass;
    for (int d = t; d < 256; d += kNT) hist[d] = 0;
    __syncthreads();
    const unsigned long long prefix = s_prefix;
    const unsigned long long hmask = pass == 0 ? 0ull : ~0ull << (shift + 8);
    for (long long k = t; k < n; k += kNT) {
      const unsigned long long key = sample_key(seed, k);
      if ((key & hmask) == prefix) atomicAdd(&hist[(key >> shift) & 0xFF], 1u);
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
  const unsigned long long T = s_prefix;  // the m-th smallest key
  const unsigned need_eq = s_rank;        // keys equal to T that are taken (in index order)
  // gather in index order, 1024 indices per round
  unsigned base = 0, eq_base = 0;
  for (long long k0 = 0; k0 < n; k0 += kNT) {
    const long long k = k0 + t;
    const unsigned long long key = k < n ? sample_key(seed, k) : ~0ull;
    const bool lt = k < n && key < T, eq = k < n && key == T;
    // rank among this round's equal keys, then whether it is taken
    const unsigned long long eqm = __ballot(eq);
    const unsigned eq_before_wave = __popcll(eqm & ((1ull << lane) - 1));
    if (lane == 0) wave_tot[wv] = __popcll(eqm);
    __syncthreads();
    unsigned eq_rank = eq_base + eq_before_wave, eq_round = 0;
    for (int w = 0; w < kNT / 64; ++w) {
      if (w < wv) eq_rank += wave_tot[w];
      eq_round += wave_tot[w];
    }
    __syncthreads();
    const bool take = lt || (eq && eq_rank < need_eq);
    const unsigned long long tm = __ballot(take);
    const unsigned before_wave = __popcll(tm & ((1ull << lane) - 1));
    if (lane == 0) wave_tot[wv] = __popcll(tm);
    __syncthreads();
    unsigned pos = base + before_wave, round = 0;
    for (int w = 0; w < kNT / 64; ++w) {
      if (w < wv) pos += wave_tot[w];
      round += wave_tot[w];
    }
    if (take && pos < (unsigned)m) {
      sxy[2 * pos] = xy[2 * k];
      sxy[2 * pos + 1] = xy[2 * k + 1];
      sidx[pos] = (int)k;
    }
    base += round;
    eq_base += eq_round;
    __syncthreads();
  }
}

__global__ void k_unmap(lms_result* out, const int* __restrict__ sidx) {
  if (threadIdx.x == 0) {
    if (out->pair_i >= 0) out->pair_i = sidx[out->pair_i];
    if (out->pair_j >= 0) out->pair_j = sidx[out->pair_j];
  }
}

}  // namespace

extern "C" lms_status lms_solve_sampled(const double* d_xy, int64_t n, int64_t h, int64_t m,
                                        uint64_t seed, lms_result* d_out,
                                        const lms_options* opt, void* stream) {
  lms_host::clear_error();
  if (!d_xy || !d_out) return fail(LMS_ERR_ARG, "null pointer");
  if (n < 2 || n > LMS_SAMPLE_MAX_N)
    return fail(LMS_ERR_ARG, "n must be in [2, 2^30]");
  if (m < 2 || m > n || m > LMS_MAX_N)
    return fail(LMS_ERR_ARG, "m must be in [2, min(n, " + std::to_string(LMS_MAX_N) + ")]");
  if (h != 0 && (h < 2 || h > n)) return fail(LMS_ERR_ARG, "h must be 0 or in [2, n]");
  // the same fraction of the sample: ceil(h m / n), at least 2
  int64_t hm = 0;
  if (h != 0) {
    hm = (h * m + n - 1) / n;
    if (hm < 2) hm = 2;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t o_idx = ((size_t)m * 2 * sizeof(double) + 255) & ~size_t(255);
  char* base = nullptr;
  lms_status st = lms_host::get_workspace(kWorkspaceTag, stream, o_idx + (size_t)m * sizeof(int),
                                          &base);
  if (st != LMS_OK) return st;
  double* sxy = (double*)base;
  int* sidx = (int*)(base + o_idx);
  hipLaunchKernelGGL(k_sample, dim3(1), dim3(kNT), 0, s, d_xy, (long long)n, (int)m,
                     (unsigned long long)seed, sxy, sidx);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return fail(LMS_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(err));
  st = lms_solve(sxy, m, hm, d_out, opt, stream);
  if (st != LMS_OK) return st;
  hipLaunchKernelGGL(k_unmap, dim3(1), dim3(64), 0, s, d_out, sidx);
  err = hipGetLastError();
  if (err != hipSuccess) return fail(LMS_ERR_DEVICE, std::string("launch: ") + hipGetErrorString(err));
  return LMS_OK;
}
