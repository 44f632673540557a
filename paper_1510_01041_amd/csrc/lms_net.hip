// Point-set network that proposes a seed slope for the exact search.
//
// Not part of the paper's method: a proposal can only tighten the screen's
// initial width bound, because F(theta) >= the optimal width for every theta
// (Eq. (1)). The exhaustive search stays exact whatever the network says.
//
// Architecture, for one set of points in a [-1, 1]^2 frame:
//   h1 = relu(W1 p + b1) (64) -> BF16
//   h2 = relu(W2 h1 + b2) (64), W2 . h1 by v_dot2 BF16 pairs into FP32
//   g = max over points of h2 (64)
//   h3 = relu(W3 g + b3) (64);  out = W4 h3 + b4 (2) ~ (cos 2phi, sin 2phi)
// Weights are BF16 roundings (ties to even) of FP32 masters, taken at load.
// Parameters are packed FP32 in the order W1 b1 W2 b2 W3 b3 W4 b4 (row-major,
// W[out][in]).
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

using lms_host::fail;

constexpr int H = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + H * 2, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H * H, OFF_W4 = OFF_B3 + H,
              OFF_B4 = OFF_W4 + 2 * H, N_PARAMS = OFF_B4 + 2;
static_assert(N_PARAMS == LMS_NET_PARAMS, "parameter count");

constexpr int NT = 256;

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// FP32 -> BF16 bits, round to nearest, ties to even.
__device__ __forceinline__ unsigned bf16_bits(float f) {
  const unsigned u = __float_as_uint(f);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_round(float f) { return __uint_as_float(bf16_bits(f) << 16); }
__device__ __forceinline__ unsigned pack2(float a, float b) {
  return bf16_bits(a) | (bf16_bits(b) << 16);
}
__device__ __forceinline__ float dot2(unsigned w, unsigned x, float acc) {
  return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, w),
                                         __builtin_bit_cast(bf16x2, x), acc, false);
}

// Weights of the point MLP in LDS: W1/b1/b2 as FP32 (W1 rounded), W2 as BF16
// pairs: s_w2[c][k/2] = (W2[c][k], W2[c][k+1]).
struct PointMLP {
  float w1[H * 2], b1[H], b2[H];
  unsigned w2[H * H / 2];
};

__device__ void load_point_mlp(const float* __restrict__ P, PointMLP& s) {
  for (int i = threadIdx.x; i < H * 2; i += blockDim.x) s.w1[i] = bf16_round(P[OFF_W1 + i]);
  for (int i = threadIdx.x; i < H; i += blockDim.x) {
    s.b1[i] = P[OFF_B1 + i];
    s.b2[i] = P[OFF_B2 + i];
  }
  for (int i = threadIdx.x; i < H * H / 2; i += blockDim.x)
    s.w2[i] = pack2(P[OFF_W2 + 2 * i], P[OFF_W2 + 2 * i + 1]);
  __syncthreads();
}

// Layer 1 of one point, packed as BF16 pairs.
__device__ __forceinline__ void layer1(const PointMLP& s, float x, float y, unsigned (&h1)[H / 2]) {
#pragma unroll
  for (int k = 0; k < H / 2; ++k) {
    const float a = fmaxf(fmaf(s.w1[4 * k + 1], y, fmaf(s.w1[4 * k], x, s.b1[2 * k])), 0.0f);
    const float b = fmaxf(fmaf(s.w1[4 * k + 3], y, fmaf(s.w1[4 * k + 2], x, s.b1[2 * k + 1])), 0.0f);
    h1[k] = pack2(a, b);
  }
}

// Pre-activation of layer 2, channel c.
__device__ __forceinline__ float layer2(const PointMLP& s, const unsigned (&h1)[H / 2], int c) {
  float acc = s.b2[c];
#pragma unroll
  for (int k = 0; k < H / 2; ++k) acc = dot2(s.w2[c * (H / 2) + k], h1[k], acc);
  return acc;
}

__device__ __forceinline__ float wave_max(float v) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ int wave_min_i(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

// ---------------------------------------------------------------- kernels

// Frame of set b: per coordinate the lower median of a fixed sample of its
// points (all of them up to kFrameSample, else indices floor(k n /
// kFrameSample)), and as scale the lower median of the absolute deviations
// from it (the MAD), else the largest deviation, else 1. The sample is
// sorted in LDS (a value of given rank does not depend on how equal values
// are ordered). Called by all NT threads; every thread gets (cx, cy, sx, sy).
constexpr int kFrameSample = 255;
static_assert(kFrameSample <= NT, "one sample value per thread");

// Ascending bitonic sort of 256 doubles in LDS by one wavefront (two pairs
// per lane per stage). A wavefront's LDS operations execute in order, so a
// stage sees the previous one's writes; the fence only keeps the compiler
// from reordering them.
__device__ void wave_sort256(double* a) {
  const int lane = threadIdx.x & 63;
  for (int k = 2; k <= 256; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int pidx = lane + 64 * q;
        const int lo = 2 * pidx - (pidx & (j - 1)), hi = lo + j;
        const bool up = (lo & k) == 0;
        const double x = a[lo], y = a[hi];
        if ((x > y) == up) {
          a[lo] = y;
          a[hi] = x;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// set_frame: wavefront 0 takes x, wavefront 1 takes y, each on its own LDS
// array: sort the sample values, read the median (a value, so the order of
// equal values does not matter), then sort the absolute deviations from it
// and read their median and largest value. One block barrier at the end.
__device__ double4 set_frame(const double* __restrict__ xy, int64_t o, int64_t n) {
  static_assert(NT >= 128 && kFrameSample < 256, "two wavefronts, 256 slots");
  __shared__ double sv[2][256];
  __shared__ double s_out[6];  // medians x, y; MADs x, y; largest deviations x, y
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int m = n < kFrameSample ? (int)n : kFrameSample;
  const int target = m > 0 ? (m - 1) / 2 : 0;
  if (wv < 2) {
    double* a = sv[wv];
    double orig[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = r * 64 + lane;
      double val = INFINITY;
      if (v < m) {
        const int64_t q = n <= kFrameSample ? v : ((int64_t)v * n) / kFrameSample;
        val = xy[2 * (o + q) + wv];
      }
      orig[r] = val;
      a[v] = val;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    wave_sort256(a);
    const double c = m > 0 ? a[target] : 0.0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int v = r * 64 + lane;
      a[v] = v < m ? fabs(orig[r] - c) : INFINITY;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    wave_sort256(a);
    if (lane == 0) {
      s_out[wv] = c;
      s_out[2 + wv] = m > 0 ? a[target] : 0.0;
      s_out[4 + wv] = m > 0 ? a[m - 1] : 0.0;
    }
  }
  __syncthreads();
  double sx = s_out[2], sy = s_out[3];
  if (!(sx > 0)) sx = s_out[4];
  if (!(sx > 0)) sx = 1.0;
  if (!(sy > 0)) sy = s_out[5];
  if (!(sy > 0)) sy = 1.0;
  const double4 f = make_double4(s_out[0], s_out[1], sx, sy);
  __syncthreads();  // the shared values are reused by the next call
  return f;
}

__device__ __forceinline__ float2 to_frame(const double* __restrict__ xy, int64_t k,
                                           const double4& f) {
  return make_float2((float)((xy[2 * k] - f.x) / f.z), (float)((xy[2 * k + 1] - f.y) / f.w));
}

// Robust frame per set (set_frame); FP32 points in that frame.
__global__ __launch_bounds__(NT) void k_net_prepare(const double* __restrict__ xy,
                                                    const int64_t* __restrict__ off,
                                                    float2* __restrict__ pts,
                                                    double* __restrict__ scale) {
  const int b = blockIdx.x, t = threadIdx.x;
  const int64_t o = off[b], n = off[b + 1] - off[b];
  const double4 f = set_frame(xy, o, n);
  if (t == 0) {
    scale[4 * b] = f.x; scale[4 * b + 1] = f.y; scale[4 * b + 2] = f.z; scale[4 * b + 3] = f.w;
  }
  for (int64_t k = t; k < n; k += NT) pts[o + k] = to_frame(xy, o + k, f);
}

// Max-pooled point features g (B x 64) and the head's output (B x 2).
__global__ __launch_bounds__(NT) void k_net_forward(const float* __restrict__ P,
                                                    const float2* __restrict__ pts,
                                                    const int64_t* __restrict__ off,
                                                    float* __restrict__ out, float* __restrict__ g_out) {
  __shared__ PointMLP s;
  __shared__ float s_max[NT / 64][H];
  __shared__ float s_g[H], s_h3[H];
  load_point_mlp(P, s);
  const int b = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t o = off[b], n = off[b + 1] - off[b];
  float run[H];
#pragma unroll
  for (int c = 0; c < H; ++c) run[c] = 0.0f;  // h2 >= 0 after relu
  for (int64_t k = t; k < n; k += NT) {
    // keep the weights in LDS: without this the compiler hoists all 2048 W2
    // loads out of the point loop and spills them
    asm volatile("" ::: "memory");
    const float2 p = pts[o + k];
    unsigned h1[H / 2];
    layer1(s, p.x, p.y, h1);
#pragma unroll
    for (int c = 0; c < H; ++c) run[c] = fmaxf(run[c], fmaxf(layer2(s, h1, c), 0.0f));
  }
#pragma unroll
  for (int c = 0; c < H; ++c) {
    const float m = wave_max(run[c]);
    if (lane == 0) s_max[wv][c] = m;
  }
  __syncthreads();
  if (t < H) {
    float m = s_max[0][t];
    for (int w = 1; w < NT / 64; ++w) m = fmaxf(m, s_max[w][t]);
    s_g[t] = m;
    if (g_out) g_out[(size_t)b * H + t] = m;
  }
  __syncthreads();
  if (t < H) {
    float a = P[OFF_B3 + t];
    for (int k = 0; k < H; ++k) a = fmaf(bf16_round(P[OFF_W3 + t * H + k]), s_g[k], a);
    s_h3[t] = fmaxf(a, 0.0f);
  }
  __syncthreads();
  if (t < 2) {
    float a = P[OFF_B4 + t];
    for (int k = 0; k < H; ++k) a = fmaf(bf16_round(P[OFF_W4 + t * H + k]), s_h3[k], a);
    out[2 * b + t] = a;
  }
}

// ---------------------------------------------------------------- inference

// Inference spreads each set over many workgroups: the frame kernel finds
// the set's frame (set_frame), the pool kernel gives every workgroup
// kPoolPoints points (one per lane) and each of its NT / 64 wavefronts a
// quarter of the channels, and the head kernel runs once g is complete. The
// max-pool is order-free, so the workgroups merge their maxima into g with
// atomicMax on the float bits (every h2 >= 0 after the ReLU, and non-negative
// floats order as their bit patterns): the result equals k_net_forward's bit
// for bit. A set of more than max_points points is read at max_points evenly
// strided indices floor(j n / max_points).
constexpr int NTF = 256;
constexpr int kPoolPoints = 64;
constexpr int kPoolChannels = H / (NT / 64);

// The point MLP's weights as the pool kernel reads them, written by the
// frame kernel's block 0 from the FP32 masters: W1 rounded to BF16 (as FP32),
// b1, b2, then W2 as BF16 pairs (the PointMLP layout). Each pool workgroup
// copies them to LDS once and its wavefronts read them as broadcasts.
constexpr int WPK_W1 = 0, WPK_B1 = WPK_W1 + 2 * H, WPK_B2 = WPK_B1 + H, WPK_W2 = WPK_B2 + H,
              WPK_WORDS = WPK_W2 + H * H / 2;

__global__ __launch_bounds__(NTF) void k_net_frame(const float* __restrict__ P,
                                                   const double* __restrict__ xy,
                                                   const int64_t* __restrict__ off,
                                                   int64_t n_single, double* __restrict__ scale,
                                                   unsigned* __restrict__ g,
                                                   unsigned* __restrict__ wpk) {
  const int b = blockIdx.x, t = threadIdx.x;
  // the wavefronts that set_frame leaves idle pack the weights meanwhile
  if (b == 0 && t >= 128) {
    const int u = t - 128, nu = NTF - 128;
    for (int i = u; i < 2 * H; i += nu) wpk[WPK_W1 + i] = __float_as_uint(bf16_round(P[OFF_W1 + i]));
    for (int i = u; i < H; i += nu) {
      wpk[WPK_B1 + i] = __float_as_uint(P[OFF_B1 + i]);
      wpk[WPK_B2 + i] = __float_as_uint(P[OFF_B2 + i]);
    }
    for (int i = u; i < H * H / 2; i += nu)
      wpk[WPK_W2 + i] = pack2(P[OFF_W2 + 2 * i], P[OFF_W2 + 2 * i + 1]);
  }
  const int64_t o = off ? off[b] : 0, n = off ? off[b + 1] - off[b] : n_single;
  const double4 f = set_frame(xy, o, n);
  if (t == 0) {
    scale[4 * b] = f.x; scale[4 * b + 1] = f.y; scale[4 * b + 2] = f.z; scale[4 * b + 3] = f.w;
  }
  if (t < H) g[(size_t)b * H + t] = 0u;
}

// Lane = point, wavefront = a quarter of the channels: layer 1 (each
// wavefront computes it for its 64 points), then its channels of layer 2
// (the same products in the same order as layer1/layer2) and their ReLU; the
// channel maxima over the wavefront by a halving exchange (each step keeps
// half of a lane's channels and takes the partner lane's values for them:
// 8 + 4 + 2 + 1 + 1 + 1 shuffles for 16 channels); the workgroup's maxima
// merge into g. The workgroup copies the packed weights to LDS first (one
// global latency), and the wavefronts read them as broadcasts.
__global__ __launch_bounds__(NT) void k_net_pool(const unsigned* __restrict__ wpk,
                                                 const double* __restrict__ xy,
                                                 const int64_t* __restrict__ off, int64_t n_single,
                                                 int max_points, const double* __restrict__ scale,
                                                 unsigned* __restrict__ g) {
  static_assert(kPoolChannels == 16, "four halving steps");
  static_assert(WPK_WORDS % 4 == 0, "uint4 copy");
  __shared__ float s_max[H];
  __shared__ uint4 s_w[WPK_WORDS / 4];  // the packed weights, one copy per workgroup
  const int b = blockIdx.y, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t o = off ? off[b] : 0, n = off ? off[b + 1] - off[b] : n_single;
  const int64_t m = n < max_points ? n : max_points;
  const int64_t j0 = (int64_t)blockIdx.x * kPoolPoints;
  if (j0 >= m) return;  // uniform over the block
  // the point's load, then the weights' (all in flight together), one wait
  const int64_t j = j0 + lane;
  const bool live = j < m;
  const int64_t k = n <= max_points ? j : (j * n) / max_points;
  const double2 pt = live ? reinterpret_cast<const double2*>(xy)[o + k] : make_double2(0.0, 0.0);
  const uint4* wsrc = reinterpret_cast<const uint4*>(wpk);
  for (int e = t; e < WPK_WORDS / 4; e += NT) s_w[e] = wsrc[e];
  __syncthreads();
  const double4 f = make_double4(scale[4 * b], scale[4 * b + 1], scale[4 * b + 2], scale[4 * b + 3]);
  const float2 p = make_float2((float)((pt.x - f.x) / f.z), (float)((pt.y - f.y) / f.w));
  const unsigned* sw = reinterpret_cast<const unsigned*>(s_w);
  const float* w1 = reinterpret_cast<const float*>(sw + WPK_W1);
  const float* b1 = reinterpret_cast<const float*>(sw + WPK_B1);
  unsigned h1[H / 2];
#pragma unroll
  for (int q = 0; q < H / 2; ++q) {
    const float a = fmaxf(fmaf(w1[4 * q + 1], p.y, fmaf(w1[4 * q], p.x, b1[2 * q])), 0.0f);
    const float c = fmaxf(fmaf(w1[4 * q + 3], p.y, fmaf(w1[4 * q + 2], p.x, b1[2 * q + 1])), 0.0f);
    h1[q] = pack2(a, c);
  }
  const int c0 = wv * kPoolChannels;
  const uint4* w2v = s_w + (WPK_W2 + c0 * (H / 2)) / 4;
  const float* b2v = reinterpret_cast<const float*>(sw + WPK_B2 + c0);
  float r[kPoolChannels];
#pragma unroll
  for (int cc = 0; cc < kPoolChannels; ++cc) {
    uint4 w[H / 8];
#pragma unroll
    for (int q4 = 0; q4 < H / 8; ++q4) w[q4] = w2v[cc * (H / 8) + q4];
    float acc = b2v[cc];
#pragma unroll
    for (int q4 = 0; q4 < H / 8; ++q4) {
      acc = dot2(w[q4].x, h1[4 * q4], acc);
      acc = dot2(w[q4].y, h1[4 * q4 + 1], acc);
      acc = dot2(w[q4].z, h1[4 * q4 + 2], acc);
      acc = dot2(w[q4].w, h1[4 * q4 + 3], acc);
    }
    // relu; a lane past the set's end contributes 0 (every h2 >= 0)
    r[cc] = live ? fmaxf(acc, 0.0f) : 0.0f;
  }
  // halving exchange: after the steps with partner distance 32, 16, 8, 4,
  // lane l holds the maximum over its group of the channel
  // 8 b5 + 4 b4 + 2 b3 + b2 (b_k: bit k of l), then 2 and 1 finish it
#pragma unroll
  for (int step = 0, half = kPoolChannels / 2, d = 32; step < 4; ++step, half >>= 1, d >>= 1) {
    const bool hi = (lane & d) != 0;
#pragma unroll
    for (int i = 0; i < half; ++i) {
      const float send = hi ? r[i] : r[i + half];
      const float keep = hi ? r[i + half] : r[i];
      r[i] = fmaxf(keep, __shfl_xor(send, d));
    }
  }
  float mx = fmaxf(r[0], __shfl_xor(r[0], 2));
  mx = fmaxf(mx, __shfl_xor(mx, 1));
  if ((lane & 3) == 0) {
    const int ch = ((lane >> 5) & 1) * 8 + ((lane >> 4) & 1) * 4 + ((lane >> 3) & 1) * 2 +
                   ((lane >> 2) & 1);
    s_max[c0 + ch] = mx;
  }
  __syncthreads();
  // clear the sign bit: a -0 from the ReLU orders as +0
  if (t < H) atomicMax(&g[(size_t)b * H + t], __float_as_uint(s_max[t]) & 0x7FFFFFFFu);
}

// Head and slope of set b: out = W4 relu(W3 g + b3) + b4 (as k_net_forward,
// the same products in the same order), theta = tan(atan2(out1, out0) / 2)
// sy / sx. The block first copies W3 (transposed, so that the lanes of a
// wavefront read distinct banks) and W4 to LDS with coalesced loads.
__global__ __launch_bounds__(NT) void k_net_head(const float* __restrict__ P,
                                                 const unsigned* __restrict__ g,
                                                 const double* __restrict__ scale,
                                                 float* __restrict__ out,
                                                 double* __restrict__ theta) {
  __shared__ float s_w3t[H * H], s_w4[2 * H];
  __shared__ float s_g[H], s_h3[H], s_out[2];
  const int b = blockIdx.x, t = threadIdx.x;
  for (int e = t; e < H * H; e += NT) s_w3t[(e % H) * H + e / H] = bf16_round(P[OFF_W3 + e]);
  for (int e = t; e < 2 * H; e += NT) s_w4[e] = bf16_round(P[OFF_W4 + e]);
  if (t < H) s_g[t] = __uint_as_float(g[(size_t)b * H + t]);
  __syncthreads();
  if (t < H) {
    float a = P[OFF_B3 + t];
    for (int k = 0; k < H; ++k) a = fmaf(s_w3t[k * H + t], s_g[k], a);
    s_h3[t] = fmaxf(a, 0.0f);
  }
  __syncthreads();
  if (t < 2) {
    float a2 = P[OFF_B4 + t];
    for (int k = 0; k < H; ++k) a2 = fmaf(s_w4[t * H + k], s_h3[k], a2);
    s_out[t] = a2;
    if (out) out[2 * b + t] = a2;
  }
  __syncthreads();
  if (t == 0) {
    const double phi = 0.5 * atan2((double)s_out[1], (double)s_out[0]);
    theta[b] = tan(phi) * scale[4 * b + 3] / scale[4 * b + 2];
  }
}

// Gradient of the mean loss 0.5 ||out - target||^2 / B for each set, written
// per set (B x N_PARAMS) so that the sum over sets has a fixed order.
__global__ __launch_bounds__(NT) void k_net_backward(const float* __restrict__ P,
                                                     const float2* __restrict__ pts,
                                                     const int64_t* __restrict__ off, int B,
                                                     const float* __restrict__ target,
                                                     const float* __restrict__ out,
                                                     const float* __restrict__ g_in,
                                                     float* __restrict__ grad_set,
                                                     float* __restrict__ loss_set) {
  __shared__ PointMLP s;
  __shared__ float s_g[H], s_z3[H], s_dz3[H], s_dg[H], s_dz2[H];
  __shared__ float s_dout[2];
  __shared__ int s_arg[NT / 64][H];
  __shared__ int s_argf[H];
  load_point_mlp(P, s);
  const int b = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t o = off[b], n = off[b + 1] - off[b];
  float* G = grad_set + (size_t)b * N_PARAMS;
  if (t < H) s_g[t] = g_in[(size_t)b * H + t];
  if (t < 2) {
    const float d = out[2 * b + t] - target[2 * b + t];
    s_dout[t] = d / (float)B;
  }
  __syncthreads();
  if (t == 0) loss_set[b] = 0.5f * (s_dout[0] * s_dout[0] + s_dout[1] * s_dout[1]) * (float)B;
  // head
  if (t < H) {
    float a = P[OFF_B3 + t];
    for (int k = 0; k < H; ++k) a = fmaf(bf16_round(P[OFF_W3 + t * H + k]), s_g[k], a);
    s_z3[t] = a;
  }
  __syncthreads();
  if (t < H) {
    const float h3 = fmaxf(s_z3[t], 0.0f);
    const float w40 = bf16_round(P[OFF_W4 + t]), w41 = bf16_round(P[OFF_W4 + H + t]);
    G[OFF_W4 + t] = s_dout[0] * h3;
    G[OFF_W4 + H + t] = s_dout[1] * h3;
    const float dh3 = w40 * s_dout[0] + w41 * s_dout[1];
    s_dz3[t] = s_z3[t] > 0.0f ? dh3 : 0.0f;
  }
  if (t < 2) G[OFF_B4 + t] = s_dout[t];
  __syncthreads();
  if (t < H) {
    G[OFF_B3 + t] = s_dz3[t];
    for (int k = 0; k < H; ++k) G[OFF_W3 + t * H + k] = s_dz3[t] * s_g[k];
    float dg = 0.0f;
    for (int c = 0; c < H; ++c) dg = fmaf(bf16_round(P[OFF_W3 + c * H + t]), s_dz3[c], dg);
    s_dg[t] = dg;
  }
  // first point attaining each channel's maximum (same arithmetic as forward)
  int first[H];
#pragma unroll
  for (int c = 0; c < H; ++c) first[c] = INT_MAX;
  for (int64_t k = t; k < n; k += NT) {
    asm volatile("" ::: "memory");
    const float2 p = pts[o + k];
    unsigned h1[H / 2];
    layer1(s, p.x, p.y, h1);
#pragma unroll
    for (int c = 0; c < H; ++c)
      if (first[c] == INT_MAX && fmaxf(layer2(s, h1, c), 0.0f) == s_g[c]) first[c] = (int)k;
  }
#pragma unroll
  for (int c = 0; c < H; ++c) {
    const int m = wave_min_i(first[c]);
    if (lane == 0) s_arg[wv][c] = m;
  }
  __syncthreads();
  if (t < H) {
    int m = s_arg[0][t];
    for (int w = 1; w < NT / 64; ++w) m = min(m, s_arg[w][t]);
    if (m == INT_MAX) m = 0;  // empty set: nothing to route (dz2 is then 0 or n is 0)
    s_argf[t] = m;
    // dz2 at that point; zero if the channel was inactive everywhere
    unsigned h1[H / 2];
    float z2 = 0.0f;
    if (n > 0) {
      const float2 p = pts[o + m];
      layer1(s, p.x, p.y, h1);
      z2 = layer2(s, h1, t);
    } else {
      for (int k = 0; k < H / 2; ++k) h1[k] = 0u;
    }
    s_dz2[t] = z2 > 0.0f ? s_dg[t] : 0.0f;
    G[OFF_B2 + t] = s_dz2[t];
    // dW2 row t = dz2_t * bf16(h1(arg_t))
    for (int k = 0; k < H / 2; ++k) {
      G[OFF_W2 + t * H + 2 * k] = s_dz2[t] * __uint_as_float(h1[k] << 16);
      G[OFF_W2 + t * H + 2 * k + 1] = s_dz2[t] * __uint_as_float(h1[k] & 0xFFFF0000u);
    }
  }
  __syncthreads();
  // layer 1: thread t = hidden unit k; sum over channels c of W2[c][k] dz2_c at point arg_c
  if (t < H) {
    const int k = t;
    const float w1x = s.w1[2 * k], w1y = s.w1[2 * k + 1], b1 = s.b1[k];
    float gw0 = 0.0f, gw1 = 0.0f, gb = 0.0f;
    for (int c = 0; c < H; ++c) {
      const float dz2 = s_dz2[c];
      if (dz2 == 0.0f) continue;
      const float2 p = pts[o + s_argf[c]];
      const float z1 = fmaf(w1y, p.y, fmaf(w1x, p.x, b1));
      if (!(z1 > 0.0f)) continue;
      const unsigned wp = s.w2[c * (H / 2) + k / 2];
      const float w2 = __uint_as_float((k & 1) ? (wp & 0xFFFF0000u) : (wp << 16));
      const float d = w2 * dz2;
      gw0 = fmaf(d, p.x, gw0);
      gw1 = fmaf(d, p.y, gw1);
      gb += d;
    }
    G[OFF_W1 + 2 * k] = gw0;
    G[OFF_W1 + 2 * k + 1] = gw1;
    G[OFF_B1 + k] = gb;
  }
}

// Sum of the per-set gradients, in set order.
__global__ __launch_bounds__(NT) void k_net_reduce(const float* __restrict__ grad_set, int B,
                                                   float* __restrict__ grad) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= N_PARAMS) return;
  float a = 0.0f;
  for (int b = 0; b < B; ++b) a += grad_set[(size_t)b * N_PARAMS + i];
  grad[i] = a;
}

// Adam (Kingma & Ba), bias-corrected, on the FP32 masters.
__global__ __launch_bounds__(NT) void k_net_adam(float* __restrict__ P, float* __restrict__ m,
                                                 float* __restrict__ v,
                                                 const float* __restrict__ grad, float lr,
                                                 float beta1, float beta2, float eps, float c1,
                                                 float c2) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i >= N_PARAMS) return;
  const float gr = grad[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * gr;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gr * gr;
  m[i] = mi;
  v[i] = vi;
  P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Slope in the original frame from (cos 2phi, sin 2phi) in the normalised one.
__global__ void k_net_slopes(const float* __restrict__ out, const double* __restrict__ scale,
                             int B, double* __restrict__ theta) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double phi = 0.5 * atan2((double)out[2 * b + 1], (double)out[2 * b]);
  theta[b] = tan(phi) * scale[4 * b + 3] / scale[4 * b + 2];
}

}  // namespace

namespace lms_host {

size_t net_infer_bytes(int64_t B) {
  return ((size_t)B * 4 * sizeof(double) + 255 & ~size_t(255)) +
         ((size_t)B * H * sizeof(unsigned) + 255 & ~size_t(255)) + WPK_WORDS * sizeof(unsigned);
}

lms_status net_infer_enqueue(const float* d_params, const double* d_xy, const int64_t* d_offsets,
                             int64_t B, int64_t max_set, int max_points, double* d_theta,
                             float* d_out, void* scratch, hipStream_t s) {
  // without offsets: one set of max_set points
  const int64_t n_single = d_offsets ? 0 : max_set;
  double* scale = (double*)scratch;
  unsigned* g = (unsigned*)((char*)scratch + ((B * 4 * sizeof(double) + 255) & ~size_t(255)));
  unsigned* wpk = (unsigned*)((char*)g + ((B * H * sizeof(unsigned) + 255) & ~size_t(255)));
  hipLaunchKernelGGL(k_net_frame, dim3((unsigned)B), dim3(NTF), 0, s, d_params, d_xy, d_offsets,
                     n_single, scale, g, wpk);
  const int64_t m = std::min<int64_t>(max_set, max_points);
  const unsigned gx = (unsigned)std::max<int64_t>(1, (m + kPoolPoints - 1) / kPoolPoints);
  hipLaunchKernelGGL(k_net_pool, dim3(gx, (unsigned)B), dim3(NT), 0, s, wpk, d_xy, d_offsets,
                     n_single, max_points, scale, g);
  hipLaunchKernelGGL(k_net_head, dim3((unsigned)B), dim3(NT), 0, s, d_params, g, scale, d_out,
                     d_theta);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LMS_ERR_DEVICE, std::string("net launch: ") + hipGetErrorString(e));
  return LMS_OK;
}

}  // namespace lms_host

namespace {

lms_status check(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LMS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return LMS_OK;
}

}  // namespace

extern "C" {

lms_status lms_net_prepare(const double* d_xy, const int64_t* d_offsets, int64_t B, float* d_pts,
                           double* d_scale, void* stream) {
  lms_host::clear_error();
  if (!d_xy || !d_offsets || !d_pts || !d_scale || B < 1 || B > INT_MAX)
    return fail(LMS_ERR_ARG, "bad arguments");
  hipLaunchKernelGGL(k_net_prepare, dim3((unsigned)B), dim3(NT), 0, (hipStream_t)stream, d_xy,
                     d_offsets, (float2*)d_pts, d_scale);
  return check("k_net_prepare");
}

lms_status lms_net_forward(const float* d_params, const float* d_pts, const int64_t* d_offsets,
                           int64_t B, float* d_out, float* d_g, void* stream) {
  lms_host::clear_error();
  if (!d_params || !d_pts || !d_offsets || !d_out || B < 1 || B > INT_MAX)
    return fail(LMS_ERR_ARG, "bad arguments");
  hipLaunchKernelGGL(k_net_forward, dim3((unsigned)B), dim3(NT), 0, (hipStream_t)stream, d_params,
                     (const float2*)d_pts, d_offsets, d_out, d_g);
  return check("k_net_forward");
}

lms_status lms_net_backward(const float* d_params, const float* d_pts, const int64_t* d_offsets,
                            int64_t B, const float* d_target, const float* d_out,
                            const float* d_g, float* d_grad_set, float* d_grad, float* d_loss,
                            void* stream) {
  lms_host::clear_error();
  if (!d_params || !d_pts || !d_offsets || !d_target || !d_out || !d_g || !d_grad_set ||
      !d_grad || !d_loss || B < 1 || B > INT_MAX)
    return fail(LMS_ERR_ARG, "bad arguments");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_net_backward, dim3((unsigned)B), dim3(NT), 0, s, d_params,
                     (const float2*)d_pts, d_offsets, (int)B, d_target, d_out, d_g, d_grad_set,
                     d_loss);
  hipLaunchKernelGGL(k_net_reduce, dim3((N_PARAMS + NT - 1) / NT), dim3(NT), 0, s, d_grad_set,
                     (int)B, d_grad);
  return check("k_net_backward");
}

lms_status lms_net_adam(float* d_params, float* d_m, float* d_v, const float* d_grad, int64_t step,
                        float lr, float beta1, float beta2, float eps, void* stream) {
  lms_host::clear_error();
  if (!d_params || !d_m || !d_v || !d_grad || step < 1) return fail(LMS_ERR_ARG, "bad arguments");
  const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_net_adam, dim3((N_PARAMS + NT - 1) / NT), dim3(NT), 0, (hipStream_t)stream,
                     d_params, d_m, d_v, d_grad, lr, beta1, beta2, eps, c1, c2);
  return check("k_net_adam");
}

lms_status lms_net_infer(const float* d_params, const double* d_xy, const int64_t* d_offsets,
                         int64_t B, int64_t max_set, int32_t max_points, double* d_theta,
                         float* d_out, void* stream) {
  lms_host::clear_error();
  if (!d_params || !d_xy || !d_offsets || !d_theta || B < 1 || B > (1 << 24) || max_set < 1 ||
      max_points < 1)
    return fail(LMS_ERR_ARG, "bad arguments");
  char* ws = nullptr;
  const lms_status st = lms_host::get_workspace(6, stream, lms_host::net_infer_bytes(B), &ws);
  if (st != LMS_OK) return st;
  return lms_host::net_infer_enqueue(d_params, d_xy, d_offsets, B, max_set, max_points, d_theta,
                                     d_out, ws, (hipStream_t)stream);
}

lms_status lms_net_slopes(const float* d_out, const double* d_scale, int64_t B, double* d_theta,
                          void* stream) {
  lms_host::clear_error();
  if (!d_out || !d_scale || !d_theta || B < 1 || B > INT_MAX) return fail(LMS_ERR_ARG, "bad arguments");
  hipLaunchKernelGGL(k_net_slopes, dim3((unsigned)((B + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, d_out, d_scale, (int)B, d_theta);
  return check("k_net_slopes");
}

}  // extern "C"
