// Device helpers shared by the kernel translation units.
#pragma once
#include <type_traits>

#include "pty_common.hpp"
#include "pty_fft.hpp"

namespace pty {

// Launch geometry of the row and column passes for window size N: each block
// holds LINES lines (rows or columns) of T threads, BS = LINES * T threads.
template <int N>
struct Geo {
  static constexpr int R = FftShape<N>::R, T = FftShape<N>::T;
  static constexpr int LINES = (256 / T < N) ? 256 / T : N;
  static constexpr int BS = LINES * T;
  static constexpr int W = LineLds<N>::words;
};

// Bilinear read of the object at patch pixel (u, v) of a patch at p
// ((S_j O)[u, v]).  The second tap is clamped to the object; it then carries
// zero weight, since valid patches only reach past the edge at integer
// positions.
__device__ __forceinline__ float2 obj_bilinear(const float2* __restrict__ o, int h, int w,
                                               const PosInfo& p, int u, int v) {
  const int r0 = p.iy + u, c0 = p.ix + v;
  const int r1 = min(r0 + 1, h - 1), c1 = min(c0 + 1, w - 1);
  const float2 a = o[(size_t)r0 * w + c0], b = o[(size_t)r0 * w + c1];
  const float2 c = o[(size_t)r1 * w + c0], d = o[(size_t)r1 * w + c1];
  const float wx1 = p.fx, wx0 = 1.f - p.fx, wy1 = p.fy, wy0 = 1.f - p.fy;
  return make_float2(wy0 * (wx0 * a.x + wx1 * b.x) + wy1 * (wx0 * c.x + wx1 * d.x),
                     wy0 * (wx0 * a.y + wx1 * b.y) + wy1 * (wx0 * c.y + wx1 * d.y));
}

// Derivatives of the bilinear patch with respect to y_j and x_j at fixed
// floor (dw_0/df = -1, dw_1/df = +1); pixels past the object edge read as 0.
__device__ __forceinline__ void obj_bilinear_grad(const float2* __restrict__ o, int h, int w,
                                                  const PosInfo& p, int u, int v, float2& dy,
                                                  float2& dx) {
  const int r0 = p.iy + u, c0 = p.ix + v, r1 = r0 + 1, c1 = c0 + 1;
  const float2 z = make_float2(0.f, 0.f);
  const float2 a = o[(size_t)r0 * w + c0];
  const float2 b = c1 < w ? o[(size_t)r0 * w + c1] : z;
  const float2 c = r1 < h ? o[(size_t)r1 * w + c0] : z;
  const float2 d = (r1 < h && c1 < w) ? o[(size_t)r1 * w + c1] : z;
  const float wx1 = p.fx, wx0 = 1.f - p.fx, wy1 = p.fy, wy0 = 1.f - p.fy;
  dy = make_float2(wx0 * (c.x - a.x) + wx1 * (d.x - b.x), wx0 * (c.y - a.y) + wx1 * (d.y - b.y));
  dx = make_float2(wy0 * (b.x - a.x) + wy1 * (d.x - c.x), wy0 * (b.y - a.y) + wy1 * (d.y - c.y));
}

// Deterministic block sum of doubles (wave64 shuffles, then wave order);
// the result is valid in thread 0.  `sh` holds BS / 64 doubles.
template <int BS>
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) r += sh[i];
  }
  return r;
}

// Block max of non-negative floats; the result is valid in every thread.
template <int BS>
__device__ __forceinline__ float block_max_all(float v, float* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  float r = 0.f;
#pragma unroll
  for (int i = 0; i < BS / 64; ++i) r = fmaxf(r, sh[i]);
  __syncthreads();
  return r;
}

template <int N>
__device__ __forceinline__ void load_twiddles(float2* tw_s, const float2* __restrict__ tw) {
  for (int i = threadIdx.x; i < N; i += blockDim.x) tw_s[i] = tw[i];
  __syncthreads();
}

template <int V>
using ic = std::integral_constant<int, V>;

// Calls f(ic<N>, ic<K>) for the runtime window size n and mode count k.
template <int N, typename F>
inline void dispatch_k(int k, F&& f) {
  switch (k) {
    case 1: f(ic<N>{}, ic<1>{}); break;
    case 2: f(ic<N>{}, ic<2>{}); break;
    case 3: f(ic<N>{}, ic<3>{}); break;
    case 4: f(ic<N>{}, ic<4>{}); break;
    default: throw std::invalid_argument("unsupported number of probe modes");
  }
}
template <typename F>
inline void dispatch_nk(int n, int k, F&& f) {
  switch (n) {
    case 32: dispatch_k<32>(k, f); break;
    case 64: dispatch_k<64>(k, f); break;
    case 128: dispatch_k<128>(k, f); break;
    case 256: dispatch_k<256>(k, f); break;
    case 512:   // 512 x 512 windows: at most 2 modes (register budget of the column pass)
      if (k == 1)
        f(ic<512>{}, ic<1>{});
      else if (k == 2)
        f(ic<512>{}, ic<2>{});
      else
        throw std::invalid_argument("512 x 512 windows take at most 2 probe modes");
      break;
    default: throw std::invalid_argument("unsupported window size");
  }
}
template <typename F>
inline void dispatch_n(int n, F&& f) {
  switch (n) {
    case 32: f(ic<32>{}); break;
    case 64: f(ic<64>{}); break;
    case 128: f(ic<128>{}); break;
    case 256: f(ic<256>{}); break;
    case 512: f(ic<512>{}); break;
    default: throw std::invalid_argument("unsupported window size");
  }
}

}  // namespace pty
