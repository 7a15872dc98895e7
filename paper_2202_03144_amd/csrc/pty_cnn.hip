// Learned initialiser: a small U-Net on bf16 MFMA (gfx950), trained on the GPU.
//
// Architecture (NHWC activations, 3 x 3 convolutions with zero padding 1,
// 2 x 2 average pooling, 2x nearest upsampling, skips concatenated after the
// upsampled channels):
//   L0 conv 2->32 @128 relu, pool; L1 32->32 @64 relu (e1), pool;
//   L2 32->64 @32 relu (e2), pool; L3 64->128 @16 relu (e3), pool;
//   L4 128->256 @8 relu; L5 256->256 @8 relu, up, concat e3;
//   L6 384->128 @16 relu, up, concat e2; L7 192->64 @32 relu, up, concat e1;
//   L8 96->32 @64 relu; L9 32->2 @64 linear (amplitude, phase).
// Input: a real-space estimate of one window's object patch, 128 x 128 x 2
// (real and imaginary part; the pattern's moduli with the known probe's
// far-field phase, transformed back and divided by the probe, central half
// upsampled 2x); output: the central 64 x 64 object patch.  Weights W[cout][ky][kx][cin] (bf16 copies of
// float32 masters), biases float32; loss = mean squared error; Adam.
//
// Convolutions with cin, cout multiples of 32 are implicit GEMMs on
// v_mfma_f32_16x16x32_bf16 (pixels x output channels, reduction over
// taps x input channels, float32 accumulation) that run from LDS-staged halo
// tiles (18 x 18 on 16-multiple images, four 10 x 10 ones for 8 x 8 images);
// the input gradient is the same kernel with transposed, spatially flipped
// weights; the weight gradient is an
// MFMA GEMM over pixels with split-K partials summed in a fixed order.  The
// 2-channel output layer runs on the halo kernel over weights zero-padded to
// 16 channels; the 2-channel input layer is a direct kernel.
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <random>
#include <string>
#include <vector>

#include "ptymi.h"
#include "pty_common.hpp"
#include "pty_kernels.hpp"

namespace pty {
namespace {

using bf16 = __bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

__device__ __forceinline__ float tof(bf16 v) { return static_cast<float>(v); }
__device__ __forceinline__ bf16 tob(float v) { return static_cast<bf16>(v); }  // round to nearest even

// 8 consecutive channels (16 bytes; every channel stride and offset here is a
// multiple of 8)
__device__ __forceinline__ void ld8(const bf16* p, float (&v)[8]) {
  const bf16x8_t x = *reinterpret_cast<const bf16x8_t*>(p);
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = static_cast<float>(x[i]);
}
__device__ __forceinline__ void st8(bf16* p, const float (&v)[8]) {
  bf16x8_t x;
#pragma unroll
  for (int i = 0; i < 8; ++i) x[i] = static_cast<bf16>(v[i]);
  *reinterpret_cast<bf16x8_t*>(p) = x;
}

// A strided NHWC view: element (b, y, x, c) at ((b*H + y)*W + x)*cs + co + c.
struct View {
  bf16* p;
  int cs, co;
  __device__ __forceinline__ bf16* at(size_t m) const { return p + m * cs + co; }
};

// ---------------------------------------------------------------------------
// Convolutions whose channel counts are multiples of 32 are implicit GEMMs on
// MFMA: out[m][n] = act(bias[n] + sum_{tap, c} in[m + tap][c] * w[n][tap][c]),
// m = (b, y, x) pixels of an S x S image, n output channels, reduction over
// taps x input channels, float32 accumulation.
// ---------------------------------------------------------------------------
// LDS-tiled implicit GEMM.  Block = 4 wavefronts on a BM-pixel x BN-channel
// tile, each wavefront on 64 pixels x 32 channels (4 x 2 MFMA tiles); the
// reduction runs over (tap, 32-channel block) steps; each step's A (BM x 32)
// and B (BN x 32) bf16 tiles are fetched from global memory into registers
// while the MFMAs of the previous step run from LDS (two LDS buffers).  The
// epilogue goes through LDS so that every pixel's channels are written as
// 16-byte vectors.
template <int BM, int BN, bool RELU, bool BIAS>
__global__ __launch_bounds__(256) void k_conv_gemm(View in, const bf16* __restrict__ w,
                                                   const float* __restrict__ bias, View out, int nb, int S,
                                                   int cin, int cout, View lo, int clo) {
  constexpr int WN = BN / 32, WM = 4 / WN;
  static_assert(WM * 64 == BM, "wavefront tiles must cover the block tile");
  constexpr int MT = 4, NT = 2;
  constexpr int LD = 40;                                // padded rows (80 bytes)
  constexpr int AP = BM / 64;                           // 16-byte A pieces per thread per step
  __shared__ __align__(16) bf16 sa[2][BM * LD];
  __shared__ __align__(16) bf16 sb[2][BN * LD];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv / WN, wn = wv % WN;
  const int row = lane & 15, grp = lane >> 4;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int mtot = nb * S * S;
  // loader roles: A piece r of this thread = pixel (tid + 256 r) / 4, channels
  // ((tid + 256 r) % 4) * 8 .. +8; B: output channel tid / 4, channels (tid % 4) * 8
  // .. +8 (threads below BN * 4)
  int ab[AP], ay[AP], ax[AP];
  bool aok[AP];
  const int ac = (tid & 3) * 8;
#pragma unroll
  for (int r = 0; r < AP; ++r) {
    const int am = m0 + (tid + 256 * r) / 4;
    aok[r] = am < mtot;
    ab[r] = am / (S * S);
    ay[r] = (am / S) % S;
    ax[r] = am % S;
  }
  const int bnr = tid >> 2;
  const bool b_on = tid < BN * 4;
  const int cb = cin / 32, steps = 9 * cb;
  bf16x8_t ra[AP], rb;
  // Input channels below clo (inference only) come from the half-resolution
  // tensor `lo`, read at (y / 2, x / 2): the nearest 2x upsampling of the
  // decoder, folded into the load instead of being written out first.
  const int Sl = S >> 1;
  auto fetch = [&](int st) {
    const int tap = st / cb, c0 = (st % cb) * 32;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const bool from_lo = c0 < clo;
#pragma unroll
    for (int r = 0; r < AP; ++r) {
      const int yy = ay[r] + dy, xx = ax[r] + dx;
      if (aok[r] && (unsigned)yy < (unsigned)S && (unsigned)xx < (unsigned)S) {
        if (from_lo)
          ra[r] = *reinterpret_cast<const bf16x8_t*>(lo.p + ((size_t)(ab[r] * Sl + (yy >> 1)) * Sl + (xx >> 1)) * lo.cs +
                                                     lo.co + c0 + ac);
        else
          ra[r] = *reinterpret_cast<const bf16x8_t*>(in.p + ((size_t)(ab[r] * S + yy) * S + xx) * in.cs + in.co + c0 + ac);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) ra[r][e] = static_cast<bf16>(0.0f);
      }
    }
    if (b_on) rb = *reinterpret_cast<const bf16x8_t*>(w + ((size_t)(n0 + bnr) * 9 + tap) * cin + c0 + ac);
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int r = 0; r < AP; ++r)
      *reinterpret_cast<bf16x8_t*>(&sa[buf][((tid + 256 * r) >> 2) * LD + ac]) = ra[r];
    if (b_on) *reinterpret_cast<bf16x8_t*>(&sb[buf][bnr * LD + ac]) = rb;
  };
  f32x4_t acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[i][t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  fetch(0);
  stash(0);
  __syncthreads();
  for (int st = 0; st < steps; ++st) {
    const int buf = st & 1;
    if (st + 1 < steps) fetch(st + 1);
    bf16x8_t a[MT], b[NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
      a[i] = *reinterpret_cast<const bf16x8_t*>(&sa[buf][(wm * 64 + i * 16 + row) * LD + grp * 8]);
#pragma unroll
    for (int t = 0; t < NT; ++t)
      b[t] = *reinterpret_cast<const bf16x8_t*>(&sb[buf][(wn * 32 + t * 16 + row) * LD + grp * 8]);
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[t], acc[i][t], 0, 0, 0);
    if (st + 1 < steps) stash(buf ^ 1);
    __syncthreads();
  }
  // epilogue: D[i][j], i = 4 * (lane / 16) + r (pixel), j = lane % 16 (channel),
  // staged as bf16 [pixel][channel] in the A buffers
  bf16* so = &sa[0][0];
  constexpr int LDO = BN + 8;
  static_assert(BM * LDO <= 2 * BM * LD, "epilogue tile must fit");
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int nl = wn * 32 + t * 16 + row;
    const float bv = BIAS ? bias[n0 + nl] : 0.f;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = acc[i][t][r] + bv;
        if (RELU) v = fmaxf(v, 0.f);
        so[(wm * 64 + i * 16 + grp * 4 + r) * LDO + nl] = tob(v);
      }
  }
  __syncthreads();
  for (int e = tid; e < BM * (BN / 8); e += 256) {
    const int pl = e / (BN / 8), g = (e % (BN / 8)) * 8;
    const int m = m0 + pl;
    if (m >= mtot) continue;
    *reinterpret_cast<bf16x8_t*>(out.at(m) + n0 + g) = *reinterpret_cast<const bf16x8_t*>(&so[pl * LDO + g]);
  }
}

// Halo-tiled variant for S x S images, S a multiple of 16, BN = 32 or 64
// output channels per block.  A block owns a 16 x 16 pixel tile of one image;
// per 32-channel input block it stages the 18 x 18 halo tile and the 9 taps'
// weights in LDS once (the next block's are fetched into registers
// meanwhile) and runs the 9 taps from there, so every input value is fetched
// once per channel block instead of once per tap (the GEMM above refetches
// it for each tap from cache).  Wavefront w owns tile rows 4w .. 4w + 3:
// 4 x BN/16 MFMA tiles, one tile row = 16 pixels.  Same lo / clo
// upsampled-input split as the GEMM.  With pool.p set, the block also writes
// the 2 x 2 average pool of its (bf16) output tile (the four values summed
// row by row, then scaled by 1/4), so the encoder needs no pooling pass.
// OUT2 (the 2-channel output layer, BN = 16 over weights zero-padded to 16
// output channels): channels 0 and 1 plus bias are written as float32 pairs
// to y instead.  Q8 (8 x 8 images): the block's 16 x 16 tile holds four
// images as quadrants, image 4 blockIdx.x + q in quadrant q (row-major), each
// with its own zero-padded 10 x 10 halo in a 20 x 20 staging tile; images
// past nb are zero and not written.
template <int BN, bool RELU, bool BIAS, bool OUT2 = false, bool Q8 = false>
__global__ __launch_bounds__(256) void k_conv_halo(View in, const bf16* __restrict__ w,
                                                   const float* __restrict__ bias, View out, int S, int cin,
                                                   View lo, int clo, View pool, float* __restrict__ y = nullptr,
                                                   int nb = 0) {
  static_assert(BN == 16 || BN == 32 || BN == 64, "16, 32 or 64 output channels per block");
  static_assert(!OUT2 || (BN == 16 && BIAS && !RELU), "the output layer: 16 padded channels, bias, linear");
  static_assert(!(Q8 && OUT2), "8 x 8 quadrants are for the hidden layers");
  constexpr int TS = 16, HS = Q8 ? 20 : TS + 2, HP = HS * HS;   // 400 or 324 staged pixels
  constexpr int LD = 40;                              // padded rows (80 bytes)
  constexpr int AQ = (HP * 4 + 255) / 256;            // 16-byte halo pieces per thread
  constexpr int BP = 9 * BN;                          // weight rows: tap * BN + output channel
  constexpr int BQ = (BP * 4 + 255) / 256;            // 16-byte weight pieces per thread
  constexpr int MT = 4, NT = BN / 16;
  __shared__ __align__(16) bf16 smem[(HP + BP) * LD];
  bf16* const sa = smem;                              // halo tile [pixel][channel]
  bf16* const sb = smem + HP * LD;                    // weights [tap * BN + n][channel]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int row = lane & 15, grp = lane >> 4;
  const int tiles = Q8 ? 1 : S / TS;                  // Q8: one tile of four images
  const int bt = blockIdx.x;
  const int b = bt / (tiles * tiles), tyb = (bt / tiles) % tiles, txb = bt % tiles;
  const int y0 = tyb * TS - 1, x0 = txb * TS - 1;     // halo origin in the image
  const int n0 = blockIdx.y * BN;
  const int cb = cin / 32;
  const int ac = (tid & 3) * 8;                       // channel offset of this thread's pieces
  const int Sl = S >> 1;
  bf16x8_t ra[AQ], rb[BQ];
  auto fetch = [&](int c0) {
    const bool from_lo = c0 < clo;
#pragma unroll
    for (int q = 0; q < AQ; ++q) {
      const int hp = (tid + 256 * q) >> 2;
      if constexpr (Q8) {
        // staged pixel (hy, hx) -> quadrant image, pixel (hy % 10 - 1, hx % 10 - 1)
        const int hy = hp / HS, hx = hp % HS;
        const int bq = 4 * bt + (hy / 10) * 2 + hx / 10, ly = hy % 10 - 1, lx = hx % 10 - 1;
        if (hp < HP && bq < nb && (unsigned)ly < 8u && (unsigned)lx < 8u) {
          ra[q] = *reinterpret_cast<const bf16x8_t*>(in.p + ((size_t)(bq * 8 + ly) * 8 + lx) * in.cs + in.co + c0 + ac);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) ra[q][e] = static_cast<bf16>(0.0f);
        }
        continue;
      }
      const int yy = y0 + hp / HS, xx = x0 + hp % HS;
      if (hp < HP && (unsigned)yy < (unsigned)S && (unsigned)xx < (unsigned)S) {
        if (from_lo)
          ra[q] = *reinterpret_cast<const bf16x8_t*>(lo.p + ((size_t)(b * Sl + (yy >> 1)) * Sl + (xx >> 1)) * lo.cs +
                                                     lo.co + c0 + ac);
        else
          ra[q] = *reinterpret_cast<const bf16x8_t*>(in.p + ((size_t)(b * S + yy) * S + xx) * in.cs + in.co + c0 + ac);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) ra[q][e] = static_cast<bf16>(0.0f);
      }
    }
#pragma unroll
    for (int q = 0; q < BQ; ++q) {
      const int e = (tid + 256 * q) >> 2;             // tap * BN + output channel
      const int tap = e / BN, n = e % BN;
      if (e < BP) rb[q] = *reinterpret_cast<const bf16x8_t*>(w + ((size_t)(n0 + n) * 9 + tap) * cin + c0 + ac);
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < AQ; ++q) {
      const int hp = (tid + 256 * q) >> 2;
      if (hp < HP) *reinterpret_cast<bf16x8_t*>(&sa[hp * LD + ac]) = ra[q];
    }
#pragma unroll
    for (int q = 0; q < BQ; ++q) {
      const int e = (tid + 256 * q) >> 2;
      if (e < BP) *reinterpret_cast<bf16x8_t*>(&sb[e * LD + ac]) = rb[q];
    }
  };
  f32x4_t acc[MT][NT];
#pragma unroll
  for (int i = 0; i < MT; ++i)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[i][t] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  fetch(0);
  stash();
  __syncthreads();
  for (int s = 0; s < cb; ++s) {
    if (s + 1 < cb) fetch((s + 1) * 32);
#pragma unroll 1
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap % 3;
      bf16x8_t a[MT], bw[NT];
#pragma unroll
      for (int i = 0; i < MT; ++i) {
        // tile pixel (Y, X) = (4 wv + i, row); Q8: quadrant halo coordinates
        const int Y = wv * 4 + i, X = row;
        const int hy = Q8 ? 10 * (Y >> 3) + (Y & 7) + dy : Y + dy;
        const int hx = Q8 ? 10 * (X >> 3) + (X & 7) + dx : X + dx;
        a[i] = *reinterpret_cast<const bf16x8_t*>(&sa[(hy * HS + hx) * LD + grp * 8]);
      }
#pragma unroll
      for (int t = 0; t < NT; ++t)
        bw[t] = *reinterpret_cast<const bf16x8_t*>(&sb[(tap * BN + t * 16 + row) * LD + grp * 8]);
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bw[t], acc[i][t], 0, 0, 0);
    }
    __syncthreads();
    if (s + 1 < cb) {
      stash();
      __syncthreads();
    }
  }
  if constexpr (OUT2) {
    // D[i][j] as below; lanes j < 2 hold the two real channels
    float* sf = reinterpret_cast<float*>(smem);       // [pixel][2]
    if (row < 2) {
      const float bv = bias[row];
#pragma unroll
      for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) sf[((wv * 4 + i) * TS + grp * 4 + r) * 2 + row] = acc[i][0][r] + bv;
    }
    __syncthreads();
    const size_t m = ((size_t)b * S + tyb * TS + tid / TS) * S + txb * TS + tid % TS;
    reinterpret_cast<float2*>(y)[m] = make_float2(sf[tid * 2], sf[tid * 2 + 1]);
    return;
  }
  // epilogue through LDS: D[i][j], i = 4 * (lane / 16) + r (pixel of tile row
  // 4 wv + tile), j = lane % 16 (channel); every pixel's BN channels leave as
  // 16-byte vectors
  bf16* so = smem;
  constexpr int LDO = BN + 8;
  static_assert(TS * TS * LDO <= (HP + BP) * LD, "epilogue tile must fit");
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int nl = t * 16 + row;
    const float bv = BIAS ? bias[n0 + nl] : 0.f;
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = acc[i][t][r] + bv;
        if (RELU) v = fmaxf(v, 0.f);
        so[((wv * 4 + i) * TS + grp * 4 + r) * LDO + nl] = tob(v);
      }
  }
  __syncthreads();
  constexpr int PV = BN / 8;                          // 16-byte vectors per pixel
#pragma unroll
  for (int q = 0; q < PV; ++q) {
    const int e = tid + 256 * q;
    const int pl = e / PV, g = (e % PV) * 8;
    size_t m;
    if constexpr (Q8) {
      const int Y = pl / TS, X = pl % TS, bq = 4 * bt + (Y >> 3) * 2 + (X >> 3);
      if (bq >= nb) continue;
      m = ((size_t)bq * 8 + (Y & 7)) * 8 + (X & 7);
    } else {
      m = ((size_t)b * S + tyb * TS + pl / TS) * S + txb * TS + pl % TS;
    }
    *reinterpret_cast<bf16x8_t*>(out.at(m) + n0 + g) = *reinterpret_cast<const bf16x8_t*>(&so[pl * LDO + g]);
  }
  if (!Q8 && pool.p) {
    constexpr int PT = TS / 2;                        // pooled tile side
    const int Sp = S / 2;
#pragma unroll
    for (int q = 0; q < PT * PT * PV / 256; ++q) {
      const int e = tid + 256 * q;
      const int pl = e / PV, g = (e % PV) * 8;
      const int py = pl / PT, px = pl % PT;
      float acc8[8] = {0, 0, 0, 0, 0, 0, 0, 0}, v[8];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bf16x8_t x8 = *reinterpret_cast<const bf16x8_t*>(&so[((2 * py + k / 2) * TS + 2 * px + k % 2) * LDO + g]);
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = static_cast<float>(x8[i]);
#pragma unroll
        for (int i = 0; i < 8; ++i) acc8[i] += v[i];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) acc8[i] *= 0.25f;
      const size_t mp = ((size_t)b * Sp + tyb * PT + py) * Sp + txb * PT + px;
      st8(pool.at(mp) + n0 + g, acc8);
    }
  }
}

// Weight gradient on MFMA: part[split][n][tap][c] = sum over the split's pixels
// m of dz[m][n] * in[m + tap][c]; the centre-tap blocks of the first channel
// block also sum dz over the split into bpart[split][n] (the bias gradient).
// Block = 4 wavefronts on a 32 x 32 (n, c) tile of one tap; each wavefront
// owns a 16 x 16 quarter.  Pixel steps of 128 are staged through LDS
// transposed so that every fragment is 16 contiguous bytes; each wavefront
// then runs four MFMAs, one per 32-pixel chunk in pixel order.
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4_t;
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2_t;

__global__ __launch_bounds__(256) void k_wgrad_mfma(View dz, View in, float* __restrict__ part,
                                                    float* __restrict__ bpart, int nb, int S, int cin, int cout,
                                                    int px_per_split) {
  constexpr int PS = 128, LDP = PS + 8;      // pixels per step, padded row
  __shared__ __align__(16) bf16 sd[32][LDP];  // [n][pixel]
  __shared__ __align__(16) bf16 sx[32][LDP];  // [c][pixel]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int cblk = blockIdx.y % (cin / 32), tap = blockIdx.y / (cin / 32);
  const int n0 = blockIdx.x * 32, c0 = cblk * 32;
  const int split = blockIdx.z;
  const int mtot = nb * S * S;
  const int mb = split * px_per_split, me = min(mtot, mb + px_per_split);
  const int dy = tap / 3 - 1, dx = tap % 3 - 1;
  const int wi = (wv >> 1) * 16, wj = (wv & 1) * 16;
  const int row = lane & 15, grp = lane >> 4;
  const bool do_bias = tap == 4 && cblk == 0;
  const int lgS = 31 - __builtin_clz(S);
  f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
  float bacc = 0.f;
  // loader role: the pixel pairs lp, lp + 1 (+ 64 q) of the step, channels
  // lc .. lc + 3; a pair's values of one channel leave as one 4-byte store
  const int lp = (threadIdx.x >> 3) * 2, lc = (threadIdx.x & 7) * 4;
  bf16x4_t zero4;
#pragma unroll
  for (int i = 0; i < 4; ++i) zero4[i] = tob(0.f);
  for (int m = mb; m < me; m += PS) {
    bf16x4_t vd[PS / 32], vx[PS / 32];   // [2 q + e]: pixel lp + e + 64 q
#pragma unroll
    for (int h = 0; h < PS / 32; ++h) {
      vd[h] = zero4;
      vx[h] = zero4;
      const int pm = m + lp + (h & 1) + 64 * (h >> 1);
      if (pm < me) {
        // S is a power of two (64, 32, 16, 8): shifts and masks, no divisions
        const int b = pm >> (2 * lgS), y = (pm >> lgS) & (S - 1), x = pm & (S - 1);
        vd[h] = *reinterpret_cast<const bf16x4_t*>(dz.at(pm) + n0 + lc);
        const int yy = y + dy, xx = x + dx;
        if ((unsigned)yy < (unsigned)S && (unsigned)xx < (unsigned)S)
          vx[h] = *reinterpret_cast<const bf16x4_t*>(in.at((size_t)(b * S + yy) * S + xx) + c0 + lc);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PS / 64; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        bf16x2_t pd, px;
        pd[0] = vd[2 * q][i];
        pd[1] = vd[2 * q + 1][i];
        px[0] = vx[2 * q][i];
        px[1] = vx[2 * q + 1][i];
        *reinterpret_cast<bf16x2_t*>(&sd[lc + i][lp + 64 * q]) = pd;
        *reinterpret_cast<bf16x2_t*>(&sx[lc + i][lp + 64 * q]) = px;
      }
    __syncthreads();
#pragma unroll
    for (int kc = 0; kc < PS / 32; ++kc) {
      const bf16x8_t a = *reinterpret_cast<const bf16x8_t*>(&sd[wi + row][kc * 32 + grp * 8]);
      const bf16x8_t bb = *reinterpret_cast<const bf16x8_t*>(&sx[wj + row][kc * 32 + grp * 8]);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc, 0, 0, 0);
    }
    if (do_bias && threadIdx.x < 32) {
#pragma unroll 8
      for (int q = 0; q < PS; ++q) bacc += tof(sd[threadIdx.x][q]);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int n = n0 + wi + grp * 4 + r, c = c0 + wj + row;
    part[(((size_t)split * cout + n) * 9 + tap) * cin + c] = acc[r];
  }
  if (do_bias && threadIdx.x < 32) bpart[(size_t)split * cout + n0 + threadIdx.x] = bacc;
}

// dst[i] = sum over s of part[s * n + i], in order.  Sixteen partials are
// loaded before they are added (same order), so a thread has sixteen loads in
// flight instead of one: the big layers have few outputs (36 blocks at L1)
// and up to 256 splits.
__global__ void k_sum_splits(const float* __restrict__ part, int splits, size_t n, float* __restrict__ dst) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  constexpr int U = 16;
  float s = 0.f;
  int k = 0;
  for (; k + U <= splits; k += U) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = part[(size_t)(k + u) * n + i];
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u];
  }
  for (; k < splits; ++k) s += part[(size_t)k * n + i];
  dst[i] = s;
}

// split a [n][k + 1] gradient block (k weights, then the bias) into w[n][k] and b[n]
__global__ void k_unpack_wb(const float* __restrict__ src, int k, int cout, float* __restrict__ w,
                            float* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cout * (k + 1)) return;
  const int n = i / (k + 1), r = i % (k + 1);
  if (r < k) w[n * k + r] = src[i];
  else b[n] = src[i];
}

// transposed, spatially flipped weights for the input gradient:
// wt[c][tap][n] = w[n][8 - tap][c]
__global__ void k_wflip(const bf16* __restrict__ w, bf16* __restrict__ wt, int cin, int cout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cin * 9 * cout) return;
  const int n = i % cout, tap = (i / cout) % 9, c = i / (cout * 9);
  wt[i] = w[((size_t)n * 9 + (8 - tap)) * cin + c];
}

// ---------------------------------------------------------------------------
// The 2-channel input and output layers
// ---------------------------------------------------------------------------
// L0 + ReLU + 2 x 2 pooling: one thread per pooled pixel computes the four
// 32-channel pre-activations below it; writes the pooled p0 and, for
// training, the activations a0.
constexpr int kIn = 2;   // input channels (Re, Im of the estimate)
template <bool STORE_A0>
__global__ __launch_bounds__(256) void k_conv_in_pool(const float* __restrict__ x, const bf16* __restrict__ w,
                                                      const float* __restrict__ bias, View a0, View p0, int nb) {
  constexpr int S = 128, P = 64, C = 32, CI = kIn;
  __shared__ float ws[C * 9 * CI], bs[C];
  for (int i = threadIdx.x; i < C * 9 * CI; i += 256) ws[i] = tof(w[i]);
  if (threadIdx.x < C) bs[threadIdx.x] = bias[threadIdx.x];
  __syncthreads();
  const size_t q = blockIdx.x * (size_t)256 + threadIdx.x;
  if (q >= (size_t)nb * P * P) return;
  const int b = (int)(q / (P * P)), py = (int)(q / P) % P, px = (int)(q % P);
  float v[4][4][CI];  // input rows 2py-1 .. 2py+2, cols 2px-1 .. 2px+2
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int yy = 2 * py - 1 + r, xx = 2 * px - 1 + c;
      const bool ok = (unsigned)yy < (unsigned)S && (unsigned)xx < (unsigned)S;
#pragma unroll
      for (int ci = 0; ci < CI; ++ci) v[r][c][ci] = ok ? x[(((size_t)b * S + yy) * S + xx) * CI + ci] : 0.f;
    }
#pragma unroll 1
  for (int g = 0; g < C; g += 8) {
    float pool[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) pool[k] = 0.f;
#pragma unroll
    for (int sy = 0; sy < 2; ++sy)
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) {
        float o[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          float s = bs[g + k];
#pragma unroll
          for (int tap = 0; tap < 9; ++tap)
#pragma unroll
            for (int ci = 0; ci < CI; ++ci) s += v[sy + tap / 3][sx + tap % 3][ci] * ws[((g + k) * 9 + tap) * CI + ci];
          o[k] = fmaxf(s, 0.f);
          pool[k] += o[k];
        }
        if (STORE_A0) st8(a0.at(((size_t)b * S + 2 * py + sy) * S + 2 * px + sx) + g, o);
      }
#pragma unroll
    for (int k = 0; k < 8; ++k) pool[k] *= 0.25f;
    st8(p0.at(q) + g, pool);
  }
}

// L9's weights zero-padded to 16 output channels for the MFMA output layer
__global__ void k_pad_out_w(const bf16* __restrict__ w, bf16* __restrict__ wp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 16 * 9 * 32) wp[i] = i < 2 * 9 * 32 ? w[i] : static_cast<bf16>(0.0f);
}

// L9 input gradient with L8's ReLU: dz8[m][c] = (a8[m][c] > 0) *
// sum_{n, tap} dy[m - tap][n] w[n][tap][c]
__global__ __launch_bounds__(256) void k_conv_out_dgrad(const float* __restrict__ dy, const bf16* __restrict__ w,
                                                        View a8, View dz8, int nb) {
  constexpr int S = 64, C = 32;
  __shared__ float ws[2 * 9 * C];
  for (int i = threadIdx.x; i < 2 * 9 * C; i += 256) ws[i] = tof(w[i]);
  __syncthreads();
  const size_t m = blockIdx.x * (size_t)256 + threadIdx.x;
  if (m >= (size_t)nb * S * S) return;
  const int b = (int)(m / (S * S)), y0 = (int)(m / S) % S, x0 = (int)(m % S);
  float g[2][9];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int yy = y0 - (tap / 3 - 1), xx = x0 - (tap % 3 - 1);
    const bool ok = (unsigned)yy < (unsigned)S && (unsigned)xx < (unsigned)S;
    const size_t o = (((size_t)b * S + yy) * S + xx) * 2;
    g[0][tap] = ok ? dy[o] : 0.f;
    g[1][tap] = ok ? dy[o + 1] : 0.f;
  }
#pragma unroll
  for (int c0 = 0; c0 < C; c0 += 8) {
    float act[8], out[8];
    ld8(a8.at(m) + c0, act);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      float s = 0.f;
#pragma unroll
      for (int tap = 0; tap < 9; ++tap)
        s += g[0][tap] * ws[tap * C + c0 + k] + g[1][tap] * ws[(9 + tap) * C + c0 + k];
      out[k] = act[k] > 0.f ? s : 0.f;
    }
    st8(dz8.at(m) + c0, out);
  }
}

// L0 weight and bias gradient, tiled: each block sums over bands of 4 image
// rows (grid-stride, fixed assignment), dz formed on the fly from the pooled
// gradient and the ReLU of a0: dz[p][n] = (a0[p][n] > 0) gp0[parent(p)][n] / 4.
// part[block][n * 10 + k]: k < 9 tap, k = 9 bias.
constexpr int kInRows = 4;
constexpr int kInK = 9 * kIn + 1;   // weight-gradient entries per output channel (taps x channels, bias)
__global__ __launch_bounds__(256) void k_wgrad_in(const float* __restrict__ x, View a0, View gp0,
                                                  float* __restrict__ part, int nb) {
  constexpr int S = 128, C = 32, R = kInRows, CI = kIn, K = kInK;
  __shared__ float xs[R + 2][S + 2][CI];
  __shared__ float ds[R * S][C + 1];
  __shared__ float red[8][C * K];
  const int n = threadIdx.x & 31, q = threadIdx.x >> 5;
  float acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.f;
  const int bands = nb * (S / R);
  for (int band = blockIdx.x; band < bands; band += gridDim.x) {
    const int b = band / (S / R), y0 = (band % (S / R)) * R;
    __syncthreads();
    for (int i = threadIdx.x; i < (R + 2) * (S + 2) * CI; i += 256) {
      const int ci = i % CI, rc = i / CI;
      const int r = rc / (S + 2), cc = rc % (S + 2);
      const int yy = y0 - 1 + r, xx = cc - 1;
      xs[r][cc][ci] = ((unsigned)yy < (unsigned)S && (unsigned)xx < (unsigned)S)
                          ? x[(((size_t)b * S + yy) * S + xx) * CI + ci] : 0.f;
    }
    for (int i = threadIdx.x; i < R * S * (C / 8); i += 256) {
      const int pix = i / (C / 8), g = (i % (C / 8)) * 8;
      const int yy = y0 + pix / S, xx = pix % S;
      float a[8], d[8];
      ld8(a0.at(((size_t)b * S + yy) * S + xx) + g, a);
      ld8(gp0.at(((size_t)b * (S / 2) + yy / 2) * (S / 2) + xx / 2) + g, d);
#pragma unroll
      for (int k = 0; k < 8; ++k) ds[pix][g + k] = a[k] > 0.f ? 0.25f * d[k] : 0.f;
    }
    __syncthreads();
    for (int pix = q; pix < R * S; pix += 8) {
      const int r = pix / S, cc = pix % S;
      const float d = ds[pix][n];
#pragma unroll
      for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int ci = 0; ci < CI; ++ci) acc[tap * CI + ci] += d * xs[r + tap / 3][cc + tap % 3][ci];
      acc[K - 1] += d;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) red[q][n * K + k] = acc[k];
  __syncthreads();
  for (int i = threadIdx.x; i < C * K; i += 256) {
    float s = 0.f;
#pragma unroll
    for (int qq = 0; qq < 8; ++qq) s += red[qq][i];
    part[(size_t)blockIdx.x * C * K + i] = s;
  }
}

// L9 weight and bias gradient, tiled over bands of 4 rows:
// part[block][n][k], k = tap * 32 + c (weights) and k = 288 (bias).
constexpr int kOutRows = 4;
__global__ __launch_bounds__(256) void k_wgrad_out(View in, const float* __restrict__ dy, float* __restrict__ part,
                                                   int nb) {
  constexpr int S = 64, C = 32, R = kOutRows, K1 = 9 * C + 1;
  __shared__ float as[R + 2][S + 2][C + 1];
  __shared__ float dys[R * S][2];
  __shared__ float red[8][2 * K1];
  const int c = threadIdx.x & 31, q = threadIdx.x >> 5;
  float acc[2][9], bacc[2] = {0.f, 0.f};
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[0][t] = acc[1][t] = 0.f;
  const int bands = nb * (S / R);
  for (int band = blockIdx.x; band < bands; band += gridDim.x) {
    const int b = band / (S / R), y0 = (band % (S / R)) * R;
    __syncthreads();
    for (int i = threadIdx.x; i < (R + 2) * (S + 2) * (C / 8); i += 256) {
      const int cell = i / (C / 8), g = (i % (C / 8)) * 8;
      const int r = cell / (S + 2), cc = cell % (S + 2);
      const int yy = y0 - 1 + r, xx = cc - 1;
      float a[8];
      if ((unsigned)yy < (unsigned)S && (unsigned)xx < (unsigned)S) {
        ld8(in.at(((size_t)b * S + yy) * S + xx) + g, a);
      } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) a[k] = 0.f;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) as[r][cc][g + k] = a[k];
    }
    for (int i = threadIdx.x; i < R * S * 2; i += 256)
      dys[i / 2][i % 2] = dy[(((size_t)b * S + y0) * S) * 2 + i];
    __syncthreads();
    for (int pix = q; pix < R * S; pix += 8) {
      const int r = pix / S, cc = pix % S;
      const float d0 = dys[pix][0], d1 = dys[pix][1];
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const float a = as[r + tap / 3][cc + tap % 3][c];
        acc[0][tap] += d0 * a;
        acc[1][tap] += d1 * a;
      }
      bacc[0] += d0;
      bacc[1] += d1;
    }
  }
  __syncthreads();
#pragma unroll
  for (int n = 0; n < 2; ++n) {
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) red[q][n * K1 + tap * C + c] = acc[n][tap];
    if (c == 0) red[q][n * K1 + 9 * C] = bacc[n];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * K1; i += 256) {
    float s = 0.f;
#pragma unroll
    for (int qq = 0; qq < 8; ++qq) s += red[qq][i];
    part[(size_t)blockIdx.x * 2 * K1 + i] = s;
  }
}

// ---------------------------------------------------------------------------
// Pooling gradients, upsampling, ReLU masks (8 channels per thread), loss, Adam
// (the forward pooling is fused into the convolutions that produce e1 - e3).
// Image sides and channel counts here are powers of two: indices by shifts.
// ---------------------------------------------------------------------------
// dx (S) += dy (S/2) / 4 broadcast, then dx *= (act > 0): the skip gradient
// of an encoder layer plus its pooled path, through its ReLU
__global__ void k_pool_back_relu(View dy, View dx, View act, int nb, int S, int c) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int c8 = c / 8;
  if (i >= (size_t)nb * S * S * c8) return;
  const int lc = __builtin_ctz(c8), ls = __builtin_ctz(S);   // powers of two
  const int g = (int)(i & (c8 - 1)) * 8;
  const size_t m = i >> lc;
  const int b = (int)(m >> (2 * ls)), y = (int)(m >> ls) & (S - 1), x = (int)m & (S - 1), so = S / 2;
  float d[8], v[8], a[8];
  ld8(dy.at(((size_t)b * so + y / 2) * so + x / 2) + g, d);
  ld8(dx.at(m) + g, v);
  ld8(act.at(m) + g, a);
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = a[e] > 0.f ? v[e] + 0.25f * d[e] : 0.f;
  st8(dx.at(m) + g, v);
}

// out (2S) = nearest upsampling of in (S)
__global__ void k_up(View in, View out, int nb, int S, int c) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int so = 2 * S, c8 = c / 8;
  if (i >= (size_t)nb * so * so * c8) return;
  const int lc = __builtin_ctz(c8), ls = __builtin_ctz(so);  // powers of two
  const int g = (int)(i & (c8 - 1)) * 8;
  const size_t m = i >> lc;
  const int b = (int)(m >> (2 * ls)), y = (int)(m >> ls) & (so - 1), x = (int)m & (so - 1);
  *reinterpret_cast<bf16x8_t*>(out.at(m) + g) =
      *reinterpret_cast<const bf16x8_t*>(in.at(((size_t)b * S + y / 2) * S + x / 2) + g);
}

// dz (S) = sum of the 2x2 block of dy (2S), through the ReLU of act (S)
__global__ void k_up_back_relu(View dy, View act, View dz, int nb, int S, int c) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int c8 = c / 8;
  if (i >= (size_t)nb * S * S * c8) return;
  const int lc = __builtin_ctz(c8), ls = __builtin_ctz(S);   // powers of two
  const int g = (int)(i & (c8 - 1)) * 8;
  const size_t m = i >> lc;
  const int b = (int)(m >> (2 * ls)), y = (int)(m >> ls) & (S - 1), x = (int)m & (S - 1), si = 2 * S;
  float s[8] = {0, 0, 0, 0, 0, 0, 0, 0}, v[8], a[8];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    ld8(dy.at(((size_t)b * si + 2 * y + k / 2) * si + 2 * x + k % 2) + g, v);
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] += v[e];
  }
  ld8(act.at(m) + g, a);
#pragma unroll
  for (int e = 0; e < 8; ++e) s[e] = a[e] > 0.f ? s[e] : 0.f;
  st8(dz.at(m) + g, s);
}

// in place: d = d * (act > 0)
__global__ void k_relu_mask(View d, View act, size_t npx, int c) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const int c8 = c / 8;
  if (i >= npx * c8) return;
  const int g = (int)(i % c8) * 8;
  const size_t m = i / c8;
  float v[8], a[8];
  ld8(d.at(m) + g, v);
  ld8(act.at(m) + g, a);
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = a[e] > 0.f ? v[e] : 0.f;
  st8(d.at(m) + g, v);
}

// mean squared error: dy = 2 (y - t) / n, per-block partial loss sums
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t, size_t n,
                                             float* __restrict__ dy, double* __restrict__ part) {
  __shared__ double sh[256];
  const size_t i = blockIdx.x * (size_t)256 + threadIdx.x;
  double s = 0.0;
  if (i < n) {
    const float d = y[i] - t[i];
    dy[i] = 2.f * d / (float)n;
    s = (double)d * d;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// out = scale * sum of n partials (one block, fixed order)
__global__ __launch_bounds__(256) void k_sum_d(const double* part, int n, double scale, double* out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0] * scale;
}

// Adam on float32 masters
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, size_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

__global__ void k_to_bf16(const float* __restrict__ src, bf16* __restrict__ dst, size_t n) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = tob(src[i]);
}

// network input from centred counts: log1p(max(d, 0)) / log1p(photons)

inline unsigned blocks(size_t n, unsigned bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// ---------------------------------------------------------------------------
// Host side: buffers and the layer schedule
// ---------------------------------------------------------------------------
struct Conv {
  int cin, cout, S;
  bool relu;
  size_t woff, boff;  // offsets in the flat parameter vector
};

constexpr int kLayers = 10;
const int kSpec[kLayers][4] = {{kIn, 32, 128, 1},   {32, 32, 64, 1},   {32, 64, 32, 1},  {64, 128, 16, 1},
                               {128, 256, 8, 1},  {256, 256, 8, 1},  {384, 128, 16, 1}, {192, 64, 32, 1},
                               {96, 32, 64, 1},   {32, 2, 64, 0}};

}  // namespace
}  // namespace pty

using namespace pty;

struct pty_cnn {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int max_batch = 0;
  std::string err;
  std::vector<std::pair<void*, size_t>> allocs;
  Conv L[kLayers];
  size_t nparams = 0;
  float* p = nullptr;    // float32 masters
  float* g = nullptr;    // gradient
  float* m1 = nullptr;
  float* m2 = nullptr;
  bf16* wb = nullptr;    // bf16 copy of the whole vector (weights used from it)
  bf16* wt = nullptr;    // transposed-flipped weights scratch
  bf16* w9p = nullptr;   // L9 weights zero-padded to 16 output channels
  float* part = nullptr; size_t part_n = 0;
  double* lpart = nullptr; double* lsum = nullptr;
  int64_t step = 0;
  // activations (bf16 NHWC)
  bf16 *a0, *p0, *cat8, *p1, *cat7, *p2, *cat6, *p3, *a4, *a5, *a6, *a7, *a8;
  // gradients
  bf16 *gp0, *gcat8, *gp1, *gcat7, *gp2, *gcat6, *gp3, *g4, *g5, *g6, *g7, *g8;
  float *y, *gy, *xin;
  float2* planes = nullptr;   // the input's far-field phase and inverse-probe planes

  void* dalloc(size_t bytes) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw NoMemError(std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    allocs.emplace_back(q, bytes);
    return q;
  }
  template <typename T>
  T* alloc(size_t n) { return static_cast<T*>(dalloc(n * sizeof(T))); }
  ~pty_cnn() {
    for (auto& a : allocs) (void)hipFree(a.first);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

thread_local std::string g_cnn_err;

template <typename F>
pty_status cnn_guard(pty_cnn* c, F&& f) {
  try {
    f();
    return PTY_OK;
  } catch (const std::invalid_argument& e) {
    if (c) c->err = e.what();
    g_cnn_err = e.what();
    return PTY_E_INVALID;
  } catch (const NoMemError& e) {
    if (c) c->err = e.what();
    g_cnn_err = e.what();
    return PTY_E_NOMEM;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    g_cnn_err = e.what();
    return PTY_E_DEVICE;
  }
}

View V(bf16* p, int cs, int co = 0) { return View{p, cs, co}; }

// lo / clo: the first clo input channels read from the half-resolution
// tensor lo (a fused nearest 2x upsampling); clo = 0: all from `in`.
void launch_conv(pty_cnn* c, View in, const bf16* w, const float* bias, View out, int nb, int S, int cin, int cout,
                 bool relu, View lo = View{nullptr, 0, 0}, int clo = 0, View pool = View{nullptr, 0, 0}) {
  const int mtot = nb * S * S;
  if (cin % 32 != 0 || cout % 32 != 0) throw std::invalid_argument("conv channels must be multiples of 32");
  if (clo % 32 != 0 || clo > cin || (clo > 0 && (lo.p == nullptr || S % 2 != 0)))
    throw std::invalid_argument("conv: bad upsampled-input split");
  const bool halo = S % 16 == 0 && cout % 32 == 0;
  if (pool.p && !halo) throw std::invalid_argument("conv: a fused pool needs the halo-tiled kernel");
  hipStream_t s = c->stream;
  // 16 x 16 pixel halo tiles wherever the image holds whole tiles; 8 x 8
  // images four to a tile
  if (S == 8 && cout % 64 == 0 && clo == 0 && !pool.p) {
    dim3 grid((nb + 3) / 4, cout / 64);
    if (relu)
      k_conv_halo<64, true, true, false, true><<<grid, 256, 0, s>>>(in, w, bias, out, S, cin, lo, 0, View{}, nullptr, nb);
    else if (bias)
      k_conv_halo<64, false, true, false, true><<<grid, 256, 0, s>>>(in, w, bias, out, S, cin, lo, 0, View{}, nullptr, nb);
    else
      k_conv_halo<64, false, false, false, true><<<grid, 256, 0, s>>>(in, w, bias, out, S, cin, lo, 0, View{}, nullptr,
                                                                      nb);
  } else if (halo && cout % 64 == 0) {
    dim3 grid(nb * (S / 16) * (S / 16), cout / 64);
    if (relu) k_conv_halo<64, true, true><<<grid, 256, 0, s>>>(in, w, bias, out, S, cin, lo, clo, pool);
    else if (bias) k_conv_halo<64, false, true><<<grid, 256, 0, s>>>(in, w, bias, out, S, cin, lo, clo, pool);
    else k_conv_halo<64, false, false><<<grid, 256, 0, s>>>(in, w, bias, out, S, cin, lo, clo, pool);
  } else if (halo) {
    dim3 grid(nb * (S / 16) * (S / 16), cout / 32);
    if (relu) k_conv_halo<32, true, true><<<grid, 256, 0, s>>>(in, w, bias, out, S, cin, lo, clo, pool);
    else if (bias) k_conv_halo<32, false, true><<<grid, 256, 0, s>>>(in, w, bias, out, S, cin, lo, clo, pool);
    else k_conv_halo<32, false, false><<<grid, 256, 0, s>>>(in, w, bias, out, S, cin, lo, clo, pool);
  } else if (cout % 64 == 0) {
    dim3 grid(blocks(mtot, 128), cout / 64);
    if (relu) k_conv_gemm<128, 64, true, true><<<grid, 256, 0, s>>>(in, w, bias, out, nb, S, cin, cout, lo, clo);
    else if (bias) k_conv_gemm<128, 64, false, true><<<grid, 256, 0, s>>>(in, w, bias, out, nb, S, cin, cout, lo, clo);
    else k_conv_gemm<128, 64, false, false><<<grid, 256, 0, s>>>(in, w, bias, out, nb, S, cin, cout, lo, clo);
  } else {
    dim3 grid(blocks(mtot, 256), cout / 32);
    if (relu) k_conv_gemm<256, 32, true, true><<<grid, 256, 0, s>>>(in, w, bias, out, nb, S, cin, cout, lo, clo);
    else if (bias) k_conv_gemm<256, 32, false, true><<<grid, 256, 0, s>>>(in, w, bias, out, nb, S, cin, cout, lo, clo);
    else k_conv_gemm<256, 32, false, false><<<grid, 256, 0, s>>>(in, w, bias, out, nb, S, cin, cout, lo, clo);
  }
  PTY_LAUNCH_CHECK("conv_gemm");
}

// input gradient of an MFMA layer: dx = conv(dz, flipped transposed w)
void launch_dgrad(pty_cnn* c, int li, View dz, View dx, int nb) {
  const Conv& l = c->L[li];
  const int n = l.cin * 9 * l.cout;
  k_wflip<<<blocks(n), 256, 0, c->stream>>>(c->wb + l.woff, c->wt, l.cin, l.cout);
  PTY_LAUNCH_CHECK("wflip");
  launch_conv(c, dz, c->wt, nullptr, dx, nb, l.S, l.cout, l.cin, false);
}

constexpr int kWgradPx = 4096;   // pixels per split of the MFMA weight gradient
constexpr int kSmallGrid = 1024; // blocks of the tiled small-layer weight gradients

// weight + bias gradient of an MFMA layer into c->g
void launch_wgrad(pty_cnn* c, int li, View dz, View in, int nb) {
  const Conv& l = c->L[li];
  const int mtot = nb * l.S * l.S;
  const int splits = (mtot + kWgradPx - 1) / kWgradPx;
  const size_t nw = (size_t)l.cout * 9 * l.cin;
  if ((size_t)splits * (nw + l.cout) > c->part_n) throw std::invalid_argument("wgrad scratch too small");
  float* bpart = c->part + (size_t)splits * nw;
  if ((l.S & (l.S - 1)) != 0) throw std::invalid_argument("wgrad: image side must be a power of two");
  dim3 grid(l.cout / 32, 9 * (l.cin / 32), splits);
  k_wgrad_mfma<<<grid, 256, 0, c->stream>>>(dz, in, c->part, bpart, nb, l.S, l.cin, l.cout, kWgradPx);
  PTY_LAUNCH_CHECK("wgrad_mfma");
  k_sum_splits<<<blocks(nw), 256, 0, c->stream>>>(c->part, splits, nw, c->g + l.woff);
  k_sum_splits<<<blocks(l.cout), 256, 0, c->stream>>>(bpart, splits, l.cout, c->g + l.boff);
  PTY_LAUNCH_CHECK("sum_splits");
}

// Forward pass; with train the L0 activations are kept for the backward pass.
void forward(pty_cnn* c, const float* x, int nb, bool train) {
  auto& L = c->L;
  const bf16* w = c->wb;
  hipStream_t s = c->stream;
  const unsigned gb = blocks((size_t)nb * 64 * 64);
  if (train)
    k_conv_in_pool<true><<<gb, 256, 0, s>>>(x, w + L[0].woff, c->p + L[0].boff, V(c->a0, 32), V(c->p0, 32), nb);
  else
    k_conv_in_pool<false><<<gb, 256, 0, s>>>(x, w + L[0].woff, c->p + L[0].boff, V(c->a0, 32), V(c->p0, 32), nb);
  PTY_LAUNCH_CHECK("conv_in_pool");
  // e1, e2, e3 with their 2 x 2 pools written by the same kernels
  launch_conv(c, V(c->p0, 32), w + L[1].woff, c->p + L[1].boff, V(c->cat8, 96, 64), nb, 64, 32, 32, true, View{}, 0,
              V(c->p1, 32));
  launch_conv(c, V(c->p1, 32), w + L[2].woff, c->p + L[2].boff, V(c->cat7, 192, 128), nb, 32, 32, 64, true, View{}, 0,
              V(c->p2, 64));
  launch_conv(c, V(c->p2, 64), w + L[3].woff, c->p + L[3].boff, V(c->cat6, 384, 256), nb, 16, 64, 128, true, View{},
              0, V(c->p3, 128));
  launch_conv(c, V(c->p3, 128), w + L[4].woff, c->p + L[4].boff, V(c->a4, 256), nb, 8, 128, 256, true);
  launch_conv(c, V(c->a4, 256), w + L[5].woff, c->p + L[5].boff, V(c->a5, 256), nb, 8, 256, 256, true);
  if (train) {
    // the weight gradients read the concatenated inputs, so write them out
    k_up<<<blocks((size_t)nb * 16 * 16 * 32), 256, 0, s>>>(V(c->a5, 256), V(c->cat6, 384, 0), nb, 8, 256);
    launch_conv(c, V(c->cat6, 384), w + L[6].woff, c->p + L[6].boff, V(c->a6, 128), nb, 16, 384, 128, true);
    k_up<<<blocks((size_t)nb * 32 * 32 * 16), 256, 0, s>>>(V(c->a6, 128), V(c->cat7, 192, 0), nb, 16, 128);
    launch_conv(c, V(c->cat7, 192), w + L[7].woff, c->p + L[7].boff, V(c->a7, 64), nb, 32, 192, 64, true);
    k_up<<<blocks((size_t)nb * 64 * 64 * 8), 256, 0, s>>>(V(c->a7, 64), V(c->cat8, 96, 0), nb, 32, 64);
    launch_conv(c, V(c->cat8, 96), w + L[8].woff, c->p + L[8].boff, V(c->a8, 32), nb, 64, 96, 32, true);
  } else {
    // inference: the upsampled channels are read straight from the decoder's
    // half-resolution output inside the convolutions
    launch_conv(c, V(c->cat6, 384), w + L[6].woff, c->p + L[6].boff, V(c->a6, 128), nb, 16, 384, 128, true,
                V(c->a5, 256), 256);
    launch_conv(c, V(c->cat7, 192), w + L[7].woff, c->p + L[7].boff, V(c->a7, 64), nb, 32, 192, 64, true,
                V(c->a6, 128), 128);
    launch_conv(c, V(c->cat8, 96), w + L[8].woff, c->p + L[8].boff, V(c->a8, 32), nb, 64, 96, 32, true,
                V(c->a7, 64), 64);
  }
  // L9 on MFMA over the zero-padded weights
  k_pad_out_w<<<blocks(16 * 9 * 32), 256, 0, s>>>(w + L[9].woff, c->w9p);
  k_conv_halo<16, false, true, true><<<nb * 16, 256, 0, s>>>(V(c->a8, 32), c->w9p, c->p + L[9].boff, View{}, 64, 32,
                                                             View{}, 0, View{}, c->y);
  PTY_LAUNCH_CHECK("cnn_forward");
}

// gradient of the loss into c->g, given dL/dy in c->gy
void backward(pty_cnn* c, const float* x, int nb) {
  auto& L = c->L;
  hipStream_t s = c->stream;
  // L9: weight gradient (tiled, in-block partial sums) and input gradient with L8's ReLU
  {
    const int grid = std::min(nb * (64 / kOutRows), kSmallGrid), np = 2 * (9 * 32 + 1);
    k_wgrad_out<<<grid, 256, 0, s>>>(V(c->a8, 32), c->gy, c->part, nb);
    k_sum_splits<<<blocks(np), 256, 0, s>>>(c->part, grid, np, c->part + (size_t)grid * np);
    k_unpack_wb<<<blocks(np), 256, 0, s>>>(c->part + (size_t)grid * np, 9 * 32, 2, c->g + L[9].woff,
                                           c->g + L[9].boff);
    PTY_LAUNCH_CHECK("wgrad_out");
    k_conv_out_dgrad<<<blocks((size_t)nb * 64 * 64), 256, 0, s>>>(c->gy, c->wb + L[9].woff, V(c->a8, 32),
                                                                 V(c->g8, 32), nb);
    PTY_LAUNCH_CHECK("conv_out_dgrad");
  }
  // L8 (input cat8 = [up(a7) | e1]); g8 holds dz8
  launch_wgrad(c, 8, V(c->g8, 32), V(c->cat8, 96), nb);
  launch_dgrad(c, 8, V(c->g8, 32), V(c->gcat8, 96), nb);
  // upsampled part -> dz7 through L7's ReLU
  k_up_back_relu<<<blocks((size_t)nb * 32 * 32 * 8), 256, 0, s>>>(V(c->gcat8, 96, 0), V(c->a7, 64), V(c->g7, 64), nb,
                                                                 32, 64);
  launch_wgrad(c, 7, V(c->g7, 64), V(c->cat7, 192), nb);
  launch_dgrad(c, 7, V(c->g7, 64), V(c->gcat7, 192), nb);
  k_up_back_relu<<<blocks((size_t)nb * 16 * 16 * 16), 256, 0, s>>>(V(c->gcat7, 192, 0), V(c->a6, 128), V(c->g6, 128),
                                                                  nb, 16, 128);
  launch_wgrad(c, 6, V(c->g6, 128), V(c->cat6, 384), nb);
  launch_dgrad(c, 6, V(c->g6, 128), V(c->gcat6, 384), nb);
  k_up_back_relu<<<blocks((size_t)nb * 8 * 8 * 32), 256, 0, s>>>(V(c->gcat6, 384, 0), V(c->a5, 256), V(c->g5, 256), nb,
                                                                8, 256);
  launch_wgrad(c, 5, V(c->g5, 256), V(c->a4, 256), nb);
  launch_dgrad(c, 5, V(c->g5, 256), V(c->g4, 256), nb);
  k_relu_mask<<<blocks((size_t)nb * 64 * 32), 256, 0, s>>>(V(c->g4, 256), V(c->a4, 256), (size_t)nb * 64, 256);
  launch_wgrad(c, 4, V(c->g4, 256), V(c->p3, 128), nb);
  launch_dgrad(c, 4, V(c->g4, 256), V(c->gp3, 128), nb);
  // e3 gradient = skip slice of gcat6 + pooled path, through L3's ReLU
  k_pool_back_relu<<<blocks((size_t)nb * 16 * 16 * 16), 256, 0, s>>>(V(c->gp3, 128), V(c->gcat6, 384, 256),
                                                                    V(c->cat6, 384, 256), nb, 16, 128);
  launch_wgrad(c, 3, V(c->gcat6, 384, 256), V(c->p2, 64), nb);
  launch_dgrad(c, 3, V(c->gcat6, 384, 256), V(c->gp2, 64), nb);
  k_pool_back_relu<<<blocks((size_t)nb * 32 * 32 * 8), 256, 0, s>>>(V(c->gp2, 64), V(c->gcat7, 192, 128),
                                                                   V(c->cat7, 192, 128), nb, 32, 64);
  launch_wgrad(c, 2, V(c->gcat7, 192, 128), V(c->p1, 32), nb);
  launch_dgrad(c, 2, V(c->gcat7, 192, 128), V(c->gp1, 32), nb);
  k_pool_back_relu<<<blocks((size_t)nb * 64 * 64 * 4), 256, 0, s>>>(V(c->gp1, 32), V(c->gcat8, 96, 64),
                                                                   V(c->cat8, 96, 64), nb, 64, 32);
  launch_wgrad(c, 1, V(c->gcat8, 96, 64), V(c->p0, 32), nb);
  launch_dgrad(c, 1, V(c->gcat8, 96, 64), V(c->gp0, 32), nb);
  // L0: dz formed inside the tiled weight-gradient kernel from gp0 and a0
  {
    const int grid = std::min(nb * (128 / kInRows), kSmallGrid), np = 32 * kInK;
    k_wgrad_in<<<grid, 256, 0, s>>>(x, V(c->a0, 32), V(c->gp0, 32), c->part, nb);
    k_sum_splits<<<blocks(np), 256, 0, s>>>(c->part, grid, np, c->part + (size_t)grid * np);
    PTY_LAUNCH_CHECK("wgrad_in");
    k_unpack_wb<<<blocks(np), 256, 0, s>>>(c->part + (size_t)grid * np, kInK - 1, 32, c->g + L[0].woff,
                                           c->g + L[0].boff);
  }
  PTY_LAUNCH_CHECK("cnn_backward");
}

void refresh_bf16(pty_cnn* c) {
  k_to_bf16<<<blocks(c->nparams), 256, 0, c->stream>>>(c->p, c->wb, c->nparams);
  PTY_LAUNCH_CHECK("to_bf16");
}

double loss_grad(pty_cnn* c, const float* x, const float* t, int nb) {
  const size_t n = (size_t)nb * 64 * 64 * 2;
  forward(c, x, nb, true);
  const unsigned nbk = blocks(n);
  k_mse<<<nbk, 256, 0, c->stream>>>(c->y, t, n, c->gy, c->lpart);
  k_sum_d<<<1, 256, 0, c->stream>>>(c->lpart, nbk, 1.0 / (double)n, c->lsum);
  PTY_LAUNCH_CHECK("mse");
  backward(c, x, nb);
  double loss = 0.0;
  PTY_HIP(hipMemcpyAsync(&loss, c->lsum, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  PTY_HIP(hipStreamSynchronize(c->stream));
  return loss;
}

void check_batch(pty_cnn* c, int nb) {
  if (nb < 1 || nb > c->max_batch) throw std::invalid_argument("batch must be in 1..max_batch");
}

}  // namespace

namespace pty {

float* cnn_input_buffer(pty_cnn* c) { return c->xin; }
int cnn_max_batch(const pty_cnn* c) { return c->max_batch; }
int cnn_device(const pty_cnn* c) { return c->device; }

// Forward pass of nb inputs on stream s; returns the network's output buffer
// (nb x 64 x 64 x 2 float32), valid until the next call on this network.
const float* cnn_forward_batch(pty_cnn* c, const float* x, int nb, hipStream_t s) {
  check_batch(c, nb);
  hipStream_t keep = c->stream;
  c->stream = s;
  try {
    forward(c, x, nb, false);
  } catch (...) {
    c->stream = keep;
    throw;
  }
  c->stream = keep;
  return c->y;
}

}  // namespace pty

extern "C" {

pty_status pty_cnn_create(int32_t device, void* stream, int32_t max_batch, uint64_t seed, pty_cnn** out) {
  return cnn_guard(nullptr, [&] {
    if (!out || max_batch < 1) throw std::invalid_argument("pty_cnn_create: bad argument");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= device || device < 0) {
      (void)hipGetLastError();
      throw DeviceError("pty_cnn_create: no HIP device " + std::to_string(device));
    }
    PTY_HIP(hipSetDevice(device));
    std::unique_ptr<pty_cnn> c(new pty_cnn());
    c->device = device;
    c->max_batch = max_batch;
    if (stream) {
      c->stream = static_cast<hipStream_t>(stream);
    } else {
      PTY_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    size_t off = 0;
    for (int i = 0; i < kLayers; ++i) {
      Conv& l = c->L[i];
      l.cin = kSpec[i][0];
      l.cout = kSpec[i][1];
      l.S = kSpec[i][2];
      l.relu = kSpec[i][3] != 0;
      l.woff = off;
      off += (size_t)l.cout * 9 * l.cin;
      l.boff = off;
      off += l.cout;
    }
    c->nparams = off;
    c->p = c->alloc<float>(off);
    c->g = c->alloc<float>(off);
    c->m1 = c->alloc<float>(off);
    c->m2 = c->alloc<float>(off);
    c->wb = c->alloc<bf16>(off);
    c->wt = c->alloc<bf16>((size_t)384 * 9 * 256);
    c->w9p = c->alloc<bf16>((size_t)16 * 9 * 32);
    // He-normal initialisation (std sqrt(2 / (9 cin))), zero biases
    std::vector<float> hp(off, 0.f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int i = 0; i < kLayers; ++i) {
      const double sd = std::sqrt(2.0 / (9.0 * c->L[i].cin));
      for (size_t k = 0; k < (size_t)c->L[i].cout * 9 * c->L[i].cin; ++k) hp[c->L[i].woff + k] = (float)(nd(rng) * sd);
    }
    PTY_HIP(hipMemcpy(c->p, hp.data(), off * sizeof(float), hipMemcpyHostToDevice));
    PTY_HIP(hipMemset(c->m1, 0, off * sizeof(float)));
    PTY_HIP(hipMemset(c->m2, 0, off * sizeof(float)));
    const size_t B = max_batch;
    auto act = [&](size_t px, int ch) { return c->alloc<bf16>(B * px * ch); };
    c->a0 = act(16384, 32);
    c->p0 = act(4096, 32);
    c->cat8 = act(4096, 96);
    c->p1 = act(1024, 32);
    c->cat7 = act(1024, 192);
    c->p2 = act(256, 64);
    c->cat6 = act(256, 384);
    c->p3 = act(64, 128);
    c->a4 = act(64, 256);
    c->a5 = act(64, 256);
    c->a6 = act(256, 128);
    c->a7 = act(1024, 64);
    c->a8 = act(4096, 32);
    c->gp0 = act(4096, 32);
    c->gcat8 = act(4096, 96);
    c->gp1 = act(1024, 32);
    c->gcat7 = act(1024, 192);
    c->gp2 = act(256, 64);
    c->gcat6 = act(256, 384);
    c->gp3 = act(64, 128);
    c->g4 = act(64, 256);
    c->g5 = act(64, 256);
    c->g6 = act(256, 128);
    c->g7 = act(1024, 64);
    c->g8 = act(4096, 32);
    c->y = c->alloc<float>(B * 4096 * 2);
    c->gy = c->alloc<float>(B * 4096 * 2);
    c->xin = c->alloc<float>(B * 16384 * kIn);
    c->planes = c->alloc<float2>(2 * 16384);
    // split-K scratch: the largest (splits x weights) of any layer, plus unpack room
    size_t need = 0;
    for (int i = 0; i < kLayers; ++i) {
      const size_t mtot = B * c->L[i].S * c->L[i].S;
      const size_t splits = (mtot + 4095) / 4096;
      need = std::max(need, splits * ((size_t)c->L[i].cout * 9 * c->L[i].cin + c->L[i].cout) * 2 + 4096);
    }
    // the tiled L0 / L9 weight gradients: up to kSmallGrid block partials plus their sums
    need = std::max(need, (size_t)(kSmallGrid + 1) * 2 * (9 * 32 + 1));
    need = std::max(need, (size_t)(kSmallGrid + 1) * 32 * kInK);
    c->part = c->alloc<float>(need);
    c->part_n = need;
    c->lpart = c->alloc<double>(blocks(B * 4096 * 2) + 16);
    c->lsum = c->alloc<double>(2);
    refresh_bf16(c.get());
    PTY_HIP(hipStreamSynchronize(c->stream));
    *out = c.release();
  });
}

void pty_cnn_destroy(pty_cnn* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  delete c;
}

pty_status pty_cnn_num_params(const pty_cnn* c, int64_t* n) {
  return cnn_guard(const_cast<pty_cnn*>(c), [&] {
    if (!c || !n) throw std::invalid_argument("pty_cnn_num_params: null argument");
    *n = (int64_t)c->nparams;
  });
}

pty_status pty_cnn_get_params(pty_cnn* c, float* out) {
  return cnn_guard(c, [&] {
    if (!c || !out) throw std::invalid_argument("pty_cnn_get_params: null argument");
    PTY_HIP(hipSetDevice(c->device));
    PTY_HIP(hipMemcpyAsync(out, c->p, c->nparams * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    PTY_HIP(hipStreamSynchronize(c->stream));
  });
}

pty_status pty_cnn_set_params(pty_cnn* c, const float* in) {
  return cnn_guard(c, [&] {
    if (!c || !in) throw std::invalid_argument("pty_cnn_set_params: null argument");
    PTY_HIP(hipSetDevice(c->device));
    PTY_HIP(hipMemcpyAsync(c->p, in, c->nparams * sizeof(float), hipMemcpyHostToDevice, c->stream));
    refresh_bf16(c);
    PTY_HIP(hipStreamSynchronize(c->stream));
  });
}

pty_status pty_cnn_forward(pty_cnn* c, const float* x, int32_t batch, float* y) {
  return cnn_guard(c, [&] {
    if (!c || !x || !y) throw std::invalid_argument("pty_cnn_forward: null argument");
    check_batch(c, batch);
    PTY_HIP(hipSetDevice(c->device));
    forward(c, x, batch, false);
    PTY_HIP(hipMemcpyAsync(y, c->y, sizeof(float) * batch * 4096 * 2, hipMemcpyDeviceToDevice, c->stream));
    PTY_HIP(hipStreamSynchronize(c->stream));
  });
}

pty_status pty_cnn_grad(pty_cnn* c, const float* x, const float* target, int32_t batch, float* grad, double* loss) {
  return cnn_guard(c, [&] {
    if (!c || !x || !target || !grad) throw std::invalid_argument("pty_cnn_grad: null argument");
    check_batch(c, batch);
    PTY_HIP(hipSetDevice(c->device));
    const double l = loss_grad(c, x, target, batch);
    PTY_HIP(hipMemcpy(grad, c->g, c->nparams * sizeof(float), hipMemcpyDeviceToHost));
    if (loss) *loss = l;
  });
}

pty_status pty_cnn_train_step(pty_cnn* c, const float* x, const float* target, int32_t batch, float lr, double* loss) {
  return cnn_guard(c, [&] {
    if (!c || !x || !target) throw std::invalid_argument("pty_cnn_train_step: null argument");
    if (!(lr > 0.f) || !std::isfinite(lr)) throw std::invalid_argument("pty_cnn_train_step: lr must be > 0");
    check_batch(c, batch);
    PTY_HIP(hipSetDevice(c->device));
    const double l = loss_grad(c, x, target, batch);
    c->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)c->step), c2 = 1.f - std::pow(b2, (float)c->step);
    k_adam<<<blocks(c->nparams), 256, 0, c->stream>>>(c->p, c->g, c->m1, c->m2, c->nparams, lr, b1, b2, 1e-8f, c1, c2);
    PTY_LAUNCH_CHECK("adam");
    refresh_bf16(c);
    PTY_HIP(hipStreamSynchronize(c->stream));
    if (loss) *loss = l;
  });
}

pty_status pty_cnn_input(pty_cnn* c, const float* counts, int32_t batch, const void* probe, float* x) {
  return cnn_guard(c, [&] {
    if (!c || !counts || !probe || !x) throw std::invalid_argument("pty_cnn_input: null argument");
    if (batch < 1) throw std::invalid_argument("pty_cnn_input: batch must be >= 1");
    PTY_HIP(hipSetDevice(c->device));
    launch_seed_planes(static_cast<const float2*>(probe), c->planes, c->planes + 16384, c->stream);
    launch_seed_input_counts(counts, batch, c->planes, c->planes + 16384, x, c->stream);
    PTY_HIP(hipStreamSynchronize(c->stream));
  });
}

const char* pty_cnn_last_error(const pty_cnn* c) { return c ? c->err.c_str() : g_cnn_err.c_str(); }

}  // extern "C"
