// Kernels of the learned initialiser's data path and of the evaluation
// helpers: Poisson sampling of training patterns, network inputs and targets,
// the stitching of predicted patches into an object seed, and the invariant
// NRMSE (Fienup 1997) on a region of interest.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "pty_common.hpp"
#include "pty_fft.hpp"
#include "pty_geom.hpp"
#include "pty_kernels.hpp"

namespace pty {
namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// uniform in (0, 1) from 53 random bits of a counter
__device__ __forceinline__ double unit_open(uint64_t key) {
  return ((double)(splitmix64(key) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// Poisson(lambda) draws, one counter stream per element.  lambda < 10:
// inversion of the cumulative distribution; lambda >= 10: the transformed
// rejection method with squeeze of Hormann (1993, "The transformed rejection
// method for generating Poisson random variables", algorithm PTRS), which is
// exact.  Each trial takes two uniforms from the element's counter stream;
// the acceptance rate is above 0.9, and after 64 rejected trials (probability
// below 1e-60) the draw falls back to the rounded normal approximation.
__device__ double poisson_ptrs(double lam, uint64_t base) {
  const double slam = sqrt(lam), loglam = log(lam);
  const double b = 0.931 + 2.53 * slam;
  const double a = -0.059 + 0.02483 * b;
  const double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
  const double v_r = 0.9277 - 3.6224 / (b - 2.0);
  for (int t = 0; t < 64; ++t) {
    const double u = unit_open(base + 2 * (uint64_t)t) - 0.5;
    const double v = unit_open(base + 2 * (uint64_t)t + 1);
    const double us = 0.5 - fabs(u);
    const double k = floor((2.0 * a / us + b) * u + lam + 0.43);
    if (us >= 0.07 && v <= v_r) return k;
    if (k < 0.0 || (us < 0.013 && v > us)) continue;
    if (log(v) + log(inv_alpha) - log(a / (us * us) + b) <= -lam + k * loglam - lgamma(k + 1.0)) return k;
  }
  const double u1 = unit_open(base + 128), u2 = unit_open(base + 129);
  return fmax(0.0, floor(lam + slam * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2) + 0.5));
}

__global__ void k_poisson(const float* __restrict__ lam, float* __restrict__ out, size_t n, uint64_t seed) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double l = (double)lam[i];
  const uint64_t base = splitmix64(seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(i + 1)));
  float r = 0.f;
  if (l > 0.0 && l < 10.0) {
    const double u = unit_open(base);
    double p = exp(-l), f = p;
    int k = 0;
    while (u > f && k < 200) {
      ++k;
      p *= l / k;
      f += p;
    }
    r = (float)k;
  } else if (l >= 10.0) {
    r = (float)poisson_ptrs(l, base);
  }
  out[i] = r;
}

// ---------------------------------------------------------------------------
// Network input: a real-space estimate of each window's object patch,
//   est = g * F^-1(A u),   u = F(P) / |F(P)|,   g = conj(P) / (|P|^2 + 0.01 max |P|^2),
// A the measured moduli in natural order; the central 64 x 64 of est is
// written upsampled 2x (nearest) as a 128 x 128 x 2 (Re, Im) input.  One
// 128 x 128 window per block of 128 threads (16 lines of 8), transformed in
// LDS (rows padded to 129 entries against bank conflicts).
// ---------------------------------------------------------------------------
constexpr int kSeedN = 128;
constexpr int kSeedPitch = kSeedN + 1;
constexpr int kSeedThreads = 128;
constexpr int kSeedT = FftShape<kSeedN>::T, kSeedR = FftShape<kSeedN>::R;
constexpr int kSeedLines = kSeedThreads / kSeedT;
static_assert(kSeedT * kSeedR == kSeedN && kSeedLines * kSeedT == kSeedThreads, "seed input tiling");

struct SeedLds {
  float2 data[kSeedN * kSeedPitch];
  float2 xb[kSeedLines * LineLds<kSeedN>::words];
  float2 tw[kSeedN];
};

// W_128^i = exp(-2 pi i i / 128) from the double-precision sine and cosine
__device__ void seed_twiddles(float2* tw) {
  for (int i = threadIdx.x; i < kSeedN; i += kSeedThreads) {
    double sn, cs;
    sincospi(-2.0 * i / kSeedN, &sn, &cs);
    tw[i] = make_float2((float)cs, (float)sn);
  }
}

// line transforms of every row of the LDS window (unscaled)
template <bool INV>
__device__ void seed_rows(SeedLds& L) {
  const int line = threadIdx.x / kSeedT, t = threadIdx.x % kSeedT;
  for (int r0 = 0; r0 < kSeedN; r0 += kSeedLines) {
    float2* row = L.data + (r0 + line) * kSeedPitch;
    float2 v[kSeedR];
#pragma unroll
    for (int m = 0; m < kSeedR; ++m) v[m] = row[t + kSeedT * m];
    line_fft<kSeedN, INV>(v, L.xb + line * LineLds<kSeedN>::words, L.tw, t);
#pragma unroll
    for (int m = 0; m < kSeedR; ++m) row[t + kSeedT * m] = v[m];
  }
}

// F(P) / |F(P)| and g of mode 0 of the probe (one block)
__global__ __launch_bounds__(kSeedThreads) void k_seed_planes(const float2* __restrict__ probe, float2* __restrict__ u,
                                                              float2* __restrict__ g) {
  __shared__ SeedLds L;
  __shared__ float redf[kSeedThreads / 64];
  seed_twiddles(L.tw);
  float mx = 0.f;
  for (int q = threadIdx.x; q < kSeedN * kSeedN; q += kSeedThreads) {
    const float2 p = probe[q];
    L.data[(q / kSeedN) * kSeedPitch + q % kSeedN] = p;
    mx = fmaxf(mx, cabs2(p));
  }
  mx = block_max_all<kSeedThreads>(mx, redf);
  const float eps = 0.01f * mx;
  for (int q = threadIdx.x; q < kSeedN * kSeedN; q += kSeedThreads) {
    const float2 p = probe[q];
    const float d = cabs2(p) + eps;
    g[q] = d > 0.f ? make_float2(p.x / d, -p.y / d) : make_float2(0.f, 0.f);
  }
  __syncthreads();
  seed_rows<false>(L);
  __syncthreads();
  // columns: every column, transposed through registers
  const int line = threadIdx.x / kSeedT, t = threadIdx.x % kSeedT;
  for (int c0 = 0; c0 < kSeedN; c0 += kSeedLines) {
    const int c = c0 + line;
    float2 v[kSeedR];
#pragma unroll
    for (int m = 0; m < kSeedR; ++m) v[m] = L.data[(t + kSeedT * m) * kSeedPitch + c];
    line_fft<kSeedN, false>(v, L.xb + line * LineLds<kSeedN>::words, L.tw, t);
#pragma unroll
    for (int m = 0; m < kSeedR; ++m) {
      const float a = sqrtf(cabs2(v[m]));
      u[(t + kSeedT * m) * kSeedN + c] = a > 0.f ? make_float2(v[m].x / a, v[m].y / a) : make_float2(1.f, 0.f);
    }
  }
}

// One window per block.  FROM_COUNTS: centred counts of window b (training);
// else the context's natural-order moduli of pattern jsel[b] (a set sign bit,
// a masked pixel, reads as 0).
template <bool FROM_COUNTS>
__global__ __launch_bounds__(kSeedThreads) void k_seed_input(const float* __restrict__ src, const int* __restrict__ jsel,
                                                             const float2* __restrict__ u, const float2* __restrict__ g,
                                                             float* __restrict__ x) {
  __shared__ SeedLds L;
  seed_twiddles(L.tw);
  const int b = blockIdx.x;
  const size_t base = (size_t)(FROM_COUNTS ? b : jsel[b]) * kSeedN * kSeedN;
  for (int q = threadIdx.x; q < kSeedN * kSeedN; q += kSeedThreads) {
    const int r = q / kSeedN, c = q % kSeedN;
    float a;
    if constexpr (FROM_COUNTS) {
      const float d = src[base + (size_t)((r + kSeedN / 2) % kSeedN) * kSeedN + (c + kSeedN / 2) % kSeedN];
      a = sqrtf(fmaxf(d, 0.f));
    } else {
      const float m = src[base + q];
      a = signbit(m) ? 0.f : m;
    }
    const float2 w = u[q];
    L.data[r * kSeedPitch + c] = make_float2(a * w.x, a * w.y);
  }
  __syncthreads();
  seed_rows<true>(L);
  __syncthreads();
  // columns of the central half only; keep its central rows
  const int line = threadIdx.x / kSeedT, t = threadIdx.x % kSeedT;
  constexpr int Q = kSeedN / 4;
  constexpr float inv_n = 1.0f / kSeedN;
  float* xo = x + (size_t)b * kSeedN * kSeedN * 2;
  for (int c0 = Q; c0 < 3 * Q; c0 += kSeedLines) {
    const int c = c0 + line;
    float2 v[kSeedR];
#pragma unroll
    for (int m = 0; m < kSeedR; ++m) v[m] = L.data[(t + kSeedT * m) * kSeedPitch + c];
    line_fft<kSeedN, true>(v, L.xb + line * LineLds<kSeedN>::words, L.tw, t);
#pragma unroll
    for (int m = 0; m < kSeedR; ++m) {
      const int r = t + kSeedT * m;
      if (r < Q || r >= 3 * Q) continue;
      const float2 e = cmul(g[r * kSeedN + c], inv_n * v[m]);
      const int y = 2 * (r - Q), xx = 2 * (c - Q);
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx)
          reinterpret_cast<float2*>(xo)[(size_t)(y + dy) * kSeedN + xx + dx] = e;
    }
  }
}

// Training targets: amplitude and phase of the central n/2 x n/2 object patch
// of each window at an integer position.  One block (256 threads) per pattern.
__global__ __launch_bounds__(256) void k_targets(const float2* __restrict__ obj, int w, const PosInfo* __restrict__ pos,
                                                 int n, float* __restrict__ out) {
  const int j = blockIdx.x, m = n / 2, q = n / 4;
  const PosInfo p = pos[j];
  for (int e = threadIdx.x; e < m * m; e += 256) {
    const float2 o = obj[(size_t)(p.iy + q + e / m) * w + p.ix + q + e % m];
    out[((size_t)j * m * m + e) * 2] = sqrtf(o.x * o.x + o.y * o.y);
    out[((size_t)j * m * m + e) * 2 + 1] = atan2f(o.y, o.x);
  }
}

__device__ __forceinline__ float2 patch_value(const float* __restrict__ pt, size_t idx) {
  const float a = pt[idx * 2], ph = pt[idx * 2 + 1];
  float s, c;
  sincosf(ph, &s, &c);
  return make_float2(a * c, a * s);
}

// Sequential phase-offset chain over the patches in index order, on the
// coarse grid G of object pixels whose coordinates are multiples of 8 (8 x 8
// samples per 64 x 64 patch; lane l of the single wavefront takes sample l).  For patch j: z = sum over its samples of S * conj(c_j),
// e_j = z / |z| (1 if z = 0), then S += c_j e_j on those samples.  Writes
// e_j to phasor[j].  S lives in LDS when it fits (IN_LDS), else in the
// zero-filled global array S_g.  The next patch's samples are loaded while
// the current one is processed (they do not depend on S).
constexpr int kChainGrid = 8;
template <bool IN_LDS>
__global__ __launch_bounds__(64) void k_seed_chain(const float* __restrict__ patches, const int2* __restrict__ place,
                                                   int j_count, float2* S_g, int hc, int wc,
                                                   float2* __restrict__ phasor) {
  extern __shared__ float2 S_l[];
  const int lane = threadIdx.x;
  const int sy = lane >> 3, sx = lane & 7;
  float2* S = IN_LDS ? S_l : S_g;
  if (IN_LDS) {
    for (int i = lane; i < hc * wc; i += 64) S_l[i] = make_float2(0.f, 0.f);
    __syncthreads();
  }
  auto sample = [&](int j, int& cell) -> float2 {
    const int2 t = place[j];
    const int gy = (t.x + kChainGrid - 1) & ~(kChainGrid - 1), gx = (t.y + kChainGrid - 1) & ~(kChainGrid - 1);
    const int u = gy - t.x + kChainGrid * sy, v = gx - t.y + kChainGrid * sx;
    cell = (gy / kChainGrid + sy) * wc + gx / kChainGrid + sx;
    return patch_value(patches, (size_t)j * 4096 + u * 64 + v);
  };
  int cell_next = 0;
  float2 c_next = j_count > 0 ? sample(0, cell_next) : make_float2(0.f, 0.f);
  for (int j = 0; j < j_count; ++j) {
    const float2 c = c_next;
    const int cell = cell_next;
    if (j + 1 < j_count) c_next = sample(j + 1, cell_next);
    const float2 s = S[cell];
    float zr = s.x * c.x + s.y * c.y, zi = s.y * c.x - s.x * c.y;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      zr += __shfl_xor(zr, off, 64);
      zi += __shfl_xor(zi, off, 64);
    }
    const float zn = sqrtf(zr * zr + zi * zi);
    const float er = zn > 0.f ? zr / zn : 1.f, ei = zn > 0.f ? zi / zn : 0.f;
    S[cell] = make_float2(s.x + c.x * er - c.y * ei, s.y + c.x * ei + c.y * er);
    if (lane == 0) phasor[j] = make_float2(er, ei);
    // the next patch may read what this one wrote
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    if (IN_LDS)
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    else
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  }
}

// Stitch: O(p) = mean over the patches covering p of c_j(p - t_j) e_j;
// 1 where no patch covers p.  Candidate patches come from 64 x 64 bins of the
// placements (CSR `bin_beg`, `bin_idx`): a patch covering p has its corner in
// p's bin or the bins above / to the left.
__global__ void k_seed_stitch(const float* __restrict__ patches, const int2* __restrict__ place,
                              const float2* __restrict__ phasor, const int* __restrict__ bin_beg,
                              const int* __restrict__ bin_idx, int bins_w, int bins_h, float2* __restrict__ obj, int h,
                              int w) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= (size_t)h * w) return;
  const int y = (int)(i / w), x = (int)(i % w);
  const int by = y >> 6, bx = x >> 6;
  float ar = 0.f, ai = 0.f;
  int cnt = 0;
  for (int dy = -1; dy <= 0; ++dy) {
    const int yy = by + dy;
    if (yy < 0 || yy >= bins_h) continue;
    for (int dx = -1; dx <= 0; ++dx) {
      const int xx = bx + dx;
      if (xx < 0 || xx >= bins_w) continue;
      const int b = yy * bins_w + xx;
      for (int e = bin_beg[b]; e < bin_beg[b + 1]; ++e) {
        const int j = bin_idx[e];
        const int2 t = place[j];
        const int u = y - t.x, v = x - t.y;
        if ((unsigned)u >= 64u || (unsigned)v >= 64u) continue;
        const float2 c = patch_value(patches, (size_t)j * 4096 + u * 64 + v);
        const float2 ph = phasor ? phasor[j] : make_float2(1.f, 0.f);
        ar += c.x * ph.x - c.y * ph.y;
        ai += c.x * ph.y + c.y * ph.x;
        ++cnt;
      }
    }
  }
  obj[i] = cnt ? make_float2(ar / cnt, ai / cnt) : make_float2(1.f, 0.f);
}

// NRMSE partial sums over the mask: (sum |o|^2, Re sum conj(o) t, Im ..., sum |t|^2)
constexpr int kNrmseBlocks = 512;
__global__ __launch_bounds__(256) void k_nrmse_part(const float2* __restrict__ o, const float2* __restrict__ t,
                                                    const unsigned char* __restrict__ mask, size_t n,
                                                    double* __restrict__ part) {
  __shared__ double sh[4][4];
  double a = 0, b = 0, c = 0, d = 0;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)kNrmseBlocks * 256) {
    if (!mask[i]) continue;
    const float2 x = o[i], y = t[i];
    a += (double)x.x * x.x + (double)x.y * x.y;
    b += (double)x.x * y.x + (double)x.y * y.y;
    c += (double)x.x * y.y - (double)x.y * y.x;
    d += (double)y.x * y.x + (double)y.y * y.y;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
    c += __shfl_down(c, off, 64);
    d += __shfl_down(d, off, 64);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][wv] = a;
    sh[1][wv] = b;
    sh[2][wv] = c;
    sh[3][wv] = d;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int r = threadIdx.x;
    part[blockIdx.x * 4 + r] = sh[r][0] + sh[r][1] + sh[r][2] + sh[r][3];
  }
}

// ||c o - t||^2 at the optimal c is sum|t|^2 - |<o, t>|^2 / sum|o|^2
__global__ void k_nrmse_final(const double* __restrict__ part, double* __restrict__ out, int* slot, int advance) {
  double s[4] = {0, 0, 0, 0};
  for (int b = 0; b < kNrmseBlocks; ++b)
    for (int r = 0; r < 4; ++r) s[r] += part[b * 4 + r];
  const double num = s[0] > 0 ? s[3] - (s[1] * s[1] + s[2] * s[2]) / s[0] : s[3];
  const int t = slot ? *slot : 0;
  out[t] = s[3] > 0 ? sqrt(fmax(num, 0.0) / s[3]) : 0.0;
  if (advance) *slot = t + 1;
}

__global__ void k_set_i32(int* p, int v) { *p = v; }

// mask[i] = den[i] >= frac * max(den)
__global__ void k_roi_mask(const float* __restrict__ den, const unsigned* __restrict__ den_max, float frac, size_t n,
                           unsigned char* __restrict__ mask) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  mask[i] = den[i] >= frac * __uint_as_float(*den_max) ? 1 : 0;
}

__global__ void k_fill_c64(float2* __restrict__ p, size_t n, float2 v) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned nblk(size_t n, unsigned bs = 256) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_fill_c64(float2* p, size_t n, float2 v, hipStream_t s) {
  if (n == 0) return;
  k_fill_c64<<<nblk(n), 256, 0, s>>>(p, n, v);
  PTY_LAUNCH_CHECK("fill_c64");
}

void launch_poisson(const float* lam, float* out, size_t n, uint64_t seed, hipStream_t s) {
  if (n == 0) return;
  k_poisson<<<nblk(n), 256, 0, s>>>(lam, out, n, seed);
  PTY_LAUNCH_CHECK("poisson");
}

void launch_seed_planes(const float2* probe, float2* u, float2* g, hipStream_t s) {
  k_seed_planes<<<1, kSeedThreads, 0, s>>>(probe, u, g);
  PTY_LAUNCH_CHECK("seed_planes");
}

void launch_seed_input_counts(const float* counts, int nb, const float2* u, const float2* g, float* x, hipStream_t s) {
  if (nb <= 0) return;
  k_seed_input<true><<<nb, kSeedThreads, 0, s>>>(counts, nullptr, u, g, x);
  PTY_LAUNCH_CHECK("seed_input");
}

void launch_seed_input_amp(const float* amp, const int* jsel, int nb, const float2* u, const float2* g, float* x,
                           hipStream_t s) {
  if (nb <= 0) return;
  k_seed_input<false><<<nb, kSeedThreads, 0, s>>>(amp, jsel, u, g, x);
  PTY_LAUNCH_CHECK("input_from_amp");
}

void launch_targets(const float2* obj, int w, const PosInfo* pos, int j, int n, float* out, hipStream_t s) {
  if (j == 0) return;
  k_targets<<<j, 256, 0, s>>>(obj, w, pos, n, out);
  PTY_LAUNCH_CHECK("targets");
}

int seed_chain_grid() { return kChainGrid; }

void launch_seed_chain(const float* patches, const int2* place, int j, float2* S, int hc, int wc, float2* phasor,
                       hipStream_t s) {
  const size_t lds = (size_t)hc * wc * sizeof(float2);
  if (lds <= 160 * 1024) {
    PTY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_seed_chain<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    k_seed_chain<true><<<1, 64, lds, s>>>(patches, place, j, S, hc, wc, phasor);
  }
  else
    k_seed_chain<false><<<1, 64, 0, s>>>(patches, place, j, S, hc, wc, phasor);
  PTY_LAUNCH_CHECK("seed_chain");
}

void launch_seed_stitch(const float* patches, const int2* place, const float2* phasor, const int* bin_beg,
                        const int* bin_idx, int bins_w, int bins_h, float2* obj, int h, int w, hipStream_t s) {
  k_seed_stitch<<<nblk((size_t)h * w), 256, 0, s>>>(patches, place, phasor, bin_beg, bin_idx, bins_w, bins_h, obj, h,
                                                   w);
  PTY_LAUNCH_CHECK("seed_stitch");
}

size_t nrmse_part_doubles() { return kNrmseBlocks * 4; }

void launch_nrmse(const float2* o, const float2* t, const unsigned char* mask, size_t n, double* part, double* out,
                  hipStream_t s, int* slot, bool advance) {
  k_nrmse_part<<<kNrmseBlocks, 256, 0, s>>>(o, t, mask, n, part);
  k_nrmse_final<<<1, 1, 0, s>>>(part, out, slot, advance ? 1 : 0);
  PTY_LAUNCH_CHECK("nrmse");
}

void launch_set_i32(int* p, int v, hipStream_t s) {
  k_set_i32<<<1, 1, 0, s>>>(p, v);
  PTY_LAUNCH_CHECK("set_i32");
}

void launch_roi_mask(const float* den, const unsigned* den_max, float frac, size_t n, unsigned char* mask,
                     hipStream_t s) {
  k_roi_mask<<<nblk(n), 256, 0, s>>>(den, den_max, frac, n, mask);
  PTY_LAUNCH_CHECK("roi_mask");
}

}  // namespace pty
