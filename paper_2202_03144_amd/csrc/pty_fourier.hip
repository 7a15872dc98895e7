// Fused Fourier passes of one reconstruction iteration.
//
// For a chunk of patterns the 2-D transforms are split into three passes that
// communicate through a chunk-sized scratch buffer (sized to stay in the
// MI355X Infinity Cache):
//   rows_fwd : gather S_j O (bilinear), exit wave P_k S_j O (DM: reflected
//              2 P S_j O - psi), forward FFT along x, all K modes per block;
//   cols     : forward FFT along y of all K modes, then per far-field pixel
//              the multi-mode modulus projection (Delta = (A / max(sqrt I, eps)
//              - 1) Psi) with the amplitude-error partials, or the Poisson-NLL
//              factor (1 - d / (I + eps)), then the inverse FFT along y;
//   rows_inv : inverse FFT along x and the algorithm's epilogue (DM: new exit
//              waves psi = phi + chi; LSQML / ePIE: store chi; adjoint: store
//              g_psi and the position-gradient partials), plus the per-pattern
//              contribution sum_k conj(P_k) (.) used by the object update.
// Methods: Sec. 2.3 (far-field ptychography with ePIE, DM and LSQML; multi-mode
// probes, Sec. 2.2).
#include "pty_geom.hpp"
#include "pty_kernels.hpp"
#include "pty_wave.hpp"

namespace pty {
namespace {

// Scratch layout of one pattern-mode: 4-column blocks, [x / 4][y][x % 4].
// Row passes (16 lanes per row, 4 rows per wavefront) touch 128-byte runs;
// the column pass (16 lanes per column, 4 adjacent columns per wavefront)
// reads and writes 512 contiguous bytes per instruction.
template <int N>
__device__ __forceinline__ size_t zoff(int y, int x) {
  return ((size_t)(x >> 2) * N + y) * 4 + (x & 3);
}

// Row y of S_j O at the columns t + T m a line's lanes own, for lines of
// T = 16 lanes (one DPP row): the taps of column c + 1 are the next lane's
// taps of column c (for the last lane, lane 0's of the next m; past the last
// m, one more load, clamped like obj_bilinear's), so an element costs two
// loads instead of four.  Values and arithmetic are obj_bilinear's.
__device__ __forceinline__ float2 row_rotl1(float2 v) {   // lane i <- lane i + 1 of its row of 16
  return make_float2(__int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v.x), 0x12F, 0xf, 0xf, false)),
                     __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v.y), 0x12F, 0xf, 0xf, false)));
}
template <int N>
__device__ __forceinline__ void line_bilinear(const float2* __restrict__ o, int h, int w, const PosInfo& p, int y, int t,
                                              float2* out) {
  constexpr int R = FftShape<N>::R, T = FftShape<N>::T;
  if constexpr (T != 16) {
#pragma unroll
    for (int m = 0; m < R; ++m) out[m] = obj_bilinear(o, h, w, p, y, t + T * m);
  } else {
    const int r0 = p.iy + y, r1 = min(r0 + 1, h - 1);
    const float2* a0 = o + (size_t)r0 * w + p.ix + t;
    const float2* a1 = o + (size_t)r1 * w + p.ix + t;
    float2 va[R], vc[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
      va[m] = a0[T * m];
      vc[m] = a1[T * m];
    }
    const int ce = min(p.ix + N, w - 1);
    const float2 ea = o[(size_t)r0 * w + ce], ec = o[(size_t)r1 * w + ce];
    const float wx1 = p.fx, wx0 = 1.f - p.fx, wy1 = p.fy, wy0 = 1.f - p.fy;
    const bool last = t == T - 1;
    float2 ra = row_rotl1(va[0]), rc = row_rotl1(vc[0]);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      float2 b, d;
      if (m + 1 < R) {
        const float2 na = row_rotl1(va[m + 1]), nc = row_rotl1(vc[m + 1]);
        b = last ? na : ra;
        d = last ? nc : rc;
        ra = na;
        rc = nc;
      } else {
        b = last ? ea : ra;
        d = last ? ec : rc;
      }
      const float2 a = va[m], c = vc[m];
      out[m] = make_float2(wy0 * (wx0 * a.x + wx1 * b.x) + wy1 * (wx0 * c.x + wx1 * d.x),
                           wy0 * (wx0 * a.y + wx1 * b.y) + wy1 * (wx0 * c.y + wx1 * d.y));
    }
  }
}

// Patterns per block of the forward rows: with three or more modes each
// probe row is loaded once for two patterns (with fewer modes the two
// patterns' registers do not fit beside each other).
template <int N, int K>
constexpr int rows_fwd_patterns() { return (K >= 3 && N <= 256) ? 2 : 1; }

template <int N, int K, RowIn MODE>
__global__ __launch_bounds__(Geo<N>::BS)
void k_rows_fwd(FourierArgs a) {
  using G = Geo<N>;
  constexpr int R = G::R, T = G::T, PB = rows_fwd_patterns<N, K>();
  __shared__ float2 tw_s[N];
  __shared__ float2 xb[G::LINES * G::W];
  load_twiddles<N>(tw_s, reinterpret_cast<const float2*>(a.tw));
  const int line = threadIdx.x / T, t = threadIdx.x % T;
  const int y = blockIdx.x * G::LINES + line;
  constexpr bool DMR = MODE == RowIn::DmReflect;
  if constexpr (PB == 1) {
    const int c = blockIdx.y;
    const int j = a.jlist[a.jl_off + c];
    float2 o[R];
    line_bilinear<N>(a.obj, a.h, a.w, a.pos[j], y, t, o);
    // One mode at a time keeps the register footprint at one line per thread;
    // the next mode's probe (and DM exit-wave) row is loaded before this mode's
    // transform and stores, so the loads overlap them.
    float2 pa[R], pb[DMR ? R : 1];
    auto load_mode = [&](int k) {
      const float2* pr = a.probe + ((size_t)k * N + y) * N;
#pragma unroll
      for (int m = 0; m < R; ++m) pa[m] = pr[t + T * m];
      if constexpr (DMR) {
        const float2* ps = a.psi + (((size_t)j * K + k) * N + y) * N;
#pragma unroll
        for (int m = 0; m < R; ++m) pb[m] = ps[t + T * m];
      }
    };
    load_mode(0);
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
      float2 z[R];
#pragma unroll
      for (int m = 0; m < R; ++m) {
        z[m] = cmul(pa[m], o[m]);
        if constexpr (DMR) z[m] = 2.f * z[m] - pb[m];
      }
      if (k + 1 < K) load_mode(k + 1);
      line_fft<N, false>(z, xb + line * G::W, tw_s, t);
      float2* out = a.zs + ((size_t)c * K + k) * N * N;
#pragma unroll
      for (int m = 0; m < R; ++m) out[zoff<N>(y, t + T * m)] = z[m];
    }
  } else {
    const int c0 = blockIdx.y * PB;
    const int np = min(PB, a.nc - c0);          // patterns of this block (uniform)
    int j[PB];
    float2 o[PB][R];
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      j[q] = a.jlist[a.jl_off + c0 + min(q, np - 1)];
      line_bilinear<N>(a.obj, a.h, a.w, a.pos[j[q]], y, t, o[q]);
    }
    // One mode at a time; the mode's probe row serves both patterns, and the
    // DM exit-wave rows of both are loaded with it, before the transforms.
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
      float2 pa[R], pb[DMR ? PB : 1][R];
      const float2* pr = a.probe + ((size_t)k * N + y) * N;
#pragma unroll
      for (int m = 0; m < R; ++m) pa[m] = pr[t + T * m];
      if constexpr (DMR) {
#pragma unroll
        for (int q = 0; q < PB; ++q) {
          const float2* ps = a.psi + (((size_t)j[q] * K + k) * N + y) * N;
#pragma unroll
          for (int m = 0; m < R; ++m) pb[q][m] = ps[t + T * m];
        }
      }
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        if (q >= np) break;
        float2 z[R];
#pragma unroll
        for (int m = 0; m < R; ++m) {
          z[m] = cmul(pa[m], o[q][m]);
          if constexpr (DMR) z[m] = 2.f * z[m] - pb[q][m];
        }
        line_fft<N, false>(z, xb + line * G::W, tw_s, t);
        float2* out = a.zs + ((size_t)(c0 + q) * K + k) * N * N;
#pragma unroll
        for (int m = 0; m < R; ++m) out[zoff<N>(y, t + T * m)] = z[m];
        // the second pattern's transform after the first's (interleaving the
        // two would double the live registers)
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
}

// Modes per thread group in the column pass.  The projection needs every
// mode of a far-field pixel at once; holding all K modes of an R-value line
// costs 2 K R registers, which at K = 4, R = 16 leaves one wavefront per SIMD.
// There the modes are split over MS = 2 groups of T lanes per column (one
// after the other in a wavefront), which add their partial intensities with
// one lane shuffle; a block then covers 1 / MS as many columns and a pattern
// MS times as many blocks.
template <int N, int K>
struct ColSplit {
  static constexpr int MS = (K % 2 == 0 && (K * FftShape<N>::R) > 48) ? 2 : 1;
  static constexpr int CW = Geo<N>::LINES / MS;   // columns per block
  static constexpr int BPP = N / CW;              // blocks per pattern
};

template <int N, int K, ColOp OP, bool MASK>
__device__ __forceinline__ void cols_body(const FourierArgs& a) {
  using G = Geo<N>;
  using S = ColSplit<N, K>;
  constexpr int R = G::R, T = G::T, CW = S::CW, BPP = S::BPP, MS = S::MS, KM = K / MS;
  // The block's measured amplitudes (N rows x CW columns) are staged in LDS,
  // column-major with a 16-word skew per column: each thread writes and later
  // reads the rows of its own line, so a wavefront's lines (adjacent columns)
  // touch distinct banks both ways.  Only where the register budget already
  // holds the kernel to two wavefronts per SIMD (256^2 with two or three
  // modes, one thread group per column, the ops that invert), so that the
  // 17 KB do not lower it.
  constexpr bool AMP_LDS = N == 256 && K >= 2 && MS == 1 &&
                           (OP == ColOp::Project || OP == ColOp::NllGrad || OP == ColOp::Poisson);
  constexpr int AS = N + 16;   // words per staged column
  __shared__ float2 tw_s[N];
  __shared__ float2 xb[G::LINES * G::W];
  __shared__ double red[G::BS / 64];
  __shared__ double red2[G::BS / 64][2];
  __shared__ float amp_s[AMP_LDS ? CW * AS : 1];
  // each line's T threads are consecutive lanes of one wavefront; the MS
  // groups of a column are adjacent, so their lanes differ by T
  const int grp = threadIdx.x / T, t = threadIdx.x % T;
  const int col = grp / MS, kg = grp % MS;
  const bool lead = kg == 0;
  const int c = blockIdx.y, cb = blockIdx.x, x = cb * CW + col;
  const int j = a.jlist[a.jl_off + c];
  float2* base = a.zs + ((size_t)c * K + kg * KM) * N * N;
  float2* buf = xb + grp * G::W;
  // twiddles and amplitudes first, then the column values; the LDS copies
  // wait only for the first two (an LDS-only barrier leaves the column loads
  // in flight).  At 512 the twiddles are copied before the column loads (two
  // per thread held across them spill the masked projection).
  constexpr bool TW_EARLY = N <= 256;
  constexpr int TWQ = (N + G::BS - 1) / G::BS;
  if constexpr (!TW_EARLY) load_twiddles<N>(tw_s, reinterpret_cast<const float2*>(a.tw));
  float2 twv[TW_EARLY ? TWQ : 1];
  if constexpr (TW_EARLY) {
#pragma unroll
    for (int i = 0; i < TWQ; ++i) {
      const int q = threadIdx.x + G::BS * i;
      if (q < N) twv[i] = reinterpret_cast<const float2*>(a.tw)[q];
    }
  }
  float av[AMP_LDS ? R : 1];
  if constexpr (AMP_LDS) {
#pragma unroll
    for (int m = 0; m < R; ++m) av[m] = a.amp[((size_t)j * N + t + T * m) * N + x];
  }
  float2 z[KM][R];
#pragma unroll
  for (int k = 0; k < KM; ++k) {
#pragma unroll
    for (int m = 0; m < R; ++m) z[k][m] = base[(size_t)k * N * N + zoff<N>(t + T * m, x)];
  }
  if constexpr (TW_EARLY) {
#pragma unroll
    for (int i = 0; i < TWQ; ++i) {
      const int q = threadIdx.x + G::BS * i;
      if (q < N) tw_s[q] = twv[i];
    }
  }
  if constexpr (AMP_LDS) {
#pragma unroll
    for (int m = 0; m < R; ++m) amp_s[col * AS + t + T * m] = av[m];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
#pragma unroll
  for (int k = 0; k < KM; ++k) line_fft<N, false>(z[k], buf, tw_s, t);
  // The transforms are unscaled: the unitary far field is z / N and the
  // unitary inverse of the whole pipeline contributes another 1 / N^2, both
  // folded into the per-pixel factor applied before the inverse transforms.
  constexpr float sc = 1.0f / N, sc2 = 1.0f / (float(N) * float(N));
  float e_num = 0.f, e_den = 0.f;
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int pr = t + T * m;
    float iraw = 0.f;
#pragma unroll
    for (int k = 0; k < KM; ++k) iraw += cabs2(z[k][m]);
    if constexpr (MS == 2) iraw += __shfl_xor(iraw, T, 64);
    const float inten = iraw * sc2;
    if constexpr (OP == ColOp::Intensity) {
      if (lead)
        a.intensity_out[((size_t)j * N + ((pr + N / 2) & (N - 1))) * N + ((x + N / 2) & (N - 1))] = inten;
    } else if constexpr (OP == ColOp::NllLoss) {
      if (lead) {
        const float ar = AMP_LDS ? amp_s[col * AS + pr] : a.amp[((size_t)j * N + pr) * N + x];
        const float d = ar * ar;
        const float l = inten - d * logf(inten + a.nll_eps);
        if constexpr (MASK)
          e_num += signbit(ar) ? 0.f : l;
        else
          e_num += l;
      }
    } else {
      // With a detector mask, a set sign bit marks a pixel without a
      // measurement: the projection keeps the model there and the pixel adds
      // to no sum.  (A separate instantiation, so that the unmasked kernels
      // keep their register budget.)
      const float ar = AMP_LDS ? amp_s[col * AS + pr] : a.amp[((size_t)j * N + pr) * N + x];
      float mf = 1.f, am = ar;
      if constexpr (MASK) {
        mf = signbit(ar) ? 0.f : 1.f;
        am = fabsf(ar);
      }
      float f;
      if constexpr (OP == ColOp::Project || OP == ColOp::Poisson) {
        // hardware square root and reciprocal (1 ulp each) in place of the
        // correctly rounded forms and their refinement steps
        const float mod = __builtin_amdgcn_sqrtf(iraw) * sc;
        if constexpr (OP == ColOp::Project) {
          f = am * __builtin_amdgcn_rcpf(fmaxf(mod, 1e-6f)) - 1.f;
        } else {
          // the Poisson update moves Psi by -alpha_R g Psi, g = 1 - d / (I + eps);
          // alpha_R (k_poisson_alpha) minimises the pattern's likelihood along
          // that ray and needs every pixel's I, stored here.  The hardware
          // reciprocal (1 ulp) in place of the full division keeps the kernel
          // within two wavefronts per SIMD
          const float r = (am * am) * __builtin_amdgcn_rcpf(inten + a.nll_eps);
          f = 1.f - r;
          if (lead) a.pinten[((size_t)c * N + pr) * N + x] = inten;
        }
        if constexpr (MASK) f *= mf;
        if (lead) {
          if constexpr (MASK) {
            e_num += mf * ((mod - am) * (mod - am));
            e_den += mf * (am * am);
          } else {
            e_num += (mod - am) * (mod - am);
            e_den += am * am;
          }
        }
      } else {
        const float d = am * am;
        f = a.grad_scale * (1.f - d / (inten + a.nll_eps));
        const float l = inten - d * logf(inten + a.nll_eps);
        if constexpr (MASK) {
          f *= mf;
          if (lead) e_num += mf * l;
        } else {
          if (lead) e_num += l;
        }
      }
      f *= sc2;
#pragma unroll
      for (int k = 0; k < KM; ++k) z[k][m] = f * z[k][m];
    }
  }
  if constexpr (OP == ColOp::Poisson) {
    // reduced before the inverse transforms, which then carry no sums
    const double s0 = block_sum<G::BS>((double)e_num, red);
    const double s1 = block_sum<G::BS>((double)e_den, red);
    if (threadIdx.x == 0) {
      double* e = a.errp + ((size_t)j * BPP + cb) * 2;
      e[0] = s0;
      e[1] = s1;
    }
  }
  if constexpr (OP == ColOp::Project || OP == ColOp::NllGrad || OP == ColOp::Poisson) {
    // each mode is stored as soon as its inverse transform is done, so the
    // stores drain under the next mode's transform
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      line_fft<N, true>(z[k], buf, tw_s, t);
#pragma unroll
      for (int m = 0; m < R; ++m) base[(size_t)k * N * N + zoff<N>(t + T * m, x)] = z[k][m];
    }
  }
  if constexpr (OP != ColOp::Intensity && OP != ColOp::Poisson) {
    // both sums per wavefront by DPP lane moves, then the wavefronts' in order
    const double w0 = wave_sum_d((double)e_num), w1 = wave_sum_d((double)e_den);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
      red2[wid][0] = w0;
      red2[wid][1] = w1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int w = 0; w < G::BS / 64; ++w) {
        s0 += red2[w][0];
        s1 += red2[w][1];
      }
      double* e = a.errp + ((size_t)j * BPP + cb) * 2;
      e[0] = s0;
      e[1] = s1;
    }
  }
}

template <int N, int K, ColOp OP, bool MASK>
__global__ __launch_bounds__(Geo<N>::BS)
void k_cols(FourierArgs a) {
  cols_body<N, K, OP, MASK>(a);
}

// The masked instantiations carry the mask test and its sums; left to itself
// the compiler has given the 256^2 x 3-mode projection one wavefront per
// SIMD.  Held to two, it keeps the unmasked kernel's occupancy.
template <int N, int K, ColOp OP>
__global__ __launch_bounds__(Geo<N>::BS) __attribute__((amdgpu_waves_per_eu(2)))
void k_cols_masked(FourierArgs a) {
  cols_body<N, K, OP, true>(a);
}

// The Poisson step carries two more sums and a division per pixel; left to
// itself the compiler gives the 256^2 x 3-mode instance one wavefront per
// SIMD, which doubles its time.  Held to two, it spills a few registers.
template <int N, int K, bool MASK>
__global__ __launch_bounds__(Geo<N>::BS) __attribute__((amdgpu_waves_per_eu(2)))
void k_cols_poisson(FourierArgs a) {
  cols_body<N, K, ColOp::Poisson, MASK>(a);
}

// Patterns per block of the inverse rows: storing chi with three or more
// modes, each probe row is loaded once for two patterns (the DM update's
// second object patch would not fit beside the first).
template <int N, int K, RowOut MODE>
constexpr int rows_inv_patterns() { return (K >= 3 && N <= 256 && MODE == RowOut::StoreChi) ? 2 : 1; }

template <int N, int K, RowOut MODE>
__global__ __launch_bounds__(Geo<N>::BS)
void k_rows_inv(FourierArgs a) {
  using G = Geo<N>;
  constexpr int R = G::R, T = G::T, BPP = N / G::LINES, PB = rows_inv_patterns<N, K, MODE>();
  __shared__ float2 tw_s[N];
  __shared__ float2 xb[G::LINES * G::W];
  __shared__ double red[G::BS / 64];
  load_twiddles<N>(tw_s, reinterpret_cast<const float2*>(a.tw));
  if constexpr (PB == 1) {
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int c = blockIdx.y, rb = blockIdx.x;
    const int y = rb * G::LINES + line;
    const int slot = a.slot_off + c;
    const int j = a.jlist[a.jl_off + c];
    const PosInfo p = a.pos[j];
    // the column pass already applied the unitary scales of both transforms
    float2 o[MODE == RowOut::DmUpdate ? R : 1];
    float2 gdy[MODE == RowOut::NllGrad ? R : 1], gdx[MODE == RowOut::NllGrad ? R : 1];
    if constexpr (MODE == RowOut::DmUpdate) line_bilinear<N>(a.obj, a.h, a.w, p, y, t, o);
    if constexpr (MODE == RowOut::NllGrad) {
  #pragma unroll
      for (int m = 0; m < R; ++m) obj_bilinear_grad(a.obj, a.h, a.w, p, y, t + T * m, gdy[m], gdx[m]);
    }
    // Poisson update: chi = -alpha_R F^-1[g Psi]
    float chi_s = 1.f;
    if constexpr (MODE == RowOut::StoreChi) {
      if (a.poisp) chi_s = (float)(-a.poisp[slot]);
    }
    float2 cacc[R];
  #pragma unroll
    for (int m = 0; m < R; ++m) cacc[m] = make_float2(0.f, 0.f);
    float gy = 0.f, gx = 0.f;
    // one mode at a time keeps the register footprint at one line per thread
  #pragma unroll 1
    for (int k = 0; k < K; ++k) {
      float2 z[R];
      const float2* src = a.zs + ((size_t)c * K + k) * N * N;
  #pragma unroll
      for (int m = 0; m < R; ++m) z[m] = src[zoff<N>(y, t + T * m)];
      // the probe row is read before the transform: the epilogue's stores could
      // alias it, so loads issued among them would each wait for the memory
      // (the position-gradient epilogue keeps the late loads: its registers are full)
      const float2* pr = a.probe + ((size_t)k * N + y) * N;
      constexpr bool PRE = MODE != RowOut::NllGrad;
      float2 pkr[PRE ? R : 1];
      if constexpr (PRE) {
  #pragma unroll
        for (int m = 0; m < R; ++m) pkr[m] = pr[t + T * m];
      }
      line_fft<N, true>(z, xb + line * G::W, tw_s, t);
      if constexpr (MODE == RowOut::StoreChi) {
        if (a.poisp) {
  #pragma unroll
          for (int m = 0; m < R; ++m) z[m] = chi_s * z[m];
        }
      }
      if constexpr (MODE == RowOut::DmUpdate) {
        float2* ps = a.psi + (((size_t)j * K + k) * N + y) * N;
  #pragma unroll
        for (int m = 0; m < R; ++m) {
          const float2 pk = pkr[m];
          const float2 nw = cmul(pk, o[m]) + z[m];
          ps[t + T * m] = nw;
          cacc[m] = cacc[m] + cconjmul(pk, nw);
        }
      } else {
        const float gscale = (MODE == RowOut::NllGrad) ? 2.f : 1.f;
        float2* ch = a.chi + (((size_t)slot * K + k) * N + y) * N;
  #pragma unroll
        for (int m = 0; m < R; ++m) {
          float2 pk;
          if constexpr (PRE) pk = pkr[m];
          else pk = pr[t + T * m];
          ch[t + T * m] = z[m];
          cacc[m] = cacc[m] + gscale * cconjmul(pk, z[m]);
          if constexpr (MODE == RowOut::NllGrad) {
            const float2 gpy = cmul(pk, gdy[m]), gpx = cmul(pk, gdx[m]);
            // Re(conj(g_psi) * P_k * d(S_j O))
            gy += z[m].x * gpy.x + z[m].y * gpy.y;
            gx += z[m].x * gpx.x + z[m].y * gpx.y;
          }
        }
      }
    }
    if constexpr (MODE == RowOut::NllGrad) {
      const double sy = block_sum<G::BS>(2.0 * gy, red);
      const double sx = block_sum<G::BS>(2.0 * gx, red);
      if (threadIdx.x == 0) {
        double* g = a.posgrad + ((size_t)slot * BPP + rb) * 2;
        g[0] = sy;
        g[1] = sx;
      }
    }
    float2* cb = a.contrib + ((size_t)slot * N + y) * N;
  #pragma unroll
    for (int m = 0; m < R; ++m) cb[t + T * m] = cacc[m];
  } else {
    const int line = threadIdx.x / T, t = threadIdx.x % T;
    const int y = blockIdx.x * G::LINES + line;
    const int c0 = blockIdx.y * PB;
    const int np = min(PB, a.nc - c0);          // patterns of this block (uniform)
    constexpr bool DMU = MODE == RowOut::DmUpdate;
    int j[PB], slot[PB];
    float chi_s[PB];
    float2 o[DMU ? PB : 1][R], cacc[PB][R];
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      j[q] = a.jlist[a.jl_off + c0 + min(q, np - 1)];
      slot[q] = a.slot_off + c0 + min(q, np - 1);
      if constexpr (DMU) line_bilinear<N>(a.obj, a.h, a.w, a.pos[j[q]], y, t, o[q]);
      // Poisson update: chi = -alpha_R F^-1[g Psi]
      chi_s[q] = (MODE == RowOut::StoreChi && a.poisp) ? (float)(-a.poisp[slot[q]]) : 1.f;
#pragma unroll
      for (int m = 0; m < R; ++m) cacc[q][m] = make_float2(0.f, 0.f);
    }
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
      // the mode's probe row, once for both patterns
      const float2* pr = a.probe + ((size_t)k * N + y) * N;
      float2 pkr[R];
#pragma unroll
      for (int m = 0; m < R; ++m) pkr[m] = pr[t + T * m];
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        if (q >= np) break;
        float2 z[R];
        const float2* src = a.zs + ((size_t)(c0 + q) * K + k) * N * N;
#pragma unroll
        for (int m = 0; m < R; ++m) z[m] = src[zoff<N>(y, t + T * m)];
        line_fft<N, true>(z, xb + line * G::W, tw_s, t);
        if constexpr (DMU) {
          float2* ps = a.psi + (((size_t)j[q] * K + k) * N + y) * N;
#pragma unroll
          for (int m = 0; m < R; ++m) {
            const float2 nw = cmul(pkr[m], o[q][m]) + z[m];
            ps[t + T * m] = nw;
            cacc[q][m] = cacc[q][m] + cconjmul(pkr[m], nw);
          }
        } else {
          float2* ch = a.chi + (((size_t)slot[q] * K + k) * N + y) * N;
#pragma unroll
          for (int m = 0; m < R; ++m) {
            if (a.poisp) z[m] = chi_s[q] * z[m];
            ch[t + T * m] = z[m];
            cacc[q][m] = cacc[q][m] + cconjmul(pkr[m], z[m]);
          }
        }
        // the second pattern's transform after the first's
        __builtin_amdgcn_sched_barrier(0);
      }
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      if (q >= np) break;
      float2* cb = a.contrib + ((size_t)slot[q] * N + y) * N;
#pragma unroll
      for (int m = 0; m < R; ++m) cb[t + T * m] = cacc[q][m];
    }
  }
}

// Step length of the Poisson exit-wave update of each pattern of the chunk:
// the minimiser on [0, 1] of the pattern's likelihood along the ray
// I s^2, s = 1 - alpha g, g = 1 - d / (I + eps): safeguarded Newton steps from
// 1/2 on L'(alpha) = -2 sum I g s (1 - r) and
// L''(alpha) = 2 sum I g^2 (1 - r + 2 r I s^2 / (I s^2 + eps)),
// r = d / (I s^2 + eps) (float32 terms with the hardware reciprocal,
// per-thread float32 and block-wide float64 sums), kept inside the bracket
// the sign of L' maintains (else bisection), stopping once a step moves alpha
// by at most 1e-7; 0 when sum I g^2 = 0.  One block per pattern; masked pixels
// (sign bit of the modulus) take no part.
constexpr int kPoissonSteps = 12;
constexpr int kPoissonThreads = 1024;
template <int N>
__global__ __launch_bounds__(kPoissonThreads) void k_poisson_alpha(FourierArgs a) {
  static_assert((N * N) % (4 * kPoissonThreads) == 0 || N * N < 4 * kPoissonThreads, "pixel quads");
  __shared__ double red[kPoissonThreads / 64];
  __shared__ double sh_a;
  const int c = blockIdx.x;
  const int j = a.jlist[a.jl_off + c];
  const float4* it4 = reinterpret_cast<const float4*>(a.pinten + (size_t)c * N * N);
  const float4* am4 = reinterpret_cast<const float4*>(a.amp + (size_t)j * N * N);
  const float eps = a.nll_eps;
  double lo = 0.0, hi = 1.0, al = 0.5;
  bool done = false;
  for (int step = 0; step < kPoissonSteps && !done; ++step) {
    const float af = (float)al;
    float d1 = 0.f, d2 = 0.f, s0 = 0.f;
    for (int q4 = threadIdx.x; q4 < N * N / 4; q4 += kPoissonThreads) {
      const float4 iv = it4[q4], av = am4[q4];
      const float Is[4] = {iv.x, iv.y, iv.z, iv.w}, As[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (signbit(As[e])) continue;
        const float I = Is[e], d = As[e] * As[e];
        const float g = 1.f - d * __builtin_amdgcn_rcpf(I + eps);
        const float sv = 1.f - af * g;
        const float u = I * sv * sv, rt = __builtin_amdgcn_rcpf(u + eps);
        const float r = d * rt;
        d1 += -2.f * I * g * sv * (1.f - r);
        d2 += 2.f * I * g * g * (1.f - r + 2.f * r * u * rt);
        s0 += I * g * g;
      }
    }
    const double t1 = block_sum<kPoissonThreads>((double)d1, red);
    const double t2 = block_sum<kPoissonThreads>((double)d2, red);
    const double t0 = step == 0 ? block_sum<kPoissonThreads>((double)s0, red) : 1.0;
    if (threadIdx.x == 0) {
      if (step == 0 && !(t0 > 0.0)) {
        al = 0.0;
        done = true;
      } else {
        if (t1 < 0.0)
          lo = al;
        else
          hi = al;
        double nxt = t2 > 0.0 ? al - t1 / t2 : -1.0;
        if (!(lo <= nxt && nxt <= hi)) {
          nxt = 0.5 * (lo + hi);
        } else if (fabs(nxt - al) <= 1e-7) {
          done = true;
        }
        al = nxt;
      }
      sh_a = done ? -1.0 - al : al;   // a negative value carries "done"
    }
    __syncthreads();
    const double v = sh_a;
    __syncthreads();
    if (v < 0.0) {
      al = -1.0 - v;
      done = true;
    } else {
      al = v;
    }
  }
  if (threadIdx.x == 0) a.poisp[a.slot_off + c] = al;
}

}  // namespace

void launch_poisson_alpha(const FourierArgs& a) {
  if (a.nc <= 0) return;
  dispatch_n(a.n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    k_poisson_alpha<N><<<a.nc, kPoissonThreads, 0, a.stream>>>(a);
  });
  PTY_LAUNCH_CHECK("poisson_alpha");
}

int col_blocks(int n, int k) {
  int r = 0;
  dispatch_nk(n, k, [&](auto nc, auto kc) { r = ColSplit<decltype(nc)::value, decltype(kc)::value>::BPP; });
  return r;
}
int row_blocks(int n) {
  int r = 0;
  dispatch_n(n, [&](auto nc) { constexpr int N = decltype(nc)::value; r = N / Geo<N>::LINES; });
  return r;
}

void launch_rows_fwd(const FourierArgs& a, RowIn mode) {
  if (a.nc <= 0) return;
  dispatch_nk(a.n, a.k, [&](auto nc, auto kc) {
    constexpr int N = decltype(nc)::value, K = decltype(kc)::value;
    constexpr int PB = rows_fwd_patterns<N, K>();
    const dim3 grid(N / Geo<N>::LINES, (a.nc + PB - 1) / PB);
    if (mode == RowIn::Plain)
      k_rows_fwd<N, K, RowIn::Plain><<<grid, Geo<N>::BS, 0, a.stream>>>(a);
    else
      k_rows_fwd<N, K, RowIn::DmReflect><<<grid, Geo<N>::BS, 0, a.stream>>>(a);
  });
  PTY_LAUNCH_CHECK("rows_fwd");
}

void launch_cols(const FourierArgs& a, ColOp op) {
  if (a.nc <= 0) return;
  dispatch_nk(a.n, a.k, [&](auto nc, auto kc) {
    constexpr int N = decltype(nc)::value, K = decltype(kc)::value;
    const dim3 grid(ColSplit<N, K>::BPP, a.nc);
    constexpr int BS = Geo<N>::BS;
    if (a.masked) {
      switch (op) {
        case ColOp::Project: k_cols_masked<N, K, ColOp::Project><<<grid, BS, 0, a.stream>>>(a); break;
        case ColOp::NllGrad: k_cols_masked<N, K, ColOp::NllGrad><<<grid, BS, 0, a.stream>>>(a); break;
        case ColOp::Intensity: k_cols<N, K, ColOp::Intensity, false><<<grid, BS, 0, a.stream>>>(a); break;
        case ColOp::NllLoss: k_cols_masked<N, K, ColOp::NllLoss><<<grid, BS, 0, a.stream>>>(a); break;
        case ColOp::Poisson: k_cols_poisson<N, K, true><<<grid, BS, 0, a.stream>>>(a); break;
      }
    } else {
      switch (op) {
        case ColOp::Project: k_cols<N, K, ColOp::Project, false><<<grid, BS, 0, a.stream>>>(a); break;
        case ColOp::NllGrad: k_cols<N, K, ColOp::NllGrad, false><<<grid, BS, 0, a.stream>>>(a); break;
        case ColOp::Intensity: k_cols<N, K, ColOp::Intensity, false><<<grid, BS, 0, a.stream>>>(a); break;
        case ColOp::NllLoss: k_cols<N, K, ColOp::NllLoss, false><<<grid, BS, 0, a.stream>>>(a); break;
        case ColOp::Poisson: k_cols_poisson<N, K, false><<<grid, BS, 0, a.stream>>>(a); break;
      }
    }
  });
  PTY_LAUNCH_CHECK("cols");
}

void launch_rows_inv(const FourierArgs& a, RowOut mode) {
  if (a.nc <= 0) return;
  dispatch_nk(a.n, a.k, [&](auto nc, auto kc) {
    constexpr int N = decltype(nc)::value, K = decltype(kc)::value;
    auto grid = [&](auto mc) {
      constexpr int PB = rows_inv_patterns<N, K, decltype(mc)::value>();
      return dim3(N / Geo<N>::LINES, (a.nc + PB - 1) / PB);
    };
    switch (mode) {
      case RowOut::DmUpdate:
        k_rows_inv<N, K, RowOut::DmUpdate><<<grid(std::integral_constant<RowOut, RowOut::DmUpdate>{}), Geo<N>::BS, 0, a.stream>>>(a);
        break;
      case RowOut::StoreChi:
        k_rows_inv<N, K, RowOut::StoreChi><<<grid(std::integral_constant<RowOut, RowOut::StoreChi>{}), Geo<N>::BS, 0, a.stream>>>(a);
        break;
      case RowOut::NllGrad:
        k_rows_inv<N, K, RowOut::NllGrad><<<grid(std::integral_constant<RowOut, RowOut::NllGrad>{}), Geo<N>::BS, 0, a.stream>>>(a);
        break;
    }
  });
  PTY_LAUNCH_CHECK("rows_inv");
}

}  // namespace pty
