// ePIE positions on 512 x 512 windows, one 64-lane wavefront per line.
//
// ePIE visits the positions one after another (Sec. 2.3; Maiden & Rodenburg
// 2009), so a position's transforms cannot be batched with others: at
// 512 x 512 the chunked passes give one pattern only 32 blocks, each
// wavefront carrying four lines of 512 points.  Here a line belongs to a
// whole wavefront (8 values per lane, three radix-8 stages and two LDS
// exchanges), so every pass spreads over 128 blocks, and the ePIE steps are
// folded into the transforms:
//   rows     : patch S_j O (stored for the probe update), exit waves
//              P_k S_j O, x-transforms; per block the maxima of
//              sum_k |P_k|^2 and |S_j O|^2;
//   cols     : y-transforms of every mode, the multi-mode modulus projection
//              with the amplitude-error partials, inverse y-transforms;
//   rows_inv : the two maxima and the error of the position (reduced in a
//              fixed order), inverse x-transforms, the object-update
//              contribution sum_k conj(P_k) chi_k, the probe update
//              P_k += beta / max|S_j O|^2 conj(S_j O) chi_k (into probe_out)
//              and the object update over the block's rows of the (N+1)^2
//              footprint, O += alpha / max sum_k |P_k|^2 S_j^T (contribution).
// The scratch between passes has the layout of the chunked Fourier passes
// ([x / 4][y][x % 4] per mode), so a block's four columns are one
// contiguous run.
#include "pty_geom.hpp"
#include "pty_kernels.hpp"
#include "pty_wave.hpp"

namespace pty {
namespace {

constexpr int kWN = 512;                 // window side
constexpr int kWNN = kWN * kWN;
constexpr int kWLines = 4;               // lines (wavefronts) per block
constexpr int kWBlocks = kWN / kWLines;  // blocks per pass
constexpr int kWX1 = 72;                 // exchange 1: row stride (8 rows x 8 lanes of a half wavefront on distinct banks)
constexpr int kWXb = 8 * kWX1;           // exchange area per wavefront (float2)
constexpr int kWTile = kWN + 8;          // column tile stride (a wavefront's column and the load's 4 x 8 lanes conflict-free)

__device__ __forceinline__ size_t wzoff(int y, int x) { return ((size_t)(x >> 2) * kWN + y) * 4 + (x & 3); }

// Per-lane twiddles of the two twiddle stages: W_512^(t q) and W_64^((t mod 8) s).
struct WideTw {
  float2 a[7], b[7];
};
__device__ __forceinline__ void wide_twiddles(WideTw& w, const float2* __restrict__ tw, int t) {
#pragma unroll
  for (int q = 1; q < 8; ++q) {
    w.a[q - 1] = tw[(t * q) & (kWN - 1)];
    w.b[q - 1] = tw[(8 * (t & 7) * q) & (kWN - 1)];
  }
}

// Exchange-2 swizzle of row r = 8 s + q (q, s < 8): the write (4 q x 8 lanes)
// and the read (8 q x 4 s) of a half wavefront land on distinct banks.
__device__ __forceinline__ int wide_swz(int r) { return ((r >> 2) & 1) | (((r >> 3) & 3) << 1); }

// One 512-point line transform (unscaled; forward: exp(-2 pi i ...)) held by
// the 64 lanes of a wavefront, lane t owning x[t + 64 m] in v[m] before and
// X[t + 64 m] after.  With n = t + 64 m, k = q + 8 s, t = t1 + 8 t2 and
// s = s1 + 8 s2: X[q + 8 s1 + 64 s2] = sum_t1 W_8^(t1 s2) W_64^(t1 s1)
// sum_t2 W_8^(t2 s1) W_512^(t q) sum_m W_8^(m q) x[t + 64 m].
template <bool INV>
__device__ __forceinline__ void wide_line(float2* v, float2* xb, const WideTw& w, int t) {
  Dft<8, INV>::run(v);
#pragma unroll
  for (int q = 1; q < 8; ++q) {
    float2 c = w.a[q - 1];
    if (INV) c.y = -c.y;
    v[q] = cmul(v[q], c);
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) xb[q * kWX1 + t] = v[q];
  wave_sync();
  const int q = t >> 3, t1 = t & 7;
  float2 u[8];
#pragma unroll
  for (int t2 = 0; t2 < 8; ++t2) u[t2] = xb[q * kWX1 + t1 + 8 * t2];
  wave_sync();
  Dft<8, INV>::run(u);
#pragma unroll
  for (int s1 = 1; s1 < 8; ++s1) {
    float2 c = w.b[s1 - 1];
    if (INV) c.y = -c.y;
    u[s1] = cmul(u[s1], c);
  }
#pragma unroll
  for (int s1 = 0; s1 < 8; ++s1) {
    const int r = 8 * s1 + q;
    xb[8 * r + (t1 ^ wide_swz(r))] = u[s1];
  }
  wave_sync();
  const int r2 = 8 * (t >> 3) + (t & 7), f2 = wide_swz(r2);
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = xb[8 * r2 + (i ^ f2)];
  wave_sync();
  Dft<8, INV>::run(v);
}

template <int K>
__global__ __launch_bounds__(256) void k_epw_rows(EpieWideArgs a) {
  __shared__ float2 xb[kWLines][kWXb];
  __shared__ float red[kWLines][2];
  const int wv = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int y = blockIdx.x * kWLines + wv;
  WideTw w;
  wide_twiddles(w, reinterpret_cast<const float2*>(a.tw), t);
  const PosInfo p = a.pos;
  // every global load first (probe pixels and the bilinear taps), so their
  // latencies overlap; the stores come after
  float2 pk[K][8];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float2* __restrict__ pr = a.probe + ((size_t)k * kWN + y) * kWN;
#pragma unroll
    for (int m = 0; m < 8; ++m) pk[k][m] = pr[t + 64 * m];
  }
  float2 o[8];
  float om = 0.f, pm = 0.f;
  float sp[8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    o[m] = obj_bilinear(a.obj, a.h, a.w, p, y, t + 64 * m);
    om = fmaxf(om, cabs2(o[m]));
    sp[m] = 0.f;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    float2 z[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      sp[m] += cabs2(pk[k][m]);
      z[m] = cmul(pk[k][m], o[m]);
    }
    wide_line<false>(z, xb[wv], w, t);
    float2* dst = a.zs + (size_t)k * kWNN;
#pragma unroll
    for (int m = 0; m < 8; ++m) dst[wzoff(y, t + 64 * m)] = z[m];
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) a.patch[(size_t)y * kWN + t + 64 * m] = o[m];
#pragma unroll
  for (int m = 0; m < 8; ++m) pm = fmaxf(pm, sp[m]);
  pm = wave_max_nonneg(pm);
  om = wave_max_nonneg(om);
  if (t == 0) {
    red[wv][0] = pm;
    red[wv][1] = om;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    float mx = 0.f;
#pragma unroll
    for (int i = 0; i < kWLines; ++i) mx = fmaxf(mx, red[i][threadIdx.x]);
    a.maxw[2 * blockIdx.x + threadIdx.x] = mx;
  }
}

template <int K, bool MASK>
__global__ __launch_bounds__(256) void k_epw_cols(EpieWideArgs a) {
  __shared__ float2 tile[K][4][kWTile];
  __shared__ float amt[4][kWTile];
  __shared__ float2 xb[kWLines][kWXb];
  __shared__ double red[kWLines][2];
  const int wv = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int x0 = blockIdx.x * 4;
  WideTw w;
  wide_twiddles(w, reinterpret_cast<const float2*>(a.tw), t);
  // the block's four columns of every mode: one contiguous run of 4 x 512
  // values; the moduli of those columns: 16 bytes of every row
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float2* src = a.zs + (size_t)k * kWNN + (size_t)x0 * kWN;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = threadIdx.x + 256 * r;
      tile[k][e & 3][e >> 2] = src[e];
    }
  }
  {
    const float* am = a.amp + (size_t)a.j * kWNN + x0;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int yy = threadIdx.x + 256 * r;
      const float4 v4 = *reinterpret_cast<const float4*>(am + (size_t)yy * kWN);
      amt[0][yy] = v4.x;
      amt[1][yy] = v4.y;
      amt[2][yy] = v4.z;
      amt[3][yy] = v4.w;
    }
  }
  __syncthreads();
  float2 z[K][8];
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int m = 0; m < 8; ++m) z[k][m] = tile[k][wv][t + 64 * m];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) wide_line<false>(z[k], xb[wv], w, t);
  // the transforms are unscaled: the unitary far field is z / N and the
  // unitary inverse of the whole pipeline contributes another 1 / N^2
  constexpr float sc = 1.0f / kWN, sc2 = 1.0f / (float(kWN) * float(kWN));
  float en = 0.f, ed = 0.f;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    float iraw = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) iraw += cabs2(z[k][m]);
    const float ar = amt[wv][t + 64 * m];
    float mf = 1.f, am = ar;
    if constexpr (MASK) {
      mf = signbit(ar) ? 0.f : 1.f;   // sign bit: no measurement
      am = fabsf(ar);
    }
    // hardware square root and reciprocal (within 1 ulp each)
    const float mod = __builtin_amdgcn_sqrtf(iraw) * sc;
    float f = am * __builtin_amdgcn_rcpf(fmaxf(mod, 1e-6f)) - 1.f;
    if constexpr (MASK) f *= mf;
    en += mf * ((mod - am) * (mod - am));
    ed += mf * (am * am);
    f *= sc2;
#pragma unroll
    for (int k = 0; k < K; ++k) z[k][m] = f * z[k][m];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    wide_line<true>(z[k], xb[wv], w, t);
#pragma unroll
    for (int m = 0; m < 8; ++m) tile[k][wv][t + 64 * m] = z[k][m];
  }
  const double s0 = wave_sum_d(en), s1 = wave_sum_d(ed);
  if (t == 0) {
    red[wv][0] = s0;
    red[wv][1] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double e0 = 0.0, e1 = 0.0;
#pragma unroll
    for (int i = 0; i < kWLines; ++i) {
      e0 += red[i][0];
      e1 += red[i][1];
    }
    a.errw[2 * blockIdx.x] = e0;
    a.errw[2 * blockIdx.x + 1] = e1;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    float2* dst = a.zs + (size_t)k * kWNN + (size_t)x0 * kWN;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = threadIdx.x + 256 * r;
      dst[e] = tile[k][e & 3][e >> 2];
    }
  }
}

// Inverse rows and the object update in one launch: a block transforms its
// four rows and the row above them (whose contribution the footprint rows
// need), keeps the five contribution rows in LDS and updates footprint rows
// 4 b .. 4 b + 3 (the last block also row N).  The probe update goes to
// probe_out (the row above belongs to another block, which must still read
// the old probe).
constexpr int kWInvWaves = kWLines + 1;
template <int K>
__global__ __launch_bounds__(64 * kWInvWaves) void k_epw_rows_inv_obj(EpieWideArgs a) {
  __shared__ float2 xb[kWInvWaves][kWXb];
  __shared__ float2 crow[kWInvWaves][kWN + 1];      // contribution rows y0 - 1 .. y0 + 3 (column N: zero)
  __shared__ float redf[kWInvWaves][2];
  __shared__ double redd[2][2];
  const int wv = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int y0 = blockIdx.x * kWLines;
  const int y = y0 - 1 + wv;                         // wave 0: the row above the block
  constexpr int kTh = 64 * kWInvWaves;
  constexpr int kOpt = ((kWLines + 1) * (kWN + 1) + kTh - 1) / kTh;   // footprint pixels per thread
  const PosInfo p = a.pos;
  const int rows = (blockIdx.x == kWBlocks - 1) ? kWLines + 1 : kWLines;
  // the old object under this block's footprint rows, fetched first
  float2 ov[kOpt];
#pragma unroll
  for (int i = 0; i < kOpt; ++i) {
    const int e = threadIdx.x + i * kTh, r = e / (kWN + 1), v = e % (kWN + 1);
    const int Y = p.iy + y0 + r, X = p.ix + v;
    ov[i] = (r < rows && Y < a.h && X < a.w) ? a.obj[(size_t)Y * a.w + X] : make_float2(0.f, 0.f);
  }
  // this wavefront's row: scratch, old probe and pre-update patch, fetched
  // before the reductions below
  const bool live = y >= 0;
  const int yl = live ? y : 0;
  float2 z[K][8], pk[K][8], o[8];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float2* src = a.zs + (size_t)k * kWNN;
    const float2* __restrict__ pr = a.probe + ((size_t)k * kWN + yl) * kWN;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      z[k][m] = src[wzoff(yl, t + 64 * m)];
      pk[k][m] = pr[t + 64 * m];
    }
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) o[m] = a.patch[(size_t)yl * kWN + t + 64 * m];
  WideTw w;
  wide_twiddles(w, reinterpret_cast<const float2*>(a.tw), t);
  // the two maxima over the row blocks of the forward pass
  float pm = 0.f, om = 0.f;
  for (int i = threadIdx.x; i < kWBlocks; i += 64 * kWInvWaves) {
    pm = fmaxf(pm, a.maxw[2 * i]);
    om = fmaxf(om, a.maxw[2 * i + 1]);
  }
  pm = wave_max_nonneg(pm);
  om = wave_max_nonneg(om);
  if (t == 0) {
    redf[wv][0] = pm;
    redf[wv][1] = om;
  }
  if (blockIdx.x == 0 && wv < 2) {
    // this position's error: the column blocks' sums (two per lane, then the
    // wavefront in a fixed order)
    const double e = a.errw[2 * t + wv] + a.errw[2 * (t + 64) + wv];
    const double s = wave_sum_d(e);
    if (t == 0) redd[0][wv] = s;
  }
  __syncthreads();
  float pmax = 0.f, omax = 0.f;
#pragma unroll
  for (int i = 0; i < kWInvWaves; ++i) {
    pmax = fmaxf(pmax, redf[i][0]);
    omax = fmaxf(omax, redf[i][1]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double* e = a.errp + (size_t)a.j * a.bpp * 2;
    e[0] = redd[0][0];
    e[1] = redd[0][1];
    for (int cb = 1; cb < a.bpp; ++cb) e[2 * cb] = e[2 * cb + 1] = 0.0;
  }
  if (live) {
    const bool own = wv > 0;
    const float bs = (own && a.probe_on && omax > 0.f) ? a.beta / omax : 0.f;
    float2 cn[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) cn[m] = make_float2(0.f, 0.f);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      float2* po = a.probe_out + ((size_t)k * kWN + y) * kWN;
      wide_line<true>(z[k], xb[wv], w, t);
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        cn[m] = cn[m] + cconjmul(pk[k][m], z[k][m]);
        if (own && (a.probe_out != a.probe || bs != 0.f)) po[t + 64 * m] = pk[k][m] + bs * cconjmul(o[m], z[k][m]);
      }
    }
#pragma unroll
    for (int m = 0; m < 8; ++m) crow[wv][t + 64 * m] = cn[m];
  } else {
#pragma unroll
    for (int m = 0; m < 8; ++m) crow[wv][t + 64 * m] = make_float2(0.f, 0.f);
  }
  if (t == 0) crow[wv][kWN] = make_float2(0.f, 0.f);
  __syncthreads();
  // object update over footprint rows u = y0 .. y0 + 3 (and N in the last block)
  if (!(pmax > 0.f)) return;
  const float as = a.alpha / pmax;
  const float wx0 = 1.f - p.fx, wx1 = p.fx, wy0 = 1.f - p.fy, wy1 = p.fy;
#pragma unroll
  for (int i = 0; i < kOpt; ++i) {
    const int e = threadIdx.x + i * kTh, r = e / (kWN + 1), v = e % (kWN + 1);
    const int Y = p.iy + y0 + r, X = p.ix + v;
    if (r >= rows || Y >= a.h || X >= a.w) continue;
    // rows u (crow[r + 1], zero at u = N) and u - 1 (crow[r]); column v - 1 zero at v = 0
    const float2 zero = make_float2(0.f, 0.f);
    const float2 c00 = r + 1 < kWInvWaves ? crow[r + 1][v] : zero;
    const float2 c01 = (r + 1 < kWInvWaves && v > 0) ? crow[r + 1][v - 1] : zero;
    const float2 c10 = crow[r][v];
    const float2 c11 = v > 0 ? crow[r][v - 1] : zero;
    const float2 sv = wy0 * (wx0 * c00 + wx1 * c01) + wy1 * (wx0 * c10 + wx1 * c11);
    a.obj[(size_t)Y * a.w + X] = ov[i] + as * sv;
  }
}

}  // namespace

bool epie_wide_supported(int n, int k) { return n == kWN && k >= 1 && k <= 2; }

size_t epie_wide_max_words() { return 2 * (size_t)kWBlocks; }
size_t epie_wide_err_words() { return 2 * (size_t)kWBlocks; }

void launch_epie_wide(const EpieWideArgs& a) {
  if (!epie_wide_supported(a.n, a.k)) throw std::invalid_argument("wide ePIE: unsupported window");
  auto go = [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    k_epw_rows<K><<<kWBlocks, 256, 0, a.stream>>>(a);
    if (a.masked)
      k_epw_cols<K, true><<<kWBlocks, 256, 0, a.stream>>>(a);
    else
      k_epw_cols<K, false><<<kWBlocks, 256, 0, a.stream>>>(a);
    k_epw_rows_inv_obj<K><<<kWBlocks, 64 * kWInvWaves, 0, a.stream>>>(a);
  };
  if (a.k == 1) go(ic<1>{});
  else go(ic<2>{});
  PTY_LAUNCH_CHECK("epie_wide");
}

}  // namespace pty
