// Object and probe updates, LSQML step lengths, ePIE update, reductions.
//
// Object planes are accumulated in gather form: every object tile walks the
// list of patches that overlap it and sums their per-pattern contributions
// through the bilinear adjoint S_j^T, in a fixed order.  No float atomics are
// used (their throughput on MI355X is far below the HBM stream rate), and the
// result is bit-for-bit reproducible run to run.
// Methods: DM overlap projection (Thibault et al. 2009), LSQML directions and
// per-position steps (Odstrcil et al. 2018), ePIE (Maiden & Rodenburg 2009);
// all three named in Sec. 2.3.
#include "pty_geom.hpp"
#include "pty_kernels.hpp"
#include "pty_wave.hpp"

namespace pty {
namespace {

// ---------------------------------------------------------------------------
// Object tiles: sum_j S_j^T (.) in gather form, then the algorithm's update
// ---------------------------------------------------------------------------
// One block of four wavefronts per 16 x 64 tile (8 or 16 on grids too small
// to fill the chip); lane = column, and the wavefronts split the tile's
// patch list.  For each patch the thread walks its
// column downwards: the horizontal combination of patch row u (taps v and
// v - 1) is computed once and used for object rows u and u + 1, so each patch
// row is read once per tile column.
template <typename V>
struct Zero;
template <>
struct Zero<float> { __device__ static float v() { return 0.f; } };
template <>
struct Zero<float2> { __device__ static float2 v() { return make_float2(0.f, 0.f); } };

__device__ __forceinline__ float2 axpy(float a, float2 x, float2 y) { return make_float2(fmaf(a, x.x, y.x), fmaf(a, x.y, y.y)); }
__device__ __forceinline__ float axpy(float a, float x, float y) { return fmaf(a, x, y); }


// The value of lane i - 1 (lane 0: `first`), by a wavefront-wide DPP shift.
__device__ __forceinline__ float lane_shr1(float x, float first) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(first), __float_as_int(x), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float2 lane_shr1(float2 x, float2 first) {
  return make_float2(lane_shr1(x.x, first.x), lane_shr1(x.y, first.y));
}
// Lane l's value of x (l wavefront-uniform), for every lane.
__device__ __forceinline__ float lane_value(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ float2 lane_value(float2 x, int l) {
  return make_float2(lane_value(x.x, l), lane_value(x.y, l));
}
// Horizontal combination of patch row u at columns v (weight w0) and v - 1
// (weight w1), for a wavefront whose lanes are consecutive columns: one
// vector load of column v per lane; column v - 1 is the neighbouring lane's
// value, and lane 0's (column v1c0) is `left`, loaded for all of a patch's
// rows at once.  Branch-free: indices are clamped into the plane and the
// weights are zero where a tap falls outside it, so the loads of all rows
// can be issued together.
template <int N, typename V>
__device__ __forceinline__ V hrow_wave(const V* __restrict__ src, int u, int v0c, V left, float w0, float w1) {
  const float uok = (unsigned)u < (unsigned)N ? 1.f : 0.f;
  const V* r = src + min(max(u, 0), N - 1) * N;
  const V c0 = r[v0c];
  const V c1 = lane_shr1(c0, left);
  return axpy(w1 * uok, c1, axpy(w0 * uok, c0, Zero<V>::v()));
}


// NW wavefronts per tile (wave w takes every NW-th patch): 4, or 8 or 16
// where the grid has too few tiles to fill the chip and each tile's list is
// walked by more waves.
template <int N, ObjOp OP, int NW>
__global__ __launch_bounds__(64 * NW) void k_obj_gather(ObjGatherArgs a) {
  using V = typename std::conditional<OP == ObjOp::Density, float, float2>::type;
  constexpr int TH = kTileH;
  static_assert(TH % NW == 0, "each wave applies whole rows");
  __shared__ V part[NW - 1][TH][kTileW];
  __shared__ float redf[NW];
  const TileEntry te = a.tiles[blockIdx.x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int X = te.tx + lane;
  V acc[TH];
#pragma unroll
  for (int i = 0; i < TH; ++i) acc[i] = Zero<V>::v();
  int e = te.beg + wv;
  PatchRef rn = e < te.end ? a.refs[e] : PatchRef{};
  for (; e < te.end; e += NW) {
    const PatchRef r = rn;
    if (e + NW < te.end) rn = a.refs[e + NW];   // the next patch's entry, while this one is summed
    float wgt = 1.f;
    if constexpr (OP == ObjOp::LsqUpdate || OP == ObjOp::WeightedSum) wgt = a.alpha[r.slot].x;
    const V* src;
    if constexpr (OP == ObjOp::Density)
      src = a.pint;
    else
      src = a.src + (size_t)r.slot * N * N;
    const int v = X - r.ix;
    const float w0 = (unsigned)v < (unsigned)N ? 1.f - r.fx : 0.f;
    const float w1 = (unsigned)(v - 1) < (unsigned)N ? r.fx : 0.f;
    // lane i's column v - 1 is lane i - 1's column v (the lanes are
    // consecutive columns), lane 0's is te.tx - 1 - r.ix
    const int v0c = min(max(v, 0), N - 1), v1c0 = min(max(te.tx - 1 - r.ix, 0), N - 1);
    const float wy0 = wgt * (1.f - r.fy), wy1 = wgt * r.fy;
    const int u0 = te.ty - r.iy;
    // lane k <= TH loads column v1c0 of patch row u0 - 1 + k: every row's
    // tap left of the tile in one vector load, handed to lane 0 per row
    static_assert(TH + 1 <= 64, "one lane per patch row");
    const V* rk = src + min(max(u0 - 1 + min(lane, TH), 0), N - 1) * N;
    const V left = rk[v1c0];
    V prev = hrow_wave<N, V>(src, u0 - 1, v0c, lane_value(left, 0), w0, w1);
#pragma unroll
    for (int i = 0; i < TH; ++i) {
      const V cur = hrow_wave<N, V>(src, u0 + i, v0c, lane_value(left, i + 1), w0, w1);
      acc[i] = axpy(wy0, cur, axpy(wy1, prev, acc[i]));
      prev = cur;
    }
  }
  // combine the wavefronts' partial sums in a fixed order (wave 0 + 1 + ...)
  if (wv > 0) {
#pragma unroll
    for (int i = 0; i < TH; ++i) part[wv - 1][i][lane] = acc[i];
  }
  __syncthreads();
  // each wave applies TH / NW rows of the tile
  float mx = 0.f;
  float delta = 0.f;
  constexpr bool RAW = OP == ObjOp::Gradient || OP == ObjOp::WeightedSum;
  if constexpr (OP != ObjOp::Density && !RAW) delta = a.gamma * __uint_as_float(*a.den_max);
  if (wv == 0) {
#pragma unroll
    for (int i = 0; i < TH; ++i) {
#pragma unroll
      for (int w = 0; w < NW - 1; ++w) acc[i] = acc[i] + part[w][i][lane];
      part[0][i][lane] = acc[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int ii = 0; ii < TH / NW; ++ii) {
    const int i = wv * (TH / NW) + ii;
    const V val = part[0][i][lane];
    const int Y = te.ty + i;
    if (Y >= a.h || X >= a.w) continue;
    const size_t o = (size_t)Y * a.w + X;
    if constexpr (OP == ObjOp::Density) {
      a.den[o] = val;
      mx = fmaxf(mx, val);
    } else if constexpr (RAW) {
      a.out[o] = val;
    } else {
      const float d = a.den[o] + delta;
      if constexpr (OP == ObjOp::DmObject) {
        if (d > 0.f) {
          const float2 ov = a.obj[o];
          a.obj[o] = (1.f / d) * (val + delta * ov);
        }
      } else if constexpr (OP == ObjOp::LsqDirection) {
        a.out[o] = d > 0.f ? (1.f / d) * val : make_float2(0.f, 0.f);
      } else {
        if (d > 0.f) a.obj[o] = a.obj[o] + (a.beta / d) * val;
      }
    }
  }
  if constexpr (OP == ObjOp::Density) {
    mx = block_max_all<64 * NW>(mx, redf);
    if (threadIdx.x == 0) atomicMax(a.den_max, __float_as_uint(mx));
  }
}

// ---------------------------------------------------------------------------
// Probe reductions over positions: sum_j w_j conj(S_j O) src_jk and sum_j |S_j O|^2
// ---------------------------------------------------------------------------
// Pixel mapping shared by the probe sums and the LSQML step sums: a block of
// 256 threads covers G = 256 / TPR groups of TPR = min(N, 256) consecutive
// columns; thread (column v, group) walks RB consecutive rows u0 .. u0 + RB - 1,
// so the object rows under a patch are read once and used for two bilinear
// rows.  Windows wider than 256 take CB = N / 256 blocks per row band.
template <int N, int RB>
struct ColWalk {
  static constexpr int TPR = N < 256 ? N : 256;   // threads per row segment
  static constexpr int CB = N / TPR;              // column blocks per row band
  static constexpr int G = 256 / TPR;             // row groups per block
  static constexpr int ROWS = G * RB;             // rows per block
  static constexpr int BLOCKS = N / ROWS * CB;    // blocks per window
  static_assert(N % ROWS == 0 && N % TPR == 0 && BLOCKS >= 1, "window must tile");
  __device__ static int col(int rblk) { return (rblk % CB) * TPR + (int)threadIdx.x % TPR; }
  __device__ static int row0(int rblk) { return ((rblk / CB) * G + (int)threadIdx.x / TPR) * RB; }
};

// Horizontal bilinear combination of object row r at columns c0, c0 + 1
// (the second clamped; it then has zero weight, as in obj_bilinear).
__device__ __forceinline__ float2 obj_hrow(const float2* __restrict__ o, int h, int w, int r, int c0, float wx0,
                                           float wx1) {
  r = min(r, h - 1);
  const int c1 = min(c0 + 1, w - 1);
  const float2 a = o[(size_t)r * w + c0], b = o[(size_t)r * w + c1];
  return make_float2(wx0 * a.x + wx1 * b.x, wx0 * a.y + wx1 * b.y);
}

template <int N>
struct ProbePix {
  static constexpr int RB = 4;
  using W = ColWalk<N, RB>;
};
constexpr int kProbeSliceMax = 32;   // patterns per slice (probe_per_slice)

// A block sums the patterns of one slice for its pixels.  The slice's
// positions (and weights) are staged in LDS first, so that no pattern's
// object reads wait behind a chain of list and position loads, and the next
// pattern's source rows are loaded while the current one is summed.
template <int N, int K, PrbOp OP>
__global__ __launch_bounds__(256) void k_probe_acc(ProbeAccArgs a) {
  using W = typename ProbePix<N>::W;
  constexpr int RB = ProbePix<N>::RB;
  __shared__ PosInfo sp[kProbeSliceMax];
  __shared__ float sw[kProbeSliceMax];
  __shared__ int ss[kProbeSliceMax];
  const int slice = blockIdx.y, rblk = blockIdx.x;
  if (a.zero && slice == 0 && rblk == 0 && threadIdx.x == 0) *a.zero = 0u;
  const int s_beg = a.s0 + slice * a.per_slice;
  const int ns = min(a.per_slice, a.s0 + a.count - s_beg);
  if ((int)threadIdx.x < ns) {
    const int s = s_beg + threadIdx.x;
    const int j = a.jlist[s];
    sp[threadIdx.x] = a.pos[j];
    float w = 1.f;
    if constexpr (OP == PrbOp::AlphaWeighted) w = a.alpha[s].y;
    if constexpr (OP == PrbOp::Gradient) w = 2.f;
    sw[threadIdx.x] = w;
    ss[threadIdx.x] = a.src_by_pattern ? j : s;
  }
  __syncthreads();
  const int v = W::col(rblk);
  const int u0 = W::row0(rblk);
  float2 num[K][RB];
  float den[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    den[i] = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) num[k][i] = make_float2(0.f, 0.f);
  }
  float2 cur[K][RB], nxt[K][RB];
  auto load_src = [&](int m, float2 (&x)[K][RB]) {
    const float2* src = a.src + (size_t)ss[m] * K * N * N + u0 * N + v;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int i = 0; i < RB; ++i) x[k][i] = src[(size_t)k * N * N + i * N];
  };
  if (ns > 0) load_src(0, cur);
  for (int m = 0; m < ns; ++m) {
    if (m + 1 < ns) load_src(m + 1, nxt);
    const PosInfo p = sp[m];
    const float w = sw[m];
    const float wx0 = 1.f - p.fx, wx1 = p.fx, wy0 = 1.f - p.fy, wy1 = p.fy;
    float2 top = obj_hrow(a.obj, a.h, a.w, p.iy + u0, p.ix + v, wx0, wx1);
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const float2 bot = obj_hrow(a.obj, a.h, a.w, p.iy + u0 + i + 1, p.ix + v, wx0, wx1);
      const float2 o = make_float2(wy0 * top.x + wy1 * bot.x, wy0 * top.y + wy1 * bot.y);
      top = bot;
      if constexpr (OP == PrbOp::Plain) den[i] += cabs2(o);
      const float2 ow = w * o;
#pragma unroll
      for (int k = 0; k < K; ++k) num[k][i] = num[k][i] + cconjmul(ow, cur[k][i]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int i = 0; i < RB; ++i) cur[k][i] = nxt[k][i];
  }
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    const int q = (u0 + i) * N + v;
#pragma unroll
    for (int k = 0; k < K; ++k) a.part_num[((size_t)slice * K + k) * N * N + q] = num[k][i];
    if constexpr (OP == PrbOp::Plain) a.part_den[(size_t)slice * N * N + q] = den[i];
  }
}

// One thread per (pixel, mode): the mode is blockIdx.y, so a launch has
// K times as many blocks as the window has pixel blocks; the density and its
// maximum come from the mode-0 blocks.
__global__ __launch_bounds__(256) void k_probe_finish(ProbeFinishArgs a) {
  __shared__ float redf[4];
  const int nn = a.n * a.n;
  const int q = blockIdx.x * 256 + threadIdx.x;
  const int k = blockIdx.y;
  float dv = 0.f;
  if (q < nn) {
    float2 s = make_float2(0.f, 0.f);
#pragma unroll 8
    for (int sl = 0; sl < a.slices; ++sl) s = s + a.part_num[((size_t)sl * a.k + k) * nn + q];
    a.num[(size_t)k * nn + q] = s;
    if (k == 0 && a.part_den) {
#pragma unroll 8
      for (int sl = 0; sl < a.slices; ++sl) dv += a.part_den[(size_t)sl * nn + q];
      a.den[q] = dv;
    }
  }
  if (k == 0 && a.den_max) {
    const float mx = block_max_all<256>(dv, redf);
    if (threadIdx.x == 0) atomicMax(a.den_max, __float_as_uint(mx));
  }
}

template <PrbApply OP>
__global__ __launch_bounds__(256) void k_probe_apply(ProbeApplyArgs a) {
  const int nn = a.n * a.n;
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= nn) return;
  const float delta = a.gamma * __uint_as_float(*a.den_max);
  const float d = a.den[q] + delta;
  for (int k = 0; k < a.k; ++k) {
    const size_t o = (size_t)k * nn + q;
    if constexpr (OP == PrbApply::Dm) {
      if (d > 0.f) a.probe[o] = (1.f / d) * (a.num[o] + delta * a.probe[o]);
    } else if constexpr (OP == PrbApply::LsqDirection) {
      a.dir[o] = d > 0.f ? (1.f / d) * a.num[o] : make_float2(0.f, 0.f);
    } else {
      if (d > 0.f) a.probe[o] = a.probe[o] + (a.beta / d) * a.num[o];
    }
  }
}

// ---------------------------------------------------------------------------
// LSQML per-position step lengths (pass B)
// ---------------------------------------------------------------------------
template <int N>
struct LsqPix {
  static constexpr int RB = 4;          // rows per thread
  static constexpr int M = 8;           // positions per block
  using W = ColWalk<N, RB>;
  static constexpr int NRB = W::BLOCKS;
};

// Object taps O[r][c0], O[r][c0 + 1] for the position derivatives, zero past
// the object's last row or column (only a patch at an integer position on the
// far edge reaches them).
__device__ __forceinline__ void obj_taps(const float2* __restrict__ o, int h, int w, int r, int c0, float2& a,
                                         float2& b) {
  const bool rin = r < h, bin = rin && c0 + 1 < w;
  const size_t row = (size_t)min(r, h - 1) * w;
  a = o[row + c0];
  b = o[row + min(c0 + 1, w - 1)];
  if (!rin) a = make_float2(0.f, 0.f);
  if (!bin) b = make_float2(0.f, 0.f);
}

// Per-pixel probe quantities of one LSQML group: sum_k |P_k|^2,
// sum_k conj(P_k) dP_k and sum_k |dP_k|^2.
__global__ __launch_bounds__(256) void k_lsq_planes(const float2* probe, const float2* dprobe, int n, int k,
                                                    int probe_on, float* pint, float2* pq, float* dint) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  const int nn = n * n;
  if (q >= nn) return;
  float a = 0.f, d = 0.f;
  float2 c = make_float2(0.f, 0.f);
  for (int i = 0; i < k; ++i) {
    const float2 pk = probe[(size_t)i * nn + q];
    a += cabs2(pk);
    if (probe_on) {
      const float2 dk = dprobe[(size_t)i * nn + q];
      d += cabs2(dk);
      c = c + cconjmul(pk, dk);
    }
  }
  pint[q] = a;
  pq[q] = c;
  dint[q] = d;
}

// Five sums of one (position, row block): with a_k = P_k S dO, b_k = dP_k S O,
// |a|^2 = |S dO|^2 sum|P_k|^2, |b|^2 = |S O|^2 sum|dP_k|^2,
// Re conj(a) b = Re conj(S dO) S O sum conj(P_k) dP_k,
// Re conj(a) chi = Re conj(S dO) sum_k conj(P_k) chi_k (the stored contribution),
// Re conj(b) chi = Re conj(S O) sum_k conj(dP_k) chi_k.
// With POS, four more for the position refinement: with g = d(S O)/dy (and
// likewise x) and d psi_k = P_k g, Re sum_k conj(d psi_k) chi_k =
// Re conj(g) sum_k conj(P_k) chi_k and sum_k |d psi_k|^2 = |g|^2 sum_k |P_k|^2.
// A block takes one row band of M positions: the probe planes of its pixels
// (sum_k |P_k|^2, sum_k conj(P_k) dP_k, sum_k |dP_k|^2 and dP_k) are read
// once into registers and serve all M; the positions come from LDS.  Each
// wavefront reduces its sums with lane shuffles; the four wavefronts' sums are
// added in a fixed order at the end.
// M positions per block: LsqPix<N>::M, or 2 where a launch would have too
// few blocks to fill the chip (the partials, one per position and row block,
// are the same either way).
template <int N, int K, bool PROBE_ON, bool POS, int M>
__global__ __launch_bounds__(256) void k_lsq_sums(LsqStepArgs a) {
  using W = typename LsqPix<N>::W;
  constexpr int RB = LsqPix<N>::RB;
  constexpr int NV = POS ? 9 : 5;
  constexpr int KP = PROBE_ON ? K : 1;
  __shared__ PosInfo sp[M];
  __shared__ double red[M][4][NV];
  const int rblk = blockIdx.x, b0 = blockIdx.y * M;
  const int nb = min(M, a.count - b0);
  if ((int)threadIdx.x < nb) sp[threadIdx.x] = a.pos[a.jlist[b0 + threadIdx.x]];
  const int v = W::col(rblk);
  const int u0 = W::row0(rblk);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  float pint[RB], dint[RB];
  float2 pq[RB], dp[KP][RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    const int q = (u0 + i) * N + v;
    pint[i] = a.pint[q];
    if constexpr (PROBE_ON) {
      dint[i] = a.dint[q];
      pq[i] = a.pq[q];
#pragma unroll
      for (int k = 0; k < K; ++k) dp[k][i] = a.dprobe[(size_t)k * N * N + q];
    }
  }
  __syncthreads();
  for (int mi = 0; mi < nb; ++mi) {
    const int b = b0 + mi;
    const PosInfo p = sp[mi];
    const float wx0 = 1.f - p.fx, wx1 = p.fx, wy0 = 1.f - p.fy, wy1 = p.fy;
    float m00 = 0.f, m11 = 0.f, m01 = 0.f, v0 = 0.f, v1 = 0.f;
    float ny = 0.f, nx = 0.f, gyy = 0.f, gxx = 0.f;
    float2 cb[RB], ch[KP][RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int q = (u0 + i) * N + v;
      cb[i] = a.contrib[(size_t)b * N * N + q];
      if constexpr (PROBE_ON) {
#pragma unroll
        for (int k = 0; k < K; ++k) ch[k][i] = a.chi[((size_t)b * K + k) * N * N + q];
      }
    }
    float2 dtop = obj_hrow(a.dobj, a.h, a.w, p.iy + u0, p.ix + v, wx0, wx1);
    float2 otop = make_float2(0.f, 0.f);
    if constexpr (PROBE_ON) otop = obj_hrow(a.obj, a.h, a.w, p.iy + u0, p.ix + v, wx0, wx1);
    float2 ta = make_float2(0.f, 0.f), tb = make_float2(0.f, 0.f);
    if constexpr (POS) obj_taps(a.obj, a.h, a.w, p.iy + u0, p.ix + v, ta, tb);
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const float2 dbot = obj_hrow(a.dobj, a.h, a.w, p.iy + u0 + i + 1, p.ix + v, wx0, wx1);
      const float2 dob = make_float2(wy0 * dtop.x + wy1 * dbot.x, wy0 * dtop.y + wy1 * dbot.y);
      dtop = dbot;
      m00 += cabs2(dob) * pint[i];
      v0 += dob.x * cb[i].x + dob.y * cb[i].y;
      if constexpr (POS) {
        float2 ba, bb;
        obj_taps(a.obj, a.h, a.w, p.iy + u0 + i + 1, p.ix + v, ba, bb);
        // d/dy: bottom minus top row, each interpolated along x;
        // d/dx: right minus left tap, interpolated along y
        const float2 gy = make_float2(wx0 * (ba.x - ta.x) + wx1 * (bb.x - tb.x), wx0 * (ba.y - ta.y) + wx1 * (bb.y - tb.y));
        const float2 gx = make_float2(wy0 * (tb.x - ta.x) + wy1 * (bb.x - ba.x), wy0 * (tb.y - ta.y) + wy1 * (bb.y - ba.y));
        ta = ba;
        tb = bb;
        ny += gy.x * cb[i].x + gy.y * cb[i].y;
        nx += gx.x * cb[i].x + gx.y * cb[i].y;
        gyy += cabs2(gy) * pint[i];
        gxx += cabs2(gx) * pint[i];
      }
      if constexpr (PROBE_ON) {
        const float2 obot = obj_hrow(a.obj, a.h, a.w, p.iy + u0 + i + 1, p.ix + v, wx0, wx1);
        const float2 ob = make_float2(wy0 * otop.x + wy1 * obot.x, wy0 * otop.y + wy1 * obot.y);
        otop = obot;
        m11 += cabs2(ob) * dint[i];
        const float2 dc = cconjmul(dob, ob);  // conj(S dO) S O
        m01 += dc.x * pq[i].x - dc.y * pq[i].y;   // Re(dc * pq)
        float2 t = make_float2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < K; ++k) t = t + cconjmul(dp[k][i], ch[k][i]);
        v1 += ob.x * t.x + ob.y * t.y;        // Re(conj(S O) t)
      }
    }
    double sv[NV];
    sv[0] = m00;
    sv[1] = m11;
    sv[2] = m01;
    sv[3] = v0;
    sv[4] = v1;
    if constexpr (POS) {
      sv[5] = ny;
      sv[6] = nx;
      sv[7] = gyy;
      sv[8] = gxx;
    }
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) sv[i] += __shfl_down(sv[i], off, 64);
    if (lane == 0)
#pragma unroll
      for (int i = 0; i < NV; ++i) red[mi][wid][i] = sv[i];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nb * NV; t += 256) {
    const int mi = t / NV, i = t % NV;
    a.part[((size_t)(b0 + mi) * LsqPix<N>::NRB + rblk) * NV + i] =
        red[mi][0][i] + red[mi][1][i] + red[mi][2][i] + red[mi][3][i];
  }
}

// One wavefront per position: lane r sums row-block partials r, r + 64, ...
// (coalesced across the lanes), the wavefront adds the lanes' sums in a fixed
// DPP order, lane 0 solves.
constexpr int kLsqSolveWaves = 4;
template <int NV>
__device__ __forceinline__ void lsq_solve_one(const LsqStepArgs& a, int b, int nrb) {
  const int lane = threadIdx.x & 63;
  double s[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) s[i] = 0.0;
  for (int r = lane; r < nrb; r += 64) {
    const double* pp = a.part + ((size_t)b * nrb + r) * NV;
#pragma unroll
    for (int i = 0; i < NV; ++i) s[i] += pp[i];
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) s[i] = wave_sum_d(s[i]);
  if (lane != 0) return;
  if constexpr (NV == 9) {
    // least-squares shift along each axis, clipped
    const double m = a.max_shift;
    const double sy = s[7] > 0.0 ? s[5] / s[7] : 0.0, sx = s[8] > 0.0 ? s[6] / s[8] : 0.0;
    a.shift[b] = make_float2((float)fmin(fmax(sy, -m), m), (float)fmin(fmax(sx, -m), m));
  }
  const double m00 = s[0], m11 = s[1], m01 = s[2], v0 = s[3], v1 = s[4];
  const double mx = fmax(m00, m11);
  double ao = 0.0, ap = 0.0;
  if (mx > 0.0) {
    const double eta = 1e-6 * mx;
    if (!a.probe_on) {
      ao = v0 / (m00 + eta);
    } else {
      const double a00 = m00 + eta, a11 = m11 + eta;
      const double det = a00 * a11 - m01 * m01;
      ao = (a11 * v0 - m01 * v1) / det;
      ap = (a00 * v1 - m01 * v0) / det;
    }
  }
  const float2 al = make_float2((float)ao, (float)ap);
  a.alpha[b] = al;
  a.alpha_by_j[a.jlist[b]] = al;
}

__global__ __launch_bounds__(64 * kLsqSolveWaves) void k_lsq_solve(LsqStepArgs a, int nrb) {
  const int b = blockIdx.x * kLsqSolveWaves + (threadIdx.x >> 6);
  if (b >= a.count) return;   // whole wavefronts
  if (a.shift)
    lsq_solve_one<9>(a, b, nrb);
  else
    lsq_solve_one<5>(a, b, nrb);
}

// ---------------------------------------------------------------------------
// ePIE update of one position (positions are sequential): the two step
// normalisers max_r sum_k |P_k|^2 and max_r |S_j O|^2 (storing the
// pre-update patch S_j O), then the probe update with that patch and the
// object update with the pre-update probe — two grid-wide launches
// ---------------------------------------------------------------------------
// Few blocks, each striding over the window, so that only a few hundred
// atomics meet on the two slots (one per block and slot).
constexpr int kEpieMaxBlocks = 64;

template <int N, int K>
__global__ __launch_bounds__(256) void k_epie_max(EpieArgs a) {
  __shared__ float redf[4];
  constexpr int NN = N * N;
  float s = 0.f, o = 0.f;
  for (int q = blockIdx.x * 256 + threadIdx.x; q < NN; q += kEpieMaxBlocks * 256) {
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) t += cabs2(a.probe[(size_t)k * NN + q]);
    s = fmaxf(s, t);
    const float2 ov = obj_bilinear(a.obj, a.h, a.w, a.pos, q / N, q % N);
    a.patch[q] = ov;      // the pre-update patch, for the probe update
    o = fmaxf(o, cabs2(ov));
  }
  const float ps = block_max_all<256>(s, redf);
  const float os = block_max_all<256>(o, redf);
  // non-negative floats order like their bit patterns
  if (threadIdx.x == 0) {
    atomicMax(a.maxes, __float_as_uint(ps));
    atomicMax(a.maxes + 1, __float_as_uint(os));
  }
}

// Probe and object updates in one launch: the first blocks update the probe
// pixels from the stored pre-update patch (into probe_out), the rest the
// object footprint with the pre-update probe, so the two never touch the
// same memory.
template <int N, int K>
__global__ __launch_bounds__(256) void k_epie_apply(EpieArgs a, int probe_blocks) {
  constexpr int NN = N * N;
  if ((int)blockIdx.x < probe_blocks) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= NN) return;
    const float omax = __uint_as_float(a.maxes[1]);
    const bool pu = a.probe_on && omax > 0.f;
    const float bs = pu ? a.beta / omax : 0.f;
    const float2 o = a.patch[q];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const size_t i = (size_t)k * NN + q;
      a.probe_out[i] = a.probe[i] + bs * cconjmul(o, a.chi[i]);
    }
    return;
  }
  const float pmax = __uint_as_float(a.maxes[0]);
  if (!(pmax > 0.f)) return;
  const int e = (blockIdx.x - probe_blocks) * 256 + threadIdx.x;
  if (e >= (N + 1) * (N + 1)) return;
  const PosInfo p = a.pos;
  const int u = e / (N + 1), v = e % (N + 1);
  const int Y = p.iy + u, X = p.ix + v;
  if (Y >= a.h || X >= a.w) return;
  // S_j^T over the (N+1)^2 footprint: the up to four patch pixels whose taps reach (Y, X)
  const float as = a.alpha / pmax;
  const float wx0 = 1.f - p.fx, wx1 = p.fx, wy0 = 1.f - p.fy, wy1 = p.fy;
  float2 sum = make_float2(0.f, 0.f);
#pragma unroll
  for (int tap = 0; tap < 4; ++tap) {
    const int uu = u - (tap >> 1), vv = v - (tap & 1);
    if ((unsigned)uu >= (unsigned)N || (unsigned)vv >= (unsigned)N) continue;
    const float wt = ((tap >> 1) ? wy1 : wy0) * ((tap & 1) ? wx1 : wx0);
    float2 tv = make_float2(0.f, 0.f);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const size_t i = (size_t)k * NN + uu * N + vv;
      tv = tv + cconjmul(a.probe[i], a.chi[i]);
    }
    sum = sum + wt * tv;
  }
  const size_t o = (size_t)Y * a.w + X;
  a.obj[o] = a.obj[o] + as * sum;
}

// ---------------------------------------------------------------------------
// DM exit-wave initialisation: psi_jk = P_k S_j O, contribution sum_k |P_k|^2 S_j O
// ---------------------------------------------------------------------------
template <int N, int K>
__global__ __launch_bounds__(256) void k_dm_init(DmInitArgs a) {
  const int j = blockIdx.y;
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= N * N) return;
  const PosInfo p = a.pos[j];
  const float2 o = obj_bilinear(a.obj, a.h, a.w, p, q / N, q % N);
  float2 c = make_float2(0.f, 0.f);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float2 pk = a.probe[(size_t)k * N * N + q];
    const float2 ps = cmul(pk, o);
    a.psi[((size_t)j * K + k) * N * N + q] = ps;
    c = c + cconjmul(pk, ps);
  }
  a.contrib[(size_t)j * N * N + q] = c;
}

// ---------------------------------------------------------------------------
// Utilities
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(unsigned* p, size_t n, unsigned v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ __launch_bounds__(256) void k_amplitude(const float* __restrict__ cnt, float* __restrict__ amp, int n, size_t total) {
  const size_t i = blockIdx.x * (size_t)256 + threadIdx.x;
  if (i >= total) return;
  const size_t nn = (size_t)n * n;
  const size_t j = i / nn;
  const int pr = (int)((i % nn) / n), pc = (int)(i % n);
  const int h = n / 2;
  const float d = cnt[j * nn + (size_t)((pr + h) & (n - 1)) * n + ((pc + h) & (n - 1))];
  amp[i] = d > 0.f ? sqrtf(d) : 0.f;   // +0 for d <= 0 and NaN: a clear sign bit means measured
}

// Detector mask: the sign bit of a stored modulus marks a pixel without a
// measurement (-0 included), so masking is reversible and costs the Fourier
// passes no extra load.  mask == nullptr: every pixel measured.
__global__ __launch_bounds__(256) void k_apply_mask(float* __restrict__ amp, const unsigned char* __restrict__ mask,
                                                    size_t nn, size_t total) {
  const size_t i = blockIdx.x * (size_t)256 + threadIdx.x;
  if (i >= total) return;
  const float v = fabsf(amp[i]);
  amp[i] = (mask == nullptr || mask[i % nn]) ? v : -v;
}

__global__ __launch_bounds__(256) void k_pattern_totals(const float* __restrict__ x, double* totals, int n) {
  __shared__ double red[4];
  const size_t nn = (size_t)n * n;
  const float* xp = x + blockIdx.x * nn;
  double s = 0.0;
  for (size_t i = threadIdx.x; i < nn; i += 256) s += fmaxf(xp[i], 0.f);
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) totals[blockIdx.x] = s;
}

// Per-pattern sum of the squared stored moduli (the counts, negative ones as
// 0, whatever the mask).
__global__ __launch_bounds__(256) void k_amp_totals(const float* __restrict__ amp, double* totals, int n) {
  __shared__ double red[4];
  const size_t nn = (size_t)n * n;
  const float* ap = amp + blockIdx.x * nn;
  double s = 0.0;
  for (size_t i = threadIdx.x; i < nn; i += 256) s += (double)ap[i] * ap[i];
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) totals[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_intensity(const float2* probe, float* pint, int n, int k,
                                                         unsigned* zero) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  const int nn = n * n;
  if (q == 0 && zero) *zero = 0u;
  if (q >= nn) return;
  float s = 0.f;
  for (int i = 0; i < k; ++i) s += cabs2(probe[(size_t)i * nn + q]);
  pint[q] = s;
}

// Deterministic sum of `count` (num, den) partial pairs; out = num / den.
// out[*slot] = E (slot NULL: out[0]); with advance != 0 thread 0 then increments *slot
__global__ __launch_bounds__(1024) void k_err_reduce(const double* errp, int count, double* out, int* slot,
                                                     int advance) {
  __shared__ double red[16];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < count; i += 1024) {
    a += errp[2 * (size_t)i];
    b += errp[2 * (size_t)i + 1];
  }
  a = block_sum<1024>(a, red);
  b = block_sum<1024>(b, red);
  if (threadIdx.x == 0) {
    const int t = slot ? *slot : 0;
    out[t] = b != 0.0 ? a / b : a;
    if (advance) *slot = t + 1;
  }
}

__global__ void k_posgrad_reduce(const double* part, int count, int nrb, float* out, const int* jlist) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= count) return;
  double gy = 0.0, gx = 0.0;
  for (int r = 0; r < nrb; ++r) {
    gy += part[((size_t)s * nrb + r) * 2];
    gx += part[((size_t)s * nrb + r) * 2 + 1];
  }
  const int j = jlist[s];
  out[2 * j] = (float)gy;
  out[2 * j + 1] = (float)gx;
}

__global__ void k_scale_f32(float* p, size_t n, float s) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] *= s;
}
__global__ void k_scale_c64(float2* p, size_t n, float s) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = s * p[i];
}

inline unsigned grid_for(size_t n, unsigned bs, unsigned cap = 65535u * 4) {
  size_t g = (n + bs - 1) / bs;
  if (g < 1) g = 1;
  return (unsigned)(g > cap ? cap : g);
}


// ---------------------------------------------------------------------------
// Fused ePIE iteration for small windows (one workgroup, positions in order)
// ---------------------------------------------------------------------------
// One thread group of T lanes per line and one line per group: N groups, so
// a row pass covers every row of a mode at once and a column pass every
// column.  Per position the workgroup makes four passes with one barrier
// after each:
//   A  rows, forward: the pre-update patch S_j O (bilinear, kept in
//      registers until C), the exit waves P_k S_j O and their x-transforms;
//      the two step normalisers' partial maxima;
//   B  columns: y-transform of every mode, the multi-mode modulus
//      projection with the amplitude-error partials, inverse y-transform;
//   C  rows, inverse: chi_k, the object-update contribution
//      sum_k conj(P_k) chi_k (into plane 0) and the probe update from the
//      pre-update patch, each pixel by the thread that owns it;
//   D  the object update over the patch's (N+1)^2 footprint.
// LDS planes (field, probe) are N x N with the columns of each row
// XOR-swizzled (epie_swz): a wavefront reading 8 (N = 32: 16) rows' segments
// or 8 (16) columns' segments then touches distinct bank pairs (gfx950 LDS:
// 64 banks of 4 bytes).  The line exchange of a transform goes through a
// padded per-line area when it fits in LDS with the field and the probe,
// else in place through the line's own row or column of the field.
template <int N, int K>
struct EpieGeo {
  static constexpr int R = FftShape<N>::R, T = FftShape<N>::T;
  static constexpr int NT = N * T;                     // threads: one line per T-lane group
  static constexpr int W = LineLds<N>::words;          // padded exchange area per line
  static constexpr size_t budget = 150 * 1024;
  static constexpr size_t plane_bytes = sizeof(float2) * (size_t)N * N;
  static constexpr size_t z_bytes = plane_bytes * K;
  static constexpr size_t tw_bytes = sizeof(float2) * N;
  static constexpr size_t xb_bytes = sizeof(float2) * (size_t)N * W;
  static constexpr bool PL = z_bytes + tw_bytes + plane_bytes * K <= budget;          // probe in LDS
  static constexpr bool XB = z_bytes + tw_bytes + (PL ? plane_bytes * K : 0) + xb_bytes <= budget;
  static constexpr size_t lds = z_bytes + tw_bytes + (PL ? plane_bytes * K : 0) + (XB ? xb_bytes : 0);
  static constexpr bool TWREG = R <= 8;                // twiddles in registers (else from LDS)
  static constexpr bool PREFETCH = R <= 8;             // next position's moduli fetched a pass early
};

// Column swizzle of row y, 8 (y & 3) + 4 ((y >> 2) & 1): distinct for the 8
// rows of an aligned group of 8, and distinct in its bits 3-4 for the 4 rows
// of an aligned group of 4 (linear under XOR in y mod 8).
__device__ __forceinline__ int epie_swz(int y) { return ((y & 3) << 3) | ((y & 4) ? 4 : 0); }

// Exchange areas of one line transform: wr(q) is where register q of this
// lane goes, rd(i, s) where the i-th T-point input s of this lane comes from.
template <int N>
struct XbArea {   // padded per-line area (row stride T + 1)
  float2* b;
  int t;
  __device__ float2& wr(int q) const { return b[q * (FftShape<N>::T + 1) + t]; }
  __device__ float2& rd(int i, int s) const {
    return b[(t + i * FftShape<N>::T) * (FftShape<N>::T + 1) + s];
  }
};
template <int N>
struct RowArea {  // the line's own (swizzled) row: element e at e ^ sw
  float2* row;
  int sw, t;
  __device__ float2& wr(int q) const {
    constexpr int T = FftShape<N>::T;
    return row[(q * T + (t ^ (q & (T - 1)))) ^ sw];
  }
  __device__ float2& rd(int i, int s) const {
    constexpr int T = FftShape<N>::T;
    return row[((t + i * T) * T + (s ^ t)) ^ sw];
  }
};
template <int N>
struct ColArea {  // the line's own column x of a (swizzled) plane
  float2* plane;
  int x, t;
  __device__ float2& at(int e) const { return plane[e * N + (x ^ epie_swz(e))]; }
  __device__ float2& wr(int q) const {
    constexpr int T = FftShape<N>::T;
    return at(q * T + (t ^ (q & (T - 1))));
  }
  __device__ float2& rd(int i, int s) const {
    constexpr int T = FftShape<N>::T;
    return at((t + i * T) * T + (s ^ t));
  }
};

// Length-N line transform (the four-step scheme of line_fft) with the
// exchange through `ar`.  In the in-place areas element (q, lane) is kept at
// q T + (lane ^ (q mod T)), so the write and the transposed read touch
// distinct banks.  `twr`: W_N^(t q), q = 1 .. R-1 (forward), when TWREG.
template <int N, bool INV, bool TWREG, class Area>
__device__ __forceinline__ void epie_line(float2* v, const Area& ar, const float2* twr, const float2* tw_s, int t) {
  constexpr int R = FftShape<N>::R, T = FftShape<N>::T;
  Dft<R, INV>::run(v);
#pragma unroll
  for (int q = 1; q < R; ++q) {
    float2 w = TWREG ? twr[q - 1] : tw_s[(t * q) & (N - 1)];
    if (INV) w.y = -w.y;
    v[q] = cmul(v[q], w);
  }
#pragma unroll
  for (int q = 0; q < R; ++q) ar.wr(q) = v[q];
  wave_sync();
#pragma unroll
  for (int i = 0; i < R / T; ++i) {
    float2 u[T];
#pragma unroll
    for (int s = 0; s < T; ++s) u[s] = ar.rd(i, s);
    Dft<T, INV>::run(u);
#pragma unroll
    for (int s = 0; s < T; ++s) v[i + (R / T) * s] = u[s];
  }
  wave_sync();
}

// The iteration's amplitude-error sums of a one-workgroup ePIE kernel: each
// lane's sums over the positions, added over the wavefront (DPP, fixed
// order) and the wavefronts in order, go to the first pair of the error
// partials; every other pair of the iteration's patterns is zeroed (the
// reduction sums them all).
__device__ __forceinline__ void epie_error_out(const EpieRunArgs& a, double num, double den, double (*red)[2], int nt) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const double s0 = wave_sum_d(num), s1 = wave_sum_d(den);
  if (lane == 0) {
    red[wid][0] = s0;
    red[wid][1] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double e0 = 0.0, e1 = 0.0;
    for (int w = 0; w < nt / 64; ++w) {
      e0 += red[w][0];
      e1 += red[w][1];
    }
    a.errp[0] = e0;
    a.errp[1] = e1;
  }
  const size_t pairs = (size_t)a.count * a.bpp;
  for (size_t i = 1 + threadIdx.x; i < pairs; i += nt) a.errp[2 * i] = a.errp[2 * i + 1] = 0.0;
}

// Workgroup barrier that orders LDS only: global loads still in flight (the
// next pattern's moduli) stay in flight across it.  Global memory written in
// one pass and read by other threads in the next needs __syncthreads().
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Hides a value's origin from loop-invariant code motion: the per-thread
// LDS addresses of a pass are then formed in that pass instead of being held
// (or spilled) across the whole position loop.
__device__ __forceinline__ void opaque(int& v) { asm volatile("" : "+v"(v)); }

// Patch row u of S_j O at columns t + T m (the bilinear gather of
// obj_bilinear, with the two object rows addressed once per thread so that
// the R loads of a row differ only by constant offsets).
template <int N>
__device__ __forceinline__ void epie_patch_row(const float2* __restrict__ obj, int h, int w, const PosInfo& p,
                                               int u, int t, float2* o) {
  constexpr int R = FftShape<N>::R, T = FftShape<N>::T;
  const int r0 = p.iy + u, r1 = min(r0 + 1, h - 1);
  const float wx1 = p.fx, wx0 = 1.f - p.fx, wy1 = p.fy, wy0 = 1.f - p.fy;
  auto mix = [&](float2 va, float2 vb, float2 vc, float2 vd) {
    return make_float2(wy0 * (wx0 * va.x + wx1 * vb.x) + wy1 * (wx0 * vc.x + wx1 * vd.x),
                       wy0 * (wx0 * va.y + wx1 * vb.y) + wy1 * (wx0 * vc.y + wx1 * vd.y));
  };
  if (p.ix + N < w) {
    // no column reaches the object's last one: all taps at constant offsets
    const float2* b0 = obj + (size_t)r0 * w + p.ix + t;
    const float2* b1 = obj + (size_t)r1 * w + p.ix + t;
#pragma unroll
    for (int m = 0; m < R; ++m) o[m] = mix(b0[T * m], b0[T * m + 1], b1[T * m], b1[T * m + 1]);
  } else {
    const float2* a0 = obj + (size_t)r0 * w;
    const float2* a1 = obj + (size_t)r1 * w;
#pragma unroll
    for (int m = 0; m < R; ++m) {
      const int c0 = p.ix + t + T * m, c1 = min(c0 + 1, w - 1);
      o[m] = mix(a0[c0], a0[c1], a1[c0], a1[c1]);
    }
  }
}

template <int N, int K>
__global__ __launch_bounds__(N * FftShape<N>::T) void k_epie_fused(EpieRunArgs a) {
  using G = EpieGeo<N, K>;
  constexpr int R = G::R, T = G::T, NT = G::NT, NN = N * N, NW = NT / 64;
  constexpr bool PL = G::PL, XB = G::XB;
  extern __shared__ float2 lds[];
  float2* Z = lds;                                   // K swizzled planes: exit waves / far field / chi
  float2* tw_s = Z + (size_t)K * NN;                 // W_N table
  float2* pl = tw_s + N;                             // K swizzled probe planes (when PL)
  float2* xb = pl + (PL ? (size_t)K * NN : 0);       // per-line exchange areas (when XB)
  __shared__ float redf[NW][2];
  __shared__ double redd[NW][2];
  int li = threadIdx.x / T, t = threadIdx.x % T;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < N; i += NT) tw_s[i] = reinterpret_cast<const float2*>(a.tw)[i];
  float2 twr[G::TWREG ? R - 1 : 1];
  if constexpr (G::TWREG) {
    const float2* tw = reinterpret_cast<const float2*>(a.tw);
#pragma unroll
    for (int q = 1; q < R; ++q) twr[q - 1] = tw[(t * q) & (N - 1)];
  }
  if constexpr (PL) {
    for (int i = threadIdx.x; i < K * NN; i += NT) {
      const int y = (i / N) % N, x = i % N;
      pl[(i / N) * N + (x ^ epie_swz(y))] = a.probe0[i];
    }
  }
  // probe row y of mode k: LDS (swizzled) or global (plain)
  auto probe_row = [&](int k, int y) -> float2* { return PL ? pl + ((size_t)k * N + y) * N : a.probe0 + ((size_t)k * N + y) * N; };
  const int psw = PL ? 1 : 0;   // probe rows are swizzled in LDS only
  // moduli of the pixels this thread owns in the column pass: (t + T m, li)
  float amp_n[R];
#define PTY_EPIE_LOAD_AMP(nidx)                                                \
  do {                                                                        \
    const float* ap_ = a.amp + (size_t)a.order[(nidx)] * NN;                  \
    _Pragma("unroll") for (int m_ = 0; m_ < R; ++m_) amp_n[m_] = ap_[(unsigned)((t + T * m_) * N + li)]; \
  } while (0)
  if (G::PREFETCH && a.count > 0) PTY_EPIE_LOAD_AMP(0);
  __syncthreads();
  // the transforms are unscaled: the unitary far field is Z / N, and the
  // unitary inverse contributes another 1 / N^2, folded into the projection
  constexpr float sc = 1.0f / N, sc2 = 1.0f / (float(N) * float(N));
  double err_num = 0.0, err_den = 0.0;   // this lane's amplitude-error sums over the positions
  for (int n = 0; n < a.count; ++n) {
    const int j = a.order[n];
    const PosInfo p = a.pos[j];
    float amp_c[R];
    if constexpr (G::PREFETCH) {
#pragma unroll
      for (int m = 0; m < R; ++m) amp_c[m] = amp_n[m];
    } else {
      PTY_EPIE_LOAD_AMP(n);   // consumed in pass B, after pass A's work
#pragma unroll
      for (int m = 0; m < R; ++m) amp_c[m] = amp_n[m];
    }
    // ---- A: row li of the patch and of every exit wave, forward x-transform
    opaque(li);
    opaque(t);
    float2 o[R];
    float om = 0.f, pm = 0.f, sp[K == 1 ? 1 : R];
    epie_patch_row<N>(a.obj, a.h, a.w, p, li, t, o);
#pragma unroll
    for (int m = 0; m < R; ++m) {
      om = fmaxf(om, cabs2(o[m]));
      if constexpr (K > 1) sp[m] = 0.f;
    }
    const int rsw = epie_swz(li);
#pragma unroll 1
    for (int k = 0; k < K; ++k) {
      const float2* pr = probe_row(k, li);
      float2 z[R];
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const float2 pk = pr[(t + T * m) ^ (psw * rsw)];
        if constexpr (K == 1) pm = fmaxf(pm, cabs2(pk));
        else sp[m] += cabs2(pk);
        z[m] = cmul(pk, o[m]);
      }
      float2* row = Z + ((size_t)k * N + li) * N;
      if constexpr (XB) epie_line<N, false, G::TWREG>(z, XbArea<N>{xb + li * G::W, t}, twr, tw_s, t);
      else epie_line<N, false, G::TWREG>(z, RowArea<N>{row, rsw, t}, twr, tw_s, t);
#pragma unroll
      for (int m = 0; m < R; ++m) row[(t + T * m) ^ rsw] = z[m];
    }
    if constexpr (K > 1) {
#pragma unroll
      for (int m = 0; m < R; ++m) pm = fmaxf(pm, sp[m]);
    }
    pm = wave_max_nonneg(pm);
    om = wave_max_nonneg(om);
    if (lane == 0) {
      redf[wid][0] = pm;
      redf[wid][1] = om;
    }
    lds_barrier();
    // ---- B: column li of every mode: y-transform, projection, inverse y-transform
    opaque(li);
    opaque(t);
    {
      float2 z[K][R];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const ColArea<N> col{Z + (size_t)k * NN, li, t};
#pragma unroll
        for (int m = 0; m < R; ++m) z[k][m] = col.at(t + T * m);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if constexpr (XB) epie_line<N, false, G::TWREG>(z[k], XbArea<N>{xb + li * G::W, t}, twr, tw_s, t);
        else epie_line<N, false, G::TWREG>(z[k], ColArea<N>{Z + (size_t)k * NN, li, t}, twr, tw_s, t);
      }
      if (G::PREFETCH && n + 1 < a.count) PTY_EPIE_LOAD_AMP(n + 1);
      float en = 0.f, ed = 0.f;
#pragma unroll
      for (int m = 0; m < R; ++m) {
        float iraw = 0.f;
#pragma unroll
        for (int k = 0; k < K; ++k) iraw += cabs2(z[k][m]);
        // hardware square root and reciprocal (within 1 ulp each)
        const float mod = __builtin_amdgcn_sqrtf(iraw) * sc;
        const bool meas = !signbit(amp_c[m]);      // sign bit: no measurement
        const float am = fabsf(amp_c[m]);
        const float f = meas ? (am * __builtin_amdgcn_rcpf(fmaxf(mod, 1e-6f)) - 1.f) * sc2 : 0.f;
        if (meas) {
          en += (mod - am) * (mod - am);
          ed += am * am;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) z[k][m] = f * z[k][m];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const ColArea<N> col{Z + (size_t)k * NN, li, t};
        if constexpr (XB) epie_line<N, true, G::TWREG>(z[k], XbArea<N>{xb + li * G::W, t}, twr, tw_s, t);
        else epie_line<N, true, G::TWREG>(z[k], col, twr, tw_s, t);
#pragma unroll
        for (int m = 0; m < R; ++m) col.at(t + T * m) = z[k][m];
      }
      // the error needs only the sums over all positions: kept per lane
      err_num += en;
      err_den += ed;
    }
    lds_barrier();
    // block maxima of pass A (written before the previous barrier)
    float pmax = 0.f, omax = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      pmax = fmaxf(pmax, redf[w][0]);
      omax = fmaxf(omax, redf[w][1]);
    }
    // ---- C: row li, inverse x-transform of every mode; contribution and probe update
    opaque(li);
    opaque(t);
    {
      const float bs = (a.probe_on && omax > 0.f) ? a.beta / omax : 0.f;
      const int csw = epie_swz(li);
      float2 cn[R];
#pragma unroll
      for (int m = 0; m < R; ++m) cn[m] = make_float2(0.f, 0.f);
#pragma unroll 1
      for (int k = 0; k < K; ++k) {
        float2* row = Z + ((size_t)k * N + li) * N;
        float2 z[R];
#pragma unroll
        for (int m = 0; m < R; ++m) z[m] = row[(t + T * m) ^ csw];
        if constexpr (XB) epie_line<N, true, G::TWREG>(z, XbArea<N>{xb + li * G::W, t}, twr, tw_s, t);
        else epie_line<N, true, G::TWREG>(z, RowArea<N>{row, csw, t}, twr, tw_s, t);
        float2* pr = probe_row(k, li);
#pragma unroll
        for (int m = 0; m < R; ++m) {
          const int x = (t + T * m) ^ (psw * csw);
          const float2 pk = pr[x];
          cn[m] = cn[m] + cconjmul(pk, z[m]);
          if (bs != 0.f) pr[x] = pk + bs * cconjmul(o[m], z[m]);
        }
      }
      // plane 0, row li: read by this line group only, so it can hold the contribution
      float2* row0 = Z + (size_t)li * N;
#pragma unroll
      for (int m = 0; m < R; ++m) row0[(t + T * m) ^ csw] = cn[m];
    }
    lds_barrier();
    // ---- D: object update over the (N+1)^2 footprint with the pre-update probe
    opaque(li);
    opaque(t);
    if (pmax > 0.f) {
      // Thread (column v, row block rb) walks rows rb R .. rb R + R - 1 of
      // footprint column v; the last row block also takes row N and the
      // threads of column N - 1 also column N.  The horizontal tap pair of row
      // u - 1 is kept from the previous row, so each row reads two values of
      // the contribution plane.
      const float as = a.alpha / pmax;
      const float wx0 = 1.f - p.fx, wx1 = p.fx, wy0 = 1.f - p.fy, wy1 = p.fy;
      int tid = threadIdx.x;
      opaque(tid);
      const int v = tid % N, rb = tid / N, u0 = rb * R;
      const bool row_n = rb == T - 1 && p.iy + N < a.h;     // footprint row N lies in the object
      const bool col_n = v == N - 1 && p.ix + N < a.w;      // footprint column N lies in the object
      float2* op = a.obj + (size_t)(p.iy + u0) * a.w + p.ix + v;
      float2 ov[R + 1], ox[R + 1];
      // every old value of this thread is loaded before any is written
#pragma unroll
      for (int i = 0; i <= R; ++i) {
        const bool ok = i < R || row_n;
        ov[i] = ok ? op[(size_t)i * a.w] : make_float2(0.f, 0.f);
        ox[i] = (ok && col_n) ? op[(size_t)i * a.w + 1] : make_float2(0.f, 0.f);
      }
      const float2 zero = make_float2(0.f, 0.f);
      // contribution c(u, v) and c(u, v - 1) (zero left of the patch)
      auto ctap = [&](int u, float2& c0, float2& c1) {
        const int sw = epie_swz(u);
        c0 = Z[u * N + (v ^ sw)];
        c1 = v > 0 ? Z[u * N + ((v - 1) ^ sw)] : make_float2(0.f, 0.f);
      };
      float2 hp = zero, hxp = zero;
      if (u0 > 0) {
        float2 c0, c1;
        ctap(u0 - 1, c0, c1);
        hp = wx0 * c0 + wx1 * c1;
        hxp = wx1 * c0;
      }
#pragma unroll
      for (int i = 0; i < R; ++i) {
        float2 c0, c1;
        ctap(u0 + i, c0, c1);
        const float2 hc = wx0 * c0 + wx1 * c1, hxc = wx1 * c0;
        op[(size_t)i * a.w] = ov[i] + as * (wy0 * hc + wy1 * hp);
        if (col_n) op[(size_t)i * a.w + 1] = ox[i] + as * (wy0 * hxc + wy1 * hxp);
        hp = hc;
        hxp = hxc;
      }
      if (row_n) {   // footprint row N: only the taps of patch row N - 1
        op[(size_t)R * a.w] = ov[R] + as * (wy1 * hp);
        if (col_n) op[(size_t)R * a.w + 1] = ox[R] + as * (wy1 * hxp);
      }
    }
    // the next position reads the updated object and probe
    __syncthreads();
  }
  epie_error_out(a, err_num, err_den, redd, NT);
  // leave the probe where an alternating scheme would: probe1 after an odd count
  if (a.count % 2 == 1 || PL) {
    float2* dst = (a.count % 2 == 1) ? a.probe1 : a.probe0;
    for (int i = threadIdx.x; i < K * NN; i += NT) {
      const int y = (i / N) % N, x = i % N;
      dst[i] = PL ? pl[(i / N) * N + (x ^ epie_swz(y))] : a.probe0[i];
    }
  }
}
#undef PTY_EPIE_LOAD_AMP

// The scan order and positions, which the fused kernels only read, through
// the constant address space: their uniform loads become scalar loads.
struct ScanTables {
  const int* order;
  const PosInfo* pos;
  __device__ int operator[](int i) const {
#if defined(__HIP_DEVICE_COMPILE__)
    return ((const __attribute__((address_space(4))) int*)order)[i];
#else
    return order[i];
#endif
  }
  __device__ PosInfo at(int j) const {
#if defined(__HIP_DEVICE_COMPILE__)
    const __attribute__((address_space(4))) PosInfo& q = ((const __attribute__((address_space(4))) PosInfo*)pos)[j];
    return PosInfo{q.iy, q.ix, q.fy, q.fx};
#else
    return pos[j];
#endif
  }
};

__device__ __forceinline__ int dx_of(const PosInfo& p, const PosInfo& pn) { return p.ix - pn.ix; }

// Fused ePIE with the object footprint and the probe on chip (windows up to
// 64 x 64): the pre-update (N+1)^2 footprint of the current position sits in
// LDS (FS-strided rows), so the patch gather and the object update read no
// global memory; the footprint of the next position is assembled during the
// current one: its pixels outside the current footprint are fetched from
// global memory in pass B (they are final already), the others are taken
// from the update of pass D as it is written.  Each thread keeps the probe
// pixels it transforms (mode k, row li, columns t + T m) in registers for the
// whole iteration.  Passes and the field layout as in k_epie_fused.
template <int N, int K>
struct EpieFbGeo {
  static constexpr int R = FftShape<N>::R, T = FftShape<N>::T;
  static constexpr int NT = N * T, W = LineLds<N>::words, F = N + 1;
  static constexpr int FS = N + T;                     // footprint row stride: 8 (4) rows x 8 (4) columns conflict-free
  static constexpr size_t budget = 150 * 1024;
  static constexpr size_t z_bytes = sizeof(float2) * (size_t)K * N * N;
  static constexpr size_t tw_bytes = sizeof(float2) * N;
  static constexpr size_t fb_bytes = sizeof(float2) * 2 * (size_t)F * FS;
  static constexpr size_t xb_bytes = sizeof(float2) * (size_t)N * W;
  static constexpr bool XB = z_bytes + tw_bytes + fb_bytes + xb_bytes <= budget;
  static constexpr size_t lds = z_bytes + tw_bytes + fb_bytes + (XB ? xb_bytes : 0);
  static constexpr bool TWREG = R <= 8;
};

template <int N, int K>
__global__ __launch_bounds__(N * FftShape<N>::T) void k_epie_fused_fb(EpieRunArgs a) {
  using G = EpieFbGeo<N, K>;
  constexpr int R = G::R, T = G::T, NT = G::NT, NN = N * N, NW = NT / 64, F = G::F, FS = G::FS;
  constexpr bool XB = G::XB;
  extern __shared__ float2 lds[];
  float2* Z = lds;                                   // K swizzled planes: exit waves / far field / chi
  float2* tw_s = Z + (size_t)K * NN;                 // W_N table
  float2* fb = tw_s + N;                             // two footprints, F x FS each
  float2* xb = fb + 2 * F * FS;                      // per-line exchange areas (when XB)
  __shared__ float redf[NW][2];
  __shared__ double redd[NW][2];
  const ScanTables order{a.order, a.pos};
  int li = threadIdx.x / T, t = threadIdx.x % T;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < N; i += NT) tw_s[i] = reinterpret_cast<const float2*>(a.tw)[i];
  float2 twr[G::TWREG ? R - 1 : 1];
  if constexpr (G::TWREG) {
    const float2* tw = reinterpret_cast<const float2*>(a.tw);
#pragma unroll
    for (int q = 1; q < R; ++q) twr[q - 1] = tw[(t * q) & (N - 1)];
  }
  float2 pk[K][R];   // this thread's probe pixels (k, li, t + T m)
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int m = 0; m < R; ++m) pk[k][m] = a.probe0[((size_t)k * N + li) * N + t + T * m];
  }
  float amp_n[R];
#define PTY_EPIE_LOAD_AMP(nidx) PTY_EPIE_LOAD_AMP_J(order[(nidx)])
#define PTY_EPIE_LOAD_AMP_J(jidx)                                              \
  do {                                                                        \
    const float* ap_ = a.amp + (size_t)(jidx) * NN;                           \
    _Pragma("unroll") for (int m_ = 0; m_ < R; ++m_) amp_n[m_] = ap_[(unsigned)((t + T * m_) * N + li)]; \
  } while (0)
  // scan entries, fetched ahead: this position (jc, pc), the next (jn, pnx)
  // and the index of the one after (jnn, read in pass A, its position in C)
  int jc = 0, jn = 0;
  PosInfo pc{}, pnx{};
  if (a.count > 0) {
    jc = order[0];
    jn = a.count > 1 ? order[1] : jc;
    pc = order.at(jc);
    pnx = order.at(jn);
    PTY_EPIE_LOAD_AMP(0);
    const PosInfo p0 = pc;
    for (int e = threadIdx.x; e < F * F; e += NT) {
      const int u = e / F, v = e % F, Y = p0.iy + u, X = p0.ix + v;
      fb[u * FS + v] = (Y < a.h && X < a.w) ? a.obj[(size_t)Y * a.w + X] : make_float2(0.f, 0.f);
    }
  }
  __syncthreads();
  constexpr float sc = 1.0f / N, sc2 = 1.0f / (float(N) * float(N));
  double err_num = 0.0, err_den = 0.0;   // this lane's amplitude-error sums over the positions
  for (int n = 0; n < a.count; ++n) {
    const int j = jc;
    const PosInfo p = pc;
    const bool more = n + 1 < a.count;
    const PosInfo pn = pnx;
    const int jnn = n + 2 < a.count ? order[n + 2] : jn;
    float2* cur = fb + (n & 1) * F * FS;
    float2* nxt = fb + ((n + 1) & 1) * F * FS;
    float amp_c[R];
#pragma unroll
    for (int m = 0; m < R; ++m) amp_c[m] = amp_n[m];
    // ---- A: row li of the patch and of every exit wave, forward x-transform
    opaque(li);
    opaque(t);
    float2 o[R];
    float om = 0.f, pm = 0.f;
    {
      const float wx1 = p.fx, wx0 = 1.f - p.fx, wy1 = p.fy, wy0 = 1.f - p.fy;
      const float2* f0 = cur + li * FS + t;
      const float2* f1 = f0 + FS;
#pragma unroll
      for (int m = 0; m < R; ++m) {
        const float2 va = f0[T * m], vb = f0[T * m + 1], vc = f1[T * m], vd = f1[T * m + 1];
        o[m] = make_float2(wy0 * (wx0 * va.x + wx1 * vb.x) + wy1 * (wx0 * vc.x + wx1 * vd.x),
                           wy0 * (wx0 * va.y + wx1 * vb.y) + wy1 * (wx0 * vc.y + wx1 * vd.y));
        om = fmaxf(om, cabs2(o[m]));
        float sp = 0.f;
#pragma unroll
        for (int k = 0; k < K; ++k) sp += cabs2(pk[k][m]);
        pm = fmaxf(pm, sp);
      }
    }
    const int rsw = epie_swz(li);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      float2 z[R];
#pragma unroll
      for (int m = 0; m < R; ++m) z[m] = cmul(pk[k][m], o[m]);
      float2* row = Z + ((size_t)k * N + li) * N;
      if constexpr (XB) epie_line<N, false, G::TWREG>(z, XbArea<N>{xb + li * G::W, t}, twr, tw_s, t);
      else epie_line<N, false, G::TWREG>(z, RowArea<N>{row, rsw, t}, twr, tw_s, t);
#pragma unroll
      for (int m = 0; m < R; ++m) row[(t + T * m) ^ rsw] = z[m];
    }
    pm = wave_max_nonneg(pm);
    om = wave_max_nonneg(om);
    if (lane == 0) {
      redf[wid][0] = pm;
      redf[wid][1] = om;
    }
    // full barrier: the previous position's object stores are complete
    // before pass B fetches the next footprint from global memory
    __syncthreads();
    // ---- B: column li of every mode: y-transform, projection, inverse y-transform
    opaque(li);
    opaque(t);
    // next footprint, pixels (rb R + i, v) (+ row N, + column N), fetched now
    int tid = threadIdx.x;
    opaque(tid);
    const int v = tid % N, rb = tid / N, u0 = rb * R;
    float2 nv[R + 1], ncn;
    {
      // unconditional loads (a load under a branch would be waited for at
      // once): rows below N are inside the object, row N is clamped to it;
      // column N of the next footprint comes one pixel per thread (rows
      // tid <= N), clamped likewise; pixels past the object are dropped in D
      const float2* rp = a.obj + (size_t)(pn.iy + u0) * a.w + pn.ix + v;
#pragma unroll
      for (int i = 0; i < R; ++i) nv[i] = rp[(size_t)i * a.w];
      nv[R] = a.obj[(size_t)min(pn.iy + u0 + R, a.h - 1) * a.w + pn.ix + v];
      ncn = a.obj[(size_t)min(pn.iy + min(tid, N), a.h - 1) * a.w + min(pn.ix + N, a.w - 1)];
    }
    {
      float2 z[K][R];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const ColArea<N> col{Z + (size_t)k * NN, li, t};
#pragma unroll
        for (int m = 0; m < R; ++m) z[k][m] = col.at(t + T * m);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if constexpr (XB) epie_line<N, false, G::TWREG>(z[k], XbArea<N>{xb + li * G::W, t}, twr, tw_s, t);
        else epie_line<N, false, G::TWREG>(z[k], ColArea<N>{Z + (size_t)k * NN, li, t}, twr, tw_s, t);
      }
      if (more) PTY_EPIE_LOAD_AMP_J(jn);
      float en = 0.f, ed = 0.f;
#pragma unroll
      for (int m = 0; m < R; ++m) {
        float iraw = 0.f;
#pragma unroll
        for (int k = 0; k < K; ++k) iraw += cabs2(z[k][m]);
        // hardware square root and reciprocal (within 1 ulp each)
        const float mod = __builtin_amdgcn_sqrtf(iraw) * sc;
        const bool meas = !signbit(amp_c[m]);      // sign bit: no measurement
        const float am = fabsf(amp_c[m]);
        const float f = meas ? (am * __builtin_amdgcn_rcpf(fmaxf(mod, 1e-6f)) - 1.f) * sc2 : 0.f;
        if (meas) {
          en += (mod - am) * (mod - am);
          ed += am * am;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) z[k][m] = f * z[k][m];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const ColArea<N> col{Z + (size_t)k * NN, li, t};
        if constexpr (XB) epie_line<N, true, G::TWREG>(z[k], XbArea<N>{xb + li * G::W, t}, twr, tw_s, t);
        else epie_line<N, true, G::TWREG>(z[k], col, twr, tw_s, t);
#pragma unroll
        for (int m = 0; m < R; ++m) col.at(t + T * m) = z[k][m];
      }
      // the error needs only the sums over all positions: kept per lane
      err_num += en;
      err_den += ed;
    }
    lds_barrier();
    float pmax = 0.f, omax = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      pmax = fmaxf(pmax, redf[w][0]);
      omax = fmaxf(omax, redf[w][1]);
    }
    // ---- C: row li, inverse x-transform of every mode; contribution and probe update
    opaque(li);
    opaque(t);
    const PosInfo pnn = order.at(jnn);
    {
      const float bs = (a.probe_on && omax > 0.f) ? a.beta / omax : 0.f;
      const int csw = epie_swz(li);
      float2 cn[R];
#pragma unroll
      for (int m = 0; m < R; ++m) cn[m] = make_float2(0.f, 0.f);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        float2* row = Z + ((size_t)k * N + li) * N;
        float2 z[R];
#pragma unroll
        for (int m = 0; m < R; ++m) z[m] = row[(t + T * m) ^ csw];
        if constexpr (XB) epie_line<N, true, G::TWREG>(z, XbArea<N>{xb + li * G::W, t}, twr, tw_s, t);
        else epie_line<N, true, G::TWREG>(z, RowArea<N>{row, csw, t}, twr, tw_s, t);
#pragma unroll
        for (int m = 0; m < R; ++m) {
          cn[m] = cn[m] + cconjmul(pk[k][m], z[m]);
          pk[k][m] = pk[k][m] + bs * cconjmul(o[m], z[m]);
        }
      }
      float2* row0 = Z + (size_t)li * N;
#pragma unroll
      for (int m = 0; m < R; ++m) row0[(t + T * m) ^ csw] = cn[m];
    }
    lds_barrier();
    // ---- D: object update over the (N+1)^2 footprint; the next footprint
    {
      const float as = pmax > 0.f ? a.alpha / pmax : 0.f;
      const float wx0 = 1.f - p.fx, wx1 = p.fx, wy0 = 1.f - p.fy, wy1 = p.fy;
      const bool last_rb = rb == T - 1;
      const bool row_n = last_rb && p.iy + N < a.h;         // footprint row N lies in the object
      const bool col_n = p.ix + N < a.w;                    // footprint column N lies in the object
      // every LDS value this pass reads, before any LDS write: contribution
      // taps c(u, v), c(u, v - 1) of rows u0 - 1 .. u0 + R - 1 and the
      // footprint's old values of column v; column N (row tid <= N): the taps
      // c(u, N - 1) of rows tid - 1 and tid and its old value
      float2 c0v[R + 1], c1v[R + 1], ocv[R + 1];
#pragma unroll
      for (int i = 0; i <= R; ++i) {
        const int u = max(u0 + i - 1, 0);
        const int sw = epie_swz(u);
        c0v[i] = Z[u * N + (v ^ sw)];
        c1v[i] = Z[u * N + (max(v - 1, 0) ^ sw)];   // v = 0: weight zero below
      }
      const float2* oc = cur + u0 * FS + v;
#pragma unroll
      for (int i = 0; i <= R; ++i) ocv[i] = oc[i * FS];
      const int uc = min(tid, N);
      const float2 cnc = Z[min(uc, N - 1) * N + ((N - 1) ^ epie_swz(min(uc, N - 1)))];
      const float2 cnp = Z[max(uc - 1, 0) * N + ((N - 1) ^ epie_swz(max(uc - 1, 0)))];
      const float2 ocn = cur[uc * FS + N];
      if (more) {
        // pixels of the next footprint outside this one: from pass B's fetch
        const int du = pn.iy + u0 - p.iy;                    // row of this footprint, minus i
        const int xr = pn.ix + v - p.ix;                     // column of this footprint
        const bool xin = (unsigned)xr <= (unsigned)N;
#pragma unroll
        for (int i = 0; i <= R; ++i) {
          if (i == R && !last_rb) continue;
          const bool in_obj = i < R || pn.iy + N < a.h;
          const bool yin = (unsigned)(du + i) <= (unsigned)N && in_obj;
          if (!(yin && xin)) nxt[(u0 + i) * FS + v] = in_obj ? nv[i] : make_float2(0.f, 0.f);
        }
        if (tid <= N) {   // column N, row tid
          const bool in_obj = pn.iy + tid < a.h && pn.ix + N < a.w;
          const bool in_cur = (unsigned)(pn.iy + tid - p.iy) <= (unsigned)N &&
                              (unsigned)(pn.ix + N - p.ix) <= (unsigned)N && in_obj;
          if (!in_cur) nxt[tid * FS + N] = in_obj ? ncn : make_float2(0.f, 0.f);
        }
      }
      float2* op = a.obj + (size_t)(p.iy + u0) * a.w + p.ix + v;
      // this footprint's pixel (u, vv) is the next one's (u + dy, vv + dx)
      const int dy = p.iy - pn.iy, dx = p.ix - pn.ix, vn = v + dx;
      const bool vin = more && (unsigned)vn <= (unsigned)N;
      const float cm = v > 0 ? wx1 : 0.f;                    // weight of c(u, v - 1)
      float2 hp = u0 > 0 ? wx0 * c0v[0] + cm * c1v[0] : make_float2(0.f, 0.f);
#pragma unroll
      for (int i = 0; i <= R; ++i) {
        if (i == R && !row_n) continue;
        const float2 hc = i < R ? wx0 * c0v[i + 1] + cm * c1v[i + 1] : make_float2(0.f, 0.f);
        const float2 val = ocv[i] + as * (wy0 * hc + wy1 * hp);
        const int un = u0 + i + dy;
        if (as != 0.f) op[(size_t)i * a.w] = val;
        if (vin && (unsigned)un <= (unsigned)N) nxt[un * FS + vn] = val;
        hp = hc;
      }
      if (tid <= N && col_n && (tid < N || p.iy + N < a.h)) {
        // column N, row tid: only the taps of patch column N - 1
        const float2 hxc = tid < N ? wx1 * cnc : make_float2(0.f, 0.f);
        const float2 hxp = tid > 0 ? wx1 * cnp : make_float2(0.f, 0.f);
        const float2 vx = ocn + as * (wy0 * hxc + wy1 * hxp);
        if (as != 0.f) a.obj[(size_t)(p.iy + tid) * a.w + p.ix + N] = vx;
        const int un = tid + dy, vnn = N + dx;
        if (more && (unsigned)un <= (unsigned)N && (unsigned)vnn <= (unsigned)N) nxt[un * FS + vnn] = vx;
      }
    }
    lds_barrier();
    jc = jn;
    pc = pnx;
    jn = jnn;
    pnx = pnn;
  }
  epie_error_out(a, err_num, err_den, redd, NT);
  // probe out: probe1 after an odd count (the buffer an alternating scheme ends in)
  float2* dst = (a.count % 2 == 1) ? a.probe1 : a.probe0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int m = 0; m < R; ++m) dst[((size_t)k * N + li) * N + t + T * m] = pk[k][m];
  }
}
#undef PTY_EPIE_LOAD_AMP_J
#undef PTY_EPIE_LOAD_AMP

}  // namespace

// ---------------------------------------------------------------------------
// Strip decomposition: halo messages, probe-sum messages, applied updates
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_halo_pack(HaloPlanes p, int rows, float* __restrict__ msg) {
  const size_t n0 = (size_t)rows * p.words_per_row[0], n1 = (size_t)rows * p.words_per_row[1];
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n0 + n1; i += (size_t)gridDim.x * 256) {
    if (i < n0)
      msg[i] = p.plane[0][(size_t)p.row0 * p.words_per_row[0] + i];
    else
      msg[i] = p.plane[1][(size_t)p.row0 * p.words_per_row[1] + (i - n0)];
  }
}

template <bool ADD>
__global__ __launch_bounds__(256) void k_halo_unpack(HaloPlanes p, int rows, const float* __restrict__ msg) {
  const size_t n0 = (size_t)rows * p.words_per_row[0], n1 = (size_t)rows * p.words_per_row[1];
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n0 + n1; i += (size_t)gridDim.x * 256) {
    float* dst = i < n0 ? p.plane[0] + (size_t)p.row0 * p.words_per_row[0] + i
                        : p.plane[1] + (size_t)p.row0 * p.words_per_row[1] + (i - n0);
    if constexpr (ADD)
      *dst += msg[i];
    else
      *dst = msg[i];
  }
}

struct MsgList {
  const float* m[16];
};

__global__ __launch_bounds__(256) void k_sum_messages(MsgList l, int count, size_t words, float* __restrict__ out) {
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < words; i += (size_t)gridDim.x * 256) {
    float acc = l.m[0][i];
    for (int c = 1; c < count; ++c) acc += l.m[c][i];
    out[i] = acc;
  }
}

__global__ __launch_bounds__(256) void k_plane_max(const float* __restrict__ x, size_t n, unsigned* out) {
  __shared__ float redf[4];
  float mx = 0.f;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) mx = fmaxf(mx, x[i]);
  mx = block_max_all<256>(mx, redf);
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(mx));
}

template <ObjApply OP>
__global__ __launch_bounds__(256) void k_obj_apply(const float2* __restrict__ num, const float* __restrict__ den,
                                                   const unsigned* den_max, float gamma, float beta, float2* obj,
                                                   float2* dir, size_t n) {
  const float delta = gamma * __uint_as_float(*den_max);
  for (size_t o = blockIdx.x * (size_t)256 + threadIdx.x; o < n; o += (size_t)gridDim.x * 256) {
    const float d = den[o] + delta;
    const float2 val = num[o];
    if constexpr (OP == ObjApply::Dm) {
      if (d > 0.f) obj[o] = (1.f / d) * (val + delta * obj[o]);
    } else if constexpr (OP == ObjApply::LsqDirection) {
      dir[o] = d > 0.f ? (1.f / d) * val : make_float2(0.f, 0.f);
    } else {
      if (d > 0.f) obj[o] = obj[o] + (beta / d) * val;
    }
  }
}

__global__ __launch_bounds__(256) void k_err_scatter(const double* __restrict__ local, const int* __restrict__ jmap,
                                                     int count, int per_pattern, double* __restrict__ global) {
  const size_t total = (size_t)count * per_pattern;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
    const size_t l = i / per_pattern, e = i % per_pattern;
    global[(size_t)jmap[l] * per_pattern + e] = local[i];
  }
}

static unsigned stream_grid(size_t n) { return (unsigned)std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 4096)); }

// Tiles below which a tile's patch list is split over eight wavefronts
// instead of four (two blocks per CU), and over sixteen (half a block per CU).
constexpr int kGatherWideTiles = 512, kGatherWidestTiles = 128;

void launch_obj_gather(const ObjGatherArgs& a, ObjOp op) {
  if (a.ntiles <= 0) return;
  dispatch_n(a.n, [&](auto nc) {
    constexpr int N = decltype(nc)::value;
    auto go = [&](auto wc) {
      constexpr int NW = decltype(wc)::value;
      switch (op) {
        case ObjOp::Density: k_obj_gather<N, ObjOp::Density, NW><<<a.ntiles, 64 * NW, 0, a.stream>>>(a); break;
        case ObjOp::DmObject: k_obj_gather<N, ObjOp::DmObject, NW><<<a.ntiles, 64 * NW, 0, a.stream>>>(a); break;
        case ObjOp::LsqDirection: k_obj_gather<N, ObjOp::LsqDirection, NW><<<a.ntiles, 64 * NW, 0, a.stream>>>(a); break;
        case ObjOp::LsqUpdate: k_obj_gather<N, ObjOp::LsqUpdate, NW><<<a.ntiles, 64 * NW, 0, a.stream>>>(a); break;
        case ObjOp::Gradient: k_obj_gather<N, ObjOp::Gradient, NW><<<a.ntiles, 64 * NW, 0, a.stream>>>(a); break;
        case ObjOp::WeightedSum: k_obj_gather<N, ObjOp::WeightedSum, NW><<<a.ntiles, 64 * NW, 0, a.stream>>>(a); break;
      }
    };
    if (a.ntiles < kGatherWidestTiles)
      go(ic<16>{});
    else if (a.ntiles < kGatherWideTiles)
      go(ic<8>{});
    else
      go(ic<4>{});
  });
  PTY_LAUNCH_CHECK("obj_gather");
}

int probe_slices(int count, int per_slice) { return (count + per_slice - 1) / per_slice; }

int probe_acc_blocks(int n) {
  int b = 0;
  dispatch_n(n, [&](auto nc) { b = ProbePix<decltype(nc)::value>::W::BLOCKS; });
  return b;
}

// Patterns per slice: 32, halved (down to 8) while a launch would have
// fewer than 512 blocks, two per compute unit, so that small windows and
// small groups still keep every CU busy; the partial sums then cost at most a
// quarter of the source traffic. (Above 512 blocks the longer per-block
// loops win: at 256 x 256 x 3 in groups of 500, 16 patterns per slice take
// 10% longer than 32.)
int lsq_row_blocks(int n) {
  int b = 0;
  dispatch_n(n, [&](auto nc) { b = LsqPix<decltype(nc)::value>::NRB; });
  return b;
}

int probe_per_slice(int n, int count) {
  const int b = probe_acc_blocks(n);
  int per = 32;
  while (per > 8 && b * probe_slices(count, per) < 512) per /= 2;
  return per;
}

// Upper bound of probe_slices(c, probe_per_slice(n, c)) over 1 <= c <= count:
// a halving happens only below 512 blocks, so it leaves under 1,024.
int probe_slices_max(int n, int count) {
  const int b = probe_acc_blocks(n);
  return std::min(probe_slices(count, 8), std::max(probe_slices(count, 32), (1024 + b - 1) / b));
}

void launch_probe_acc(const ProbeAccArgs& a, PrbOp op) {
  if (a.count <= 0) return;
  if (a.per_slice < 1 || a.per_slice > kProbeSliceMax) throw std::runtime_error("probe_acc: slice size out of range");
  dispatch_nk(a.n, a.k, [&](auto nc, auto kc) {
    constexpr int N = decltype(nc)::value, K = decltype(kc)::value;
    const dim3 grid(ProbePix<N>::W::BLOCKS, probe_slices(a.count, a.per_slice));
    switch (op) {
      case PrbOp::Plain: k_probe_acc<N, K, PrbOp::Plain><<<grid, 256, 0, a.stream>>>(a); break;
      case PrbOp::AlphaWeighted: k_probe_acc<N, K, PrbOp::AlphaWeighted><<<grid, 256, 0, a.stream>>>(a); break;
      case PrbOp::Gradient: k_probe_acc<N, K, PrbOp::Gradient><<<grid, 256, 0, a.stream>>>(a); break;
    }
  });
  PTY_LAUNCH_CHECK("probe_acc");
}

void launch_probe_finish(const ProbeFinishArgs& a) {
  k_probe_finish<<<dim3((a.n * a.n + 255) / 256, a.k), 256, 0, a.stream>>>(a);
  PTY_LAUNCH_CHECK("probe_finish");
}

void launch_probe_apply(const ProbeApplyArgs& a, PrbApply op) {
  const unsigned g = (a.n * a.n + 255) / 256;
  switch (op) {
    case PrbApply::Dm: k_probe_apply<PrbApply::Dm><<<g, 256, 0, a.stream>>>(a); break;
    case PrbApply::LsqDirection: k_probe_apply<PrbApply::LsqDirection><<<g, 256, 0, a.stream>>>(a); break;
    case PrbApply::LsqUpdate: k_probe_apply<PrbApply::LsqUpdate><<<g, 256, 0, a.stream>>>(a); break;
  }
  PTY_LAUNCH_CHECK("probe_apply");
}

void launch_lsq_steps(const LsqStepArgs& a) {
  if (a.count <= 0) return;
  k_lsq_planes<<<(a.n * a.n + 255) / 256, 256, 0, a.stream>>>(a.probe, a.dprobe, a.n, a.k, a.probe_on,
                                                              const_cast<float*>(a.pint),
                                                              const_cast<float2*>(a.pq),
                                                              const_cast<float*>(a.dint));
  PTY_LAUNCH_CHECK("lsq_planes");
  int nrb = 0;
  dispatch_nk(a.n, a.k, [&](auto nc, auto kc) {
    constexpr int N = decltype(nc)::value, K = decltype(kc)::value;
    nrb = LsqPix<N>::NRB;
    auto go = [&](auto mc) {
      constexpr int M = decltype(mc)::value;
      const dim3 grid(LsqPix<N>::NRB, (a.count + M - 1) / M);
      if (a.shift) {
        if (a.probe_on)
          k_lsq_sums<N, K, true, true, M><<<grid, 256, 0, a.stream>>>(a);
        else
          k_lsq_sums<N, K, false, true, M><<<grid, 256, 0, a.stream>>>(a);
      } else {
        if (a.probe_on)
          k_lsq_sums<N, K, true, false, M><<<grid, 256, 0, a.stream>>>(a);
        else
          k_lsq_sums<N, K, false, false, M><<<grid, 256, 0, a.stream>>>(a);
      }
    };
    constexpr int MB = LsqPix<N>::M;
    if ((long)LsqPix<N>::NRB * ((a.count + MB - 1) / MB) < 512)
      go(ic<2>{});
    else
      go(ic<MB>{});
  });
  PTY_LAUNCH_CHECK("lsq_sums");
  k_lsq_solve<<<(a.count + kLsqSolveWaves - 1) / kLsqSolveWaves, 64 * kLsqSolveWaves, 0, a.stream>>>(a, nrb);
  PTY_LAUNCH_CHECK("lsq_solve");
}

// ---------------------------------------------------------------------------
// Probe-mode orthogonalisation (mixed states, Thibault & Menzel 2013)
// ---------------------------------------------------------------------------
// Gram matrix of the modes, G_kl = sum_r P_k(r) conj(P_l(r)), in FP64 by one
// 1024-thread block (fixed summation order).
template <int K>
__global__ __launch_bounds__(1024) void k_mode_gram(const float2* __restrict__ probe, int nn,
                                                    double2* __restrict__ gram) {
  constexpr int NP = K * (K + 1) / 2;
  __shared__ double sh[16][2 * NP];
  double re[NP], im[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) re[i] = im[i] = 0.0;
  for (int q = threadIdx.x; q < nn; q += 1024) {
    float2 v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = probe[(size_t)k * nn + q];
    int i = 0;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int l = k; l < K; ++l, ++i) {
        // P_k conj(P_l)
        re[i] += (double)v[k].x * v[l].x + (double)v[k].y * v[l].y;
        im[i] += (double)v[k].y * v[l].x - (double)v[k].x * v[l].y;
      }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      re[i] += __shfl_down(re[i], off, 64);
      im[i] += __shfl_down(im[i], off, 64);
    }
    if (lane == 0) {
      sh[wid][2 * i] = re[i];
      sh[wid][2 * i + 1] = im[i];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int i = 0;
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int l = k; l < K; ++l, ++i) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < 16; ++w) {
          a += sh[w][2 * i];
          b += sh[w][2 * i + 1];
        }
        gram[k * K + l] = make_double2(a, b);
        gram[l * K + k] = make_double2(a, -b);
      }
  }
}

// Eigenvectors V of the Hermitian Gram matrix by cyclic complex Jacobi
// rotations in FP64 (one thread; K <= 4), columns ordered by decreasing
// eigenvalue and each phased so that its largest-magnitude entry (the first
// of equal ones) is real and positive.  Writes the mixing matrix
// mix[k][l] = conj(V[l][k]) of the new modes P'_k = sum_l mix[k][l] P_l.
template <int K>
__global__ void k_mode_eigen(const double2* __restrict__ gram, float2* __restrict__ mix) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double gr[K][K], gi[K][K], vr[K][K], vi[K][K];
#pragma unroll
  for (int r = 0; r < K; ++r)
#pragma unroll
    for (int q = 0; q < K; ++q) {
      gr[r][q] = gram[r * K + q].x;
      gi[r][q] = gram[r * K + q].y;
      vr[r][q] = r == q ? 1.0 : 0.0;
      vi[r][q] = 0.0;
    }
#pragma unroll 1
  for (int sweep = 0; sweep < 12; ++sweep) {
#pragma unroll
    for (int p = 0; p < K - 1; ++p)
#pragma unroll
      for (int q = p + 1; q < K; ++q) {
        const double br = gr[p][q], bi = gi[p][q];
        const double ab = sqrt(br * br + bi * bi);
        const double a = gr[p][p], d = gr[q][q];
        if (!(ab > 1e-18 * (fabs(a) + fabs(d)))) continue;
        const double er = br / ab, ei = -bi / ab;   // conj(b) / |b|
        const double tau = (d - a) / (2.0 * ab);
        const double t = fabs(tau) > 1e150 ? 0.5 / tau
                                            : (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
        // U on (p, q): U_pp = c, U_pq = s, U_qp = -s e, U_qq = c e with e = conj(b)/|b|
        const double u10r = -s * er, u10i = -s * ei, u11r = c * er, u11i = c * ei;
        // columns: G <- G U, V <- V U
#pragma unroll
        for (int r = 0; r < K; ++r) {
          const double xr = gr[r][p], xi = gi[r][p], yr = gr[r][q], yi = gi[r][q];
          gr[r][p] = c * xr + (yr * u10r - yi * u10i);
          gi[r][p] = c * xi + (yr * u10i + yi * u10r);
          gr[r][q] = s * xr + (yr * u11r - yi * u11i);
          gi[r][q] = s * xi + (yr * u11i + yi * u11r);
          const double vxr = vr[r][p], vxi = vi[r][p], vyr = vr[r][q], vyi = vi[r][q];
          vr[r][p] = c * vxr + (vyr * u10r - vyi * u10i);
          vi[r][p] = c * vxi + (vyr * u10i + vyi * u10r);
          vr[r][q] = s * vxr + (vyr * u11r - vyi * u11i);
          vi[r][q] = s * vxi + (vyr * u11i + vyi * u11r);
        }
        // rows: G <- U^H G
#pragma unroll
        for (int r = 0; r < K; ++r) {
          const double xr = gr[p][r], xi = gi[p][r], yr = gr[q][r], yi = gi[q][r];
          // conj(u10) y = (u10r - i u10i)(yr + i yi)
          gr[p][r] = c * xr + (u10r * yr + u10i * yi);
          gi[p][r] = c * xi + (u10r * yi - u10i * yr);
          gr[q][r] = s * xr + (u11r * yr + u11i * yi);
          gi[q][r] = s * xi + (u11r * yi - u11i * yr);
        }
        gr[p][q] = gi[p][q] = gr[q][p] = gi[q][p] = 0.0;
        gi[p][p] = gi[q][q] = 0.0;
      }
  }
  // order by decreasing eigenvalue (stable selection)
  int ord[K];
  bool used[K];
#pragma unroll
  for (int k = 0; k < K; ++k) used[k] = false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int best = -1;
#pragma unroll
    for (int m = 0; m < K; ++m)
      if (!used[m] && (best < 0 || gr[m][m] > gr[best][best])) best = m;
    used[best] = true;
    ord[k] = best;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int col = ord[k];
    double cr[K], ci[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
      cr[r] = vr[r][col];
      ci[r] = vi[r][col];
    }
    int im = 0;
    double mm = cr[0] * cr[0] + ci[0] * ci[0];
#pragma unroll
    for (int r = 1; r < K; ++r) {
      const double m2 = cr[r] * cr[r] + ci[r] * ci[r];
      if (m2 > mm) {
        mm = m2;
        im = r;
      }
    }
    const double am = sqrt(mm);
    const double fr = cr[im] / am, fi = -ci[im] / am;   // conj(v_im) / |v_im|
#pragma unroll
    for (int l = 0; l < K; ++l) {
      const double xr = cr[l] * fr - ci[l] * fi, xi = cr[l] * fi + ci[l] * fr;
      mix[k * K + l] = make_float2((float)xr, (float)-xi);   // conj(V[l][k])
    }
  }
}

// x[set][k][q] <- sum_l mix[k][l] x[set][l][q] for every set (the probe: one
// set; DM exit waves: one per pattern).
template <int K>
__global__ __launch_bounds__(256) void k_mode_mix(float2* __restrict__ x, const float2* __restrict__ mix, size_t nn,
                                                  size_t sets) {
  const size_t i = blockIdx.x * (size_t)256 + threadIdx.x;
  if (i >= sets * nn) return;
  const size_t set = i / nn, q = i % nn;
  float2* base = x + set * K * nn + q;
  float2 v[K], m[K * K];
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = base[(size_t)k * nn];
#pragma unroll
  for (int e = 0; e < K * K; ++e) m[e] = mix[e];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int l = 0; l < K; ++l) acc = acc + cmul(m[k * K + l], v[l]);
    base[(size_t)k * nn] = acc;
  }
}

void launch_orthogonalise_modes(float2* probe, float2* psi, int n, int k, int j, double2* gram, float2* mix,
                                hipStream_t s) {
  if (k <= 1) return;
  const size_t nn = (size_t)n * n;
  auto run = [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    k_mode_gram<K><<<1, 1024, 0, s>>>(probe, (int)nn, gram);
    k_mode_eigen<K><<<1, 64, 0, s>>>(gram, mix);
    k_mode_mix<K><<<(unsigned)((nn + 255) / 256), 256, 0, s>>>(probe, mix, nn, 1);
    if (psi) k_mode_mix<K><<<(unsigned)(((size_t)j * nn + 255) / 256), 256, 0, s>>>(psi, mix, nn, (size_t)j);
  };
  switch (k) {
    case 2: run(ic<2>{}); break;
    case 3: run(ic<3>{}); break;
    case 4: run(ic<4>{}); break;
    default: throw std::invalid_argument("unsupported mode count");
  }
  PTY_LAUNCH_CHECK("orthogonalise_modes");
}

// Moves the group's positions by their shifts, kept inside the object
// (0 <= y <= lim_y, 0 <= x <= lim_x), and splits them again into floor and
// fraction.
__global__ void k_pos_update(PosInfo* pos, const int* jlist, const float2* shift, int count, int lim_y,
                             int lim_x) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= count) return;
  const int j = jlist[b];
  PosInfo p = pos[j];
  const float2 sh = shift[b];
  auto move = [](int& i, float& f, double d, int lim) {
    const double r = fmin(fmax((double)i + (double)f + d, 0.0), (double)lim);
    i = (int)floor(r);
    f = (float)(r - i);
    if (f >= 1.f) {   // rounding to float reached the next integer
      i += 1;
      f = 0.f;
    }
  };
  move(p.iy, p.fy, sh.x, lim_y);
  move(p.ix, p.fx, sh.y, lim_x);
  pos[j] = p;
}

void launch_pos_update(PosInfo* pos, const int* jlist, const float2* shift, int count, int lim_y, int lim_x,
                       hipStream_t s) {
  if (count <= 0) return;
  k_pos_update<<<(count + 127) / 128, 128, 0, s>>>(pos, jlist, shift, count, lim_y, lim_x);
  PTY_LAUNCH_CHECK("pos_update");
}

// Positions held on the device as J x 2 float32 (y, x) top-left corners:
// integer floor and fraction of each, clamped into [0, lim] (a NaN becomes 0)
// so that every patch stays inside the object.
__global__ void k_pos_from_yx(const float* __restrict__ yx, int count, int lim_y, int lim_x,
                              PosInfo* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count) return;
  auto split = [](float v, int lim, int& i, float& f) {
    const float r = fminf(fmaxf(v, 0.f), (float)lim);
    i = (int)floorf(r);
    f = r - (float)i;
  };
  PosInfo p;
  split(yx[2 * (size_t)j], lim_y, p.iy, p.fy);
  split(yx[2 * (size_t)j + 1], lim_x, p.ix, p.fx);
  out[j] = p;
}

// Tile lists built on the device from device positions: every object tile
// gets an entry (empty ones included) listing, in slot order, the patches
// whose (N+1)^2 footprint overlaps it; the same lists the host builds from
// loaded positions.  Count per tile, exclusive scan, then an ordered fill
// (wave ballots), so the lists do not depend on scheduling.
__device__ __forceinline__ bool tile_hit(const PosInfo& p, int n, int ty, int tx, int nty, int ntx) {
  const int y0 = p.iy / kTileH, y1 = min(nty - 1, (p.iy + n) / kTileH);
  const int x0 = p.ix / kTileW, x1 = min(ntx - 1, (p.ix + n) / kTileW);
  return ty >= y0 && ty <= y1 && tx >= x0 && tx <= x1;
}

__global__ __launch_bounds__(256) void k_tiles_count(const PosInfo* __restrict__ pos, const int* __restrict__ jlist,
                                                     int count, int n, int nty, int ntx, int* __restrict__ cnt) {
  __shared__ int tot;
  const int t = blockIdx.x, ty = t / ntx, tx = t % ntx;
  if (threadIdx.x == 0) tot = 0;
  __syncthreads();
  int c = 0;
  for (int s = threadIdx.x; s < count; s += 256) c += tile_hit(pos[jlist[s]], n, ty, tx, nty, ntx) ? 1 : 0;
  atomicAdd(&tot, c);   // integers: the same total in any order
  __syncthreads();
  if (threadIdx.x == 0) cnt[t] = tot;
}

__global__ __launch_bounds__(1024) void k_tiles_scan(const int* __restrict__ cnt, int ntiles, int ntx,
                                                     TileEntry* __restrict__ tiles) {
  __shared__ int wsum[16];
  __shared__ int carry;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < ntiles; base += 1024) {
    const int t = base + threadIdx.x;
    const int v = t < ntiles ? cnt[t] : 0;
    int x = v;   // inclusive scan inside the wavefront
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int beg = carry + x - v;
    for (int i = 0; i < w; ++i) beg += wsum[i];
    if (t < ntiles) tiles[t] = TileEntry{(t / ntx) * kTileH, (t % ntx) * kTileW, beg, beg + v};
    __syncthreads();
    if (threadIdx.x == 1023) carry = beg + v;
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_tiles_fill(const PosInfo* __restrict__ pos, const int* __restrict__ jlist,
                                                    int count, int n, int nty, int ntx,
                                                    const TileEntry* __restrict__ tiles,
                                                    PatchRef* __restrict__ refs) {
  __shared__ int wcnt[4];
  const int t = blockIdx.x, ty = t / ntx, tx = t % ntx;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int next = tiles[t].beg;
  for (int base = 0; base < count; base += 256) {
    const int s = base + threadIdx.x;
    bool hit = false;
    int j = 0;
    PosInfo p{};
    if (s < count) {
      j = jlist[s];
      p = pos[j];
      hit = tile_hit(p, n, ty, tx, nty, ntx);
    }
    const unsigned long long bal = __ballot(hit);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[w] = __popcll(bal);
    __syncthreads();
    int off = next;
    for (int i = 0; i < w; ++i) off += wcnt[i];
    if (hit) refs[off + before] = PatchRef{s, j, p.iy, p.ix, p.fy, p.fx, 0, 0};
    next += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
}

__global__ void k_iota_i32(int* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = i;
}

void launch_pos_from_yx(const float* yx, int count, int lim_y, int lim_x, PosInfo* out, hipStream_t s) {
  if (count <= 0) return;
  k_pos_from_yx<<<(count + 127) / 128, 128, 0, s>>>(yx, count, lim_y, lim_x, out);
  PTY_LAUNCH_CHECK("pos_from_yx");
}

size_t device_tile_refs_max(int n, int count) {
  return (size_t)count * (size_t)(n / kTileH + 2) * (size_t)(n / kTileW + 2);
}

void launch_build_tiles(const PosInfo* pos, const int* jlist, int count, int n, int h, int w, int* cnt,
                        TileEntry* tiles, PatchRef* refs, hipStream_t s) {
  const int nty = (h + kTileH - 1) / kTileH, ntx = (w + kTileW - 1) / kTileW, nt = nty * ntx;
  k_tiles_count<<<nt, 256, 0, s>>>(pos, jlist, count, n, nty, ntx, cnt);
  PTY_LAUNCH_CHECK("tiles_count");
  k_tiles_scan<<<1, 1024, 0, s>>>(cnt, nt, ntx, tiles);
  PTY_LAUNCH_CHECK("tiles_scan");
  k_tiles_fill<<<nt, 256, 0, s>>>(pos, jlist, count, n, nty, ntx, tiles, refs);
  PTY_LAUNCH_CHECK("tiles_fill");
}

void launch_iota_i32(int* p, int n, hipStream_t s) {
  if (n <= 0) return;
  k_iota_i32<<<(n + 255) / 256, 256, 0, s>>>(p, n);
  PTY_LAUNCH_CHECK("iota");
}

// One workgroup runs the iteration up to 64 x 64.  At 128 x 128 (K = 1) the
// kernel was measured slower than the per-position launches (36.7 vs 24.2 us
// per position): 1,024 threads leave 128 registers a lane and one CU's VALU
// issue is the limit, so larger windows use the launches, which spread each
// transform over many CUs.
bool epie_fused_supported(int n, int k) {
  if (n == 32 || n == 64) return k >= 1 && k <= 4;
  return false;
}

void launch_epie_fused(const EpieRunArgs& a) {
  if (a.count <= 0) return;
  if (!epie_fused_supported(a.n, a.k)) throw std::invalid_argument("fused ePIE: unsupported window");
  auto go = [&](auto nc, auto kc) {
    constexpr int N = decltype(nc)::value, K = decltype(kc)::value;
    if constexpr (N == 32 || (N == 64 && K <= 2)) {
      // footprint and probe on chip
      using G = EpieFbGeo<N, K>;
      static_assert(G::lds <= G::budget, "fused ePIE field and footprints must fit in LDS");
      PTY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_epie_fused_fb<N, K>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)G::lds));
      k_epie_fused_fb<N, K><<<1, G::NT, G::lds, a.stream>>>(a);
    } else if constexpr (N == 64) {
      using G = EpieGeo<N, K>;
      static_assert(G::lds <= G::budget, "fused ePIE field must fit in LDS");
      PTY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_epie_fused<N, K>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)G::lds));
      k_epie_fused<N, K><<<1, G::NT, G::lds, a.stream>>>(a);
    }
  };
  if (a.n == 32) dispatch_k<32>(a.k, go);
  else dispatch_k<64>(a.k, go);
  PTY_LAUNCH_CHECK("epie_fused");
}

void launch_epie_update(const EpieArgs& a) {
  dispatch_nk(a.n, a.k, [&](auto nc, auto kc) {
    constexpr int N = decltype(nc)::value, K = decltype(kc)::value;
    const unsigned g = (N * N + 255) / 256, gf = ((N + 1) * (N + 1) + 255) / 256;
    k_epie_max<N, K><<<std::min<unsigned>(g, kEpieMaxBlocks), 256, 0, a.stream>>>(a);
    k_epie_apply<N, K><<<g + gf, 256, 0, a.stream>>>(a, (int)g);
  });
  PTY_LAUNCH_CHECK("epie_update");
}

void launch_dm_init(const DmInitArgs& a) {
  dispatch_nk(a.n, a.k, [&](auto nc, auto kc) {
    constexpr int N = decltype(nc)::value, K = decltype(kc)::value;
    const dim3 grid((N * N + 255) / 256, a.j);
    k_dm_init<N, K><<<grid, 256, 0, a.stream>>>(a);
  });
  PTY_LAUNCH_CHECK("dm_init");
}

void launch_fill_u32(unsigned* p, size_t n, unsigned v, hipStream_t s) {
  if (n == 0) return;
  k_fill_u32<<<grid_for(n, 256, 4096), 256, 0, s>>>(p, n, v);
  PTY_LAUNCH_CHECK("fill");
}

void launch_amplitude(const float* counts, float* amp, double* totals, int n, int j, hipStream_t s) {
  const size_t total = (size_t)j * n * n;
  k_amplitude<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(counts, amp, n, total);
  PTY_LAUNCH_CHECK("amplitude");
  if (totals) launch_pattern_totals(counts, totals, n, j, s);
}

void launch_apply_mask(float* amp, const unsigned char* mask, int n, int j, hipStream_t s) {
  const size_t total = (size_t)j * n * n;
  k_apply_mask<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(amp, mask, (size_t)n * n, total);
  PTY_LAUNCH_CHECK("apply_mask");
}

void launch_pattern_totals(const float* x, double* totals, int n, int j, hipStream_t s) {
  k_pattern_totals<<<j, 256, 0, s>>>(x, totals, n);
  PTY_LAUNCH_CHECK("pattern_totals");
}

void launch_amp_totals(const float* amp, double* totals, int n, int j, hipStream_t s) {
  k_amp_totals<<<j, 256, 0, s>>>(amp, totals, n);
  PTY_LAUNCH_CHECK("amp_totals");
}

void launch_probe_intensity(const float2* probe, float* pint, int n, int k, hipStream_t s, unsigned* zero) {
  k_probe_intensity<<<(n * n + 255) / 256, 256, 0, s>>>(probe, pint, n, k, zero);
  PTY_LAUNCH_CHECK("probe_intensity");
}

void launch_err_reduce(const double* errp, int count, double* out, hipStream_t s, int* slot, bool advance) {
  k_err_reduce<<<1, 1024, 0, s>>>(errp, count, out, slot, advance ? 1 : 0);
  PTY_LAUNCH_CHECK("err_reduce");
}

void launch_posgrad_reduce(const double* part, int count, int nrb, float* out, const int* jlist, hipStream_t s) {
  if (count <= 0) return;
  k_posgrad_reduce<<<(count + 127) / 128, 128, 0, s>>>(part, count, nrb, out, jlist);
  PTY_LAUNCH_CHECK("posgrad_reduce");
}

void launch_scale_f32(float* p, size_t n, float s, hipStream_t st) {
  if (n == 0) return;
  k_scale_f32<<<grid_for(n, 256, 4096), 256, 0, st>>>(p, n, s);
  PTY_LAUNCH_CHECK("scale_f32");
}

void launch_scale_c64(float2* p, size_t n, float s, hipStream_t st) {
  if (n == 0) return;
  k_scale_c64<<<grid_for(n, 256, 4096), 256, 0, st>>>(p, n, s);
  PTY_LAUNCH_CHECK("scale_c64");
}


void launch_halo_pack(const HaloPlanes& p, int rows, float* msg, hipStream_t s) {
  const size_t n = (size_t)rows * (p.words_per_row[0] + p.words_per_row[1]);
  if (n == 0) return;
  k_halo_pack<<<stream_grid(n), 256, 0, s>>>(p, rows, msg);
  PTY_LAUNCH_CHECK("halo_pack");
}

void launch_halo_unpack(const HaloPlanes& p, int rows, const float* msg, bool add, hipStream_t s) {
  const size_t n = (size_t)rows * (p.words_per_row[0] + p.words_per_row[1]);
  if (n == 0) return;
  if (add)
    k_halo_unpack<true><<<stream_grid(n), 256, 0, s>>>(p, rows, msg);
  else
    k_halo_unpack<false><<<stream_grid(n), 256, 0, s>>>(p, rows, msg);
  PTY_LAUNCH_CHECK("halo_unpack");
}

void launch_sum_messages(const float* const* msgs, int count, size_t words, float* out, hipStream_t s) {
  if (count < 1 || count > 16) throw std::runtime_error("sum_messages: 1 to 16 messages");
  MsgList l{};
  for (int i = 0; i < count; ++i) l.m[i] = msgs[i];
  k_sum_messages<<<stream_grid(words), 256, 0, s>>>(l, count, words, out);
  PTY_LAUNCH_CHECK("sum_messages");
}

void launch_plane_max(const float* x, size_t n, unsigned* out, hipStream_t s) {
  if (n == 0) return;
  k_plane_max<<<stream_grid(n), 256, 0, s>>>(x, n, out);
  PTY_LAUNCH_CHECK("plane_max");
}

void launch_obj_apply(const float2* num, const float* den, const unsigned* den_max, float gamma, float beta,
                      float2* obj, float2* dir, size_t n, ObjApply op, hipStream_t s) {
  if (n == 0) return;
  const unsigned g = stream_grid(n);
  switch (op) {
    case ObjApply::Dm: k_obj_apply<ObjApply::Dm><<<g, 256, 0, s>>>(num, den, den_max, gamma, beta, obj, dir, n); break;
    case ObjApply::LsqDirection:
      k_obj_apply<ObjApply::LsqDirection><<<g, 256, 0, s>>>(num, den, den_max, gamma, beta, obj, dir, n);
      break;
    case ObjApply::LsqUpdate:
      k_obj_apply<ObjApply::LsqUpdate><<<g, 256, 0, s>>>(num, den, den_max, gamma, beta, obj, dir, n);
      break;
  }
  PTY_LAUNCH_CHECK("obj_apply");
}

void launch_err_scatter(const double* local, const int* jmap, int count, int per_pattern, double* global,
                        hipStream_t s) {
  if (count <= 0) return;
  k_err_scatter<<<stream_grid((size_t)count * per_pattern), 256, 0, s>>>(local, jmap, count, per_pattern, global);
  PTY_LAUNCH_CHECK("err_scatter");
}

}  // namespace pty
