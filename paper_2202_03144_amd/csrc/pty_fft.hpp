// Register- and LDS-resident FFT building blocks for gfx950 (wave64).
//
// A length-N line (one row or one column of an N x N window) is held by a
// group of T = N / R threads, R complex values per thread, in the "strided"
// layout: thread t owns elements t + T*m, m = 0..R-1, in register m.  One line
// transform is the four-step factorisation N = R * T:
//   1. an R-point DFT over m inside each thread's registers,
//   2. multiplication by the twiddles W_N^(t q),
//   3. an exchange through LDS and R/T T-point DFTs per thread,
// which leaves the output again in the strided layout (thread t owns X[t + T m]).
// The small in-register DFTs are split radix-2 recursions ending in radix-4
// butterflies; their twiddles are compile-time constants.  The W_N table comes
// from the host, computed in float64.
#pragma once
#include <hip/hip_runtime.h>

namespace pty {

__device__ __forceinline__ float2 operator+(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 operator-(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 operator*(float s, float2 a) { return make_float2(s * a.x, s * a.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// conj(a) * b
__device__ __forceinline__ float2 cconjmul(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// x * (-i) for the forward direction, x * (+i) for the inverse
template <bool INV>
__device__ __forceinline__ float2 mul_i(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// cos and sin of 2 pi k / 32 for k = 0..7 (first octant)
struct Oct32 {
  static constexpr float c[8] = {1.0f, 0.98078528040323044913f, 0.92387953251128675613f,
                                 0.83146961230254523708f, 0.70710678118654752440f,
                                 0.55557023301960222474f, 0.38268343236508977173f,
                                 0.19509032201612826785f};
  static constexpr float s[8] = {0.0f, 0.19509032201612826785f, 0.38268343236508977173f,
                                 0.55557023301960222474f, 0.70710678118654752440f,
                                 0.83146961230254523708f, 0.92387953251128675613f,
                                 0.98078528040323044913f};
};

// x * W_R^k, W_R = exp(-+ 2 pi i / R), for 0 <= k < R/2 and R <= 32
template <int R, bool INV>
__device__ __forceinline__ float2 twiddle_small(int k, float2 x) {
  const int idx = k * (32 / R);  // angle 2 pi idx / 32, idx in [0, 16)
  if (idx == 0) return x;
  if (idx == 8) return mul_i<INV>(x);
  float c, s;
  if (idx < 8) {
    c = Oct32::c[idx];
    s = Oct32::s[idx];
  } else {
    c = -Oct32::s[idx - 8];
    s = Oct32::c[idx - 8];
  }
  // forward: x (c - i s); inverse: x (c + i s)
  if (INV) return make_float2(x.x * c - x.y * s, x.y * c + x.x * s);
  return make_float2(x.x * c + x.y * s, x.y * c - x.x * s);
}

template <int R, bool INV>
struct Dft {
  __device__ __forceinline__ static void run(float2* v) {
    float2 e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = v[2 * i];
      o[i] = v[2 * i + 1];
    }
    Dft<R / 2, INV>::run(e);
    Dft<R / 2, INV>::run(o);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const float2 t = twiddle_small<R, INV>(k, o[k]);
      v[k] = e[k] + t;
      v[k + R / 2] = e[k] - t;
    }
  }
};

template <bool INV>
struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float2 s02 = v[0] + v[2], d02 = v[0] - v[2];
    const float2 s13 = v[1] + v[3], d13 = mul_i<INV>(v[1] - v[3]);
    v[0] = s02 + s13;
    v[2] = s02 - s13;
    v[1] = d02 + d13;
    v[3] = d02 - d13;
  }
};

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* v) {
    const float2 a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <bool INV>
struct Dft<1, INV> {
  __device__ __forceinline__ static void run(float2*) {}
};

// Compile-time factorisation of a supported window size.
template <int N>
struct FftShape;
template <>
struct FftShape<32> { static constexpr int R = 8, T = 4; };
template <>
struct FftShape<64> { static constexpr int R = 8, T = 8; };
template <>
struct FftShape<128> { static constexpr int R = 16, T = 8; };
template <>
struct FftShape<256> { static constexpr int R = 16, T = 16; };
template <>
struct FftShape<512> { static constexpr int R = 32, T = 16; };

// LDS float2 words per line for the exchange (row stride T + 1 avoids bank conflicts)
template <int N>
struct LineLds {
  static constexpr int R = FftShape<N>::R, T = FftShape<N>::T;
  static constexpr int words = R * (T + 1);
};

// Orders LDS traffic between the lanes of one wavefront.  A wavefront's LDS
// instructions execute in issue order, so a fence that keeps the compiler from
// moving them across this point is all the exchange inside one wave needs.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One length-N line transform held by T threads (t = index within the line),
// unscaled (forward: sum x e^{-2 pi i ...}; inverse: sum x e^{+2 pi i ...}).
// The T threads of a line must be consecutive lanes of one wavefront: the
// exchange is synchronised at wave level only.
// `buf`: this line's LDS exchange area (LineLds<N>::words float2).
// `tw`: W_N^i = exp(-2 pi i i / N), i = 0..N-1 (LDS or global).
template <int N, bool INV>
__device__ __forceinline__ void line_fft(float2* v, float2* buf, const float2* tw, int t) {
  constexpr int R = FftShape<N>::R, T = FftShape<N>::T;
  Dft<R, INV>::run(v);
#pragma unroll
  for (int q = 1; q < R; ++q) {
    float2 w = tw[(t * q) & (N - 1)];
    if (INV) w.y = -w.y;
    v[q] = cmul(v[q], w);
  }
  static_assert(64 % T == 0, "a line must not straddle wavefronts");
#pragma unroll
  for (int q = 0; q < R; ++q) buf[q * (T + 1) + t] = v[q];
  wave_sync();
#pragma unroll
  for (int i = 0; i < R / T; ++i) {
    float2 u[T];
    const float2* row = buf + (t + i * T) * (T + 1);
#pragma unroll
    for (int s = 0; s < T; ++s) u[s] = row[s];
    Dft<T, INV>::run(u);
#pragma unroll
    for (int s = 0; s < T; ++s) v[i + (R / T) * s] = u[s];
  }
  wave_sync();
}

}  // namespace pty
