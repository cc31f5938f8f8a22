// Register-resident DFT building blocks for the Fresnel FFT kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

namespace hh {

// cos(2 pi m / 64) for m = 0..16; every W_64^m needed below follows by symmetry.
__device__ constexpr double kCos64[17] = {
    1.0,
    0.99518472667219693, 0.98078528040323043, 0.95694033573220882, 0.92387953251128674,
    0.88192126434835505, 0.83146961230254524, 0.77301045336273699, 0.70710678118654757,
    0.63439328416364549, 0.55557023301960229, 0.47139673682599781, 0.38268343236508984,
    0.29028467725446233, 0.19509032201612833, 0.09801714032956077, 0.0};

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// x * W_64^m for 0 <= m < 32, W = exp(-2 pi i / 64).  `m` is a compile-time
// constant after unrolling, so the branches fold away.
__device__ __forceinline__ float2 mul_w64(float2 x, int m) {
  constexpr float h = 0.70710678118654752f;
  if (m == 0) return x;
  if (m == 16) return make_float2(x.y, -x.x);                        // * (-i)
  if (m == 8) return make_float2((x.x + x.y) * h, (x.y - x.x) * h);  // * (1 - i)/sqrt2
  if (m == 24) return make_float2((x.y - x.x) * h, -(x.x + x.y) * h);  // * (-1 - i)/sqrt2
  float2 w;
  if (m < 16) {
    w = make_float2((float)kCos64[m], -(float)kCos64[16 - m]);
  } else {
    w = make_float2(-(float)kCos64[32 - m], -(float)kCos64[m - 16]);
  }
  return cmul(x, w);
}

__host__ __device__ constexpr int bitrev(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r |= ((i >> b) & 1) << (bits - 1 - b);
  return r;
}

__host__ __device__ constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n >> 1); }

// In-place forward DFT of R points held in registers, natural order in and out:
// radix-2 decimation in frequency, then a compile-time bit-reversal rename.
template <int R>
__device__ __forceinline__ void dft_reg(float2 (&v)[R]) {
  static_assert(R >= 1 && R <= 64 && (R & (R - 1)) == 0, "R must be a power of two <= 64");
  if constexpr (R > 1) {
#pragma unroll
    for (int len = R; len >= 2; len >>= 1) {
      const int half = len >> 1;
      const int step = 64 / len;
#pragma unroll
      for (int s = 0; s < R; s += len) {
#pragma unroll
        for (int k = 0; k < half; ++k) {
          const float2 a = v[s + k], b = v[s + k + half];
          v[s + k] = cadd(a, b);
          v[s + k + half] = mul_w64(csub(a, b), k * step);
        }
      }
    }
    float2 t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) t[bitrev(i, ilog2(R))] = v[i];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = t[i];
  }
}

// Two-pass Stockham decomposition of an N-point transform over T threads with
// E = N / T points per thread: pass 0 is one radix-E DFT per thread, pass 1 is
// E / T radix-T DFTs per thread (twiddled by W_N^{j k}), with one LDS exchange.
template <int N>
struct FftShape {
  static constexpr int E = (N <= 32) ? N : (N == 64 ? 8 : (N <= 256 ? 16 : (N <= 1024 ? 32 : 64)));
  static constexpr int T = N / E;
  static constexpr int PADN = N + N / E;  // LDS complex slots per transform (1 pad per E)
  static_assert(T <= E && E % T == 0, "bad FFT shape");
};

// Pass 1 of the two-pass transform.  On entry v[i] holds element t + T*i of the
// pass-0 output; on exit v[i] holds X[t + T*i] (natural order).
template <int N>
__device__ __forceinline__ void fft_pass1(float2 (&v)[FftShape<N>::E], int t,
                                          const float2 *__restrict__ tw) {
  constexpr int E = FftShape<N>::E, T = FftShape<N>::T, B = E / T;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + T * b;
    float2 u[T];
#pragma unroll
    for (int k = 0; k < T; ++k) u[k] = v[b + k * B];
#pragma unroll
    for (int k = 1; k < T; ++k) u[k] = cmul(u[k], tw[j * k]);
    dft_reg<T>(u);
#pragma unroll
    for (int k = 0; k < T; ++k) v[b + k * B] = u[k];
  }
}

}  // namespace hh
