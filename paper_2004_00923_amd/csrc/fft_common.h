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

// Mixed-radix Stockham FFT of N points over T = N / E threads, E = min(16, N)
// points per thread.  Pass p has radix R_p (E for the first passes, the
// remaining factor for the last) and stride NS_p = R_0 ... R_{p-1}; each thread
// does E / R_p radix-R_p DFTs in registers, twiddled by W_N^{(j mod NS_p) k N/(NS_p R_p)},
// and the passes exchange data through LDS.  1024 = 16 * 16 * 4.
__host__ __device__ constexpr int fft_radix(int N, int E, int p) {
  int ns = 1, r = E < N ? E : N;
  for (int q = 0; q < p; ++q) {
    ns *= r;
    r = (N / ns) < E ? (N / ns) : E;
  }
  return r;
}
__host__ __device__ constexpr int fft_ns(int N, int E, int p) {
  int ns = 1;
  for (int q = 0; q < p; ++q) ns *= fft_radix(N, E, q);
  return ns;
}
__host__ __device__ constexpr int fft_npasses(int N, int E) {
  int p = 0, ns = 1;
  while (ns < N) {
    ns *= fft_radix(N, E, p);
    ++p;
  }
  return p;
}
// LDS slot of logical element e: one pad slot per 32 elements spreads the banks.
__host__ __device__ constexpr int fft_pad(int e) { return e + (e >> 5); }

__host__ __device__ constexpr int fft_e(int N, int EP) { return N < EP ? N : EP; }

template <int N, int EP = 16>
struct FftCfg {
  static constexpr int E = N < EP ? N : EP;
  static constexpr int T = N / E;
  static constexpr int P = fft_npasses(N, E);
  static constexpr int LDSN = fft_pad(N - 1) + 1;  // LDS slots per transform
};

// Exchange barrier of the passes below.  WAVE = false: the workgroup's barrier.
// WAVE = true, for a transform held by exactly one wave in an LDS area of its own:
// the LDS instructions of one wave are carried out in the order they are issued,
// so a compiler-level barrier that keeps the writes before the reads suffices.
template <bool WAVE>
__device__ __forceinline__ void fft_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// Passes P.. of the transform.  On entry v[i] holds element t + T*i of the
// sequence entering pass P; on return v[i] = X[t + T*i] (natural order).
// slot(e) maps a logical element of this transform to its LDS slot; every
// thread of the workgroup must call this (it contains barriers; with WAVE every
// thread of the wave, which must hold the whole transform).
// SPLIT = false: lds holds float2 slots and each exchange moves whole complex
// values.  SPLIT = true: lds holds float slots (half the LDS) and each exchange
// moves the real parts, then the imaginary parts.
template <int N, int EP, int P, bool SPLIT = false, bool WAVE = false, class Slot, class L>
__device__ __forceinline__ void fft_passes(float2 (&v)[fft_e(N, EP)], int t, const float2 *__restrict__ tw,
                                           L *lds, Slot slot) {
  constexpr int E = FftCfg<N, EP>::E, T = FftCfg<N, EP>::T;
  constexpr int R = fft_radix(N, E, P), NS = fft_ns(N, E, P), B = E / R;
  constexpr bool last = (P == FftCfg<N, EP>::P - 1);
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + T * b;
    float2 u[R];
#pragma unroll
    for (int k = 0; k < R; ++k) u[k] = v[b + B * k];
    if constexpr (NS > 1) {
      const int jm = j & (NS - 1);
#pragma unroll
      for (int k = 1; k < R; ++k) u[k] = cmul(u[k], tw[jm * k * (N / (NS * R))]);
    }
    dft_reg<R>(u);
    if constexpr (last || SPLIT) {
#pragma unroll
      for (int k = 0; k < R; ++k) v[b + B * k] = u[k];
    } else {
      const int base = (j / NS) * NS * R + (j & (NS - 1));
#pragma unroll
      for (int k = 0; k < R; ++k) lds[slot(base + k * NS)] = u[k];
    }
  }
  if constexpr (!last) {
    if constexpr (SPLIT) {
      // element (b, k) of this pass goes to logical position base(b) + k NS
#pragma unroll
      for (int half = 0; half < 2; ++half) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const int j = t + T * b;
          const int base = (j / NS) * NS * R + (j & (NS - 1));
#pragma unroll
          for (int k = 0; k < R; ++k) lds[slot(base + k * NS)] = half ? v[b + B * k].y : v[b + B * k].x;
        }
        fft_sync<WAVE>();
        float w[E];
#pragma unroll
        for (int i = 0; i < E; ++i) w[i] = lds[slot(t + T * i)];
        fft_sync<WAVE>();  // reads done before the next writes
#pragma unroll
        for (int i = 0; i < E; ++i) {
          if (half) v[i].y = w[i];
          else v[i].x = w[i];
        }
      }
      fft_passes<N, EP, P + 1, SPLIT, WAVE>(v, t, tw, lds, slot);
    } else {
      fft_sync<WAVE>();
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = lds[slot(t + T * i)];
      if constexpr (P + 1 < FftCfg<N, EP>::P - 1) fft_sync<WAVE>();  // reads done before the next pass writes
      fft_passes<N, EP, P + 1, SPLIT, WAVE>(v, t, tw, lds, slot);
    }
  }
}

}  // namespace hh
