// Projection-first image (steps (d)+(e) evaluated from the frames).
//
// Eq. (1) is linear in the frame, so the projected hologram of Eq. (6) is
//   Y_k = sum_t H_t V[t][k] = Fresnel(J_k),   J_k = sum_t V[t][k] I_t,
// and the image of Eq. (7) is M = sum over kept k of |Y_k|^2: K transforms of
// combined frames instead of n_t transforms of single frames, and the
// holograms H are never formed.  Three kernels:
//   proj_rows   : per (row y, group of KP kept components): J_k of the row from
//                 the uint16 frames, x chirp, row FFT -> inter[k][y][:]
//   cols_energy : per (column strip, chunk of kept components): column FFT of
//                 each inter[k] strip, sum of |.|^2 -> the chunk's partial image
//   energy_sum  : fixed-order sum of the chunk partials -> image
// J_k is accumulated in FP32 around the pixel's frame-0 value,
//   J_k = I_0 s_k + sum_{t>=1} V[t][k] (I_t - I_0),   s_k = sum_t V[t][k] (FP64),
// where every I_t - I_0 is an exact small integer, so the large common part of
// the frames never enters a long FP32 sum.
#include <type_traits>

#include "fft_common.h"
#include "hh_internal.h"

namespace hh {
namespace {

constexpr int kPfThreads = 256;

// eight uint16 pixels (one 16-byte load) as floats, exact
__device__ __forceinline__ void u16x8(const uint4 q, float (&x)[8]) {
  const unsigned w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    x[2 * i] = (float)(w[i] & 0xffffu);
    x[2 * i + 1] = (float)(w[i] >> 16);
  }
}

struct PfRowSlot {
  __device__ __forceinline__ int operator()(int e) const { return fft_pad(e); }
};
template <int W>
struct PfColSlot {
  int c;
  __device__ __forceinline__ int operator()(int e) const { return fft_pad(e) * W + c; }
};

// Row pass shape for rows of N points: 16 points per thread, U transforms at a
// time in a 256-thread group, KP kept components per group (their rows fill
// about 64 KiB of LDS), processed in ceil(KP / U) rounds.
template <int N>
struct PfRows {
  static constexpr int E = FftCfg<N, 16>::E, T = FftCfg<N, 16>::T;
  static constexpr int U = kPfThreads / T;
  static constexpr int KP = (8192 / N) < 64 ? (8192 / N) : 64;
  static constexpr int ROUNDS = (KP + U - 1) / U;
  static constexpr int LROWS = ROUNDS * U;  // LDS rows (rows >= KP of the last round are idle)
  static constexpr int LDSN = FftCfg<N, 16>::LDSN;
  static constexpr int KPAD = (KP + 3) / 4 * 4;  // coefficient columns, zero beyond the group
  static_assert(kPfThreads % T == 0, "a row transform must fit the group");
};

// CPLX: complex eigenvectors (general V); otherwise only Re V is read (the
// frame covariance N_pix I^T I is real symmetric, so its eigenvectors are real).
template <int N, bool CPLX>
__global__ __launch_bounds__(kPfThreads) void proj_rows(const uint16_t *__restrict__ frames, int nt, int ny,
                                                        const double2 *__restrict__ V, int k_lo, int K, int groups,
                                                        const float2 *__restrict__ chirp_x,
                                                        const float2 *__restrict__ chirp_y,
                                                        const float2 *__restrict__ tw, float2 *__restrict__ inter) {
  using C = PfRows<N>;
  constexpr int E = C::E, T = C::T, KP = C::KP, KPAD = C::KPAD, LDSN = C::LDSN;
  typedef typename std::conditional<CPLX, float2, float>::type Coef;
  __shared__ __align__(16) float2 jb[C::LROWS * LDSN];
  __shared__ __align__(16) Coef coef[72 * KPAD];  // coef[t][kk] = V[t][k] (t < nt), zero for t >= nt
  __shared__ Coef ssum[KPAD];                     // s_k = sum_t V[t][k]

  // XCD-aware order: workgroups go round-robin to the 8 XCDs, so the groups of one
  // row are given to blocks b, b + 8, b + 16, ... (one XCD, one L2), which read
  // the row's frames once from memory and then from that L2
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int g = slot % groups, y = (slot / groups) * 8 + xcd;
  const int kb = g * KP;                              // first kept component of this group (0-based in the list)
  const int kn = (K - kb) < KP ? (K - kb) : KP;       // components in this group
  const int tid = threadIdx.x;

  for (int i = tid; i < 72 * KPAD; i += kPfThreads) {  // rows t >= nt are zero (batches of 8 reach t < 72)
    const int t = i / KPAD, kk = i % KPAD;
    const double2 v = (t < nt && kk < kn) ? V[(size_t)t * nt + k_lo + kb + kk] : make_double2(0.0, 0.0);
    if constexpr (CPLX) coef[i] = make_float2((float)v.x, (float)v.y);
    else coef[i] = (float)v.x;
  }
  if (tid < KPAD) {
    double sr = 0.0, si = 0.0;
    if (tid < kn)
      for (int t = 0; t < nt; ++t) {
        const double2 v = V[(size_t)t * nt + k_lo + kb + tid];
        sr += v.x;
        si += v.y;
      }
    if constexpr (CPLX) ssum[tid] = make_float2((float)sr, (float)si);
    else ssum[tid] = (float)sr;
  }
  __syncthreads();

  // J_k for 8 consecutive pixels and 4 components per item, x chirp, into LDS
  constexpr int NCH = N / 8;
  const float2 cy = chirp_y[y];
  const size_t fstride = (size_t)ny * N;
  const uint16_t *row0 = frames + (size_t)y * N;
  for (int item = tid; item < NCH * (KPAD / 4); item += kPfThreads) {
    const int c = item % NCH, q = item / NCH;
    const uint4 a0 = reinterpret_cast<const uint4 *>(row0)[c];
    float i0[8];
    u16x8(a0, i0);
    float jr[4][8], ji[4][8];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int e = 0; e < 8; ++e) jr[kk][e] = ji[kk][e] = 0.0f;
    // frames in batches of eight, the next batch's loads in flight while the
    // current one is summed; slots beyond nt reload the last frame and meet zero
    // coefficients
    auto load8 = [&](int t0, uint4 (&a)[8]) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int tt = (t0 + j < nt) ? t0 + j : nt - 1;
        a[j] = reinterpret_cast<const uint4 *>(row0 + (size_t)tt * fstride)[c];
      }
    };
    uint4 a[8], nx8[8];
    load8(1, a);
    for (int t0 = 1; t0 < nt; t0 += 8) {
      if (t0 + 8 < nt) load8(t0 + 8, nx8);
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        float d[8];
        u16x8(a[j], d);
#pragma unroll
        for (int e = 0; e < 8; ++e) d[e] -= i0[e];  // exact: integers below 2^17
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const Coef v = coef[(t0 + j) * KPAD + 4 * q + kk];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            if constexpr (CPLX) {
              jr[kk][e] = fmaf(v.x, d[e], jr[kk][e]);
              ji[kk][e] = fmaf(v.y, d[e], ji[kk][e]);
            } else {
              jr[kk][e] = fmaf(v, d[e], jr[kk][e]);
            }
          }
        }
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) a[j] = nx8[j];
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int r = 4 * q + kk;
      if (r < kn) {
        const Coef sv = ssum[r];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          float re, im;
          if constexpr (CPLX) {
            re = fmaf(sv.x, i0[e], jr[kk][e]);
            im = fmaf(sv.y, i0[e], ji[kk][e]);
          } else {
            re = fmaf(sv, i0[e], jr[kk][e]);
            im = 0.0f;
          }
          const int m = 8 * c + e;
          const float2 ch = cmul(chirp_x[m], cy);
          jb[r * LDSN + fft_pad(m)] = cmul(make_float2(re, im), ch);
        }
      }
    }
  }
  __syncthreads();

  // row FFTs, U at a time; rows beyond the group's components run on zeros and are not stored
  const int u = tid / T, t = tid % T;
#pragma unroll 1
  for (int round = 0; round < C::ROUNDS; ++round) {
    const int r = round * C::U + u;
    const bool live = r < kn;
    float2 v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = live ? jb[r * LDSN + fft_pad(t + T * i)] : make_float2(0.f, 0.f);
    if constexpr (FftCfg<N, 16>::P > 1) {
      // every staged value of row r is in registers before the exchanges reuse that row;
      // only this transform reads and writes row r, so when its T <= 64 threads lie in
      // one wave the wave's own ordering suffices
      constexpr bool kWave = T <= 64;
      fft_sync<kWave>();
      fft_passes<N, 16, 0, false, kWave>(v, t, tw, jb + r * LDSN, PfRowSlot{});
    } else {
      fft_passes<N, 16, 0, false>(v, t, tw, (float2 *)nullptr, PfRowSlot{});
    }
    if (live) {
      float2 *o = inter + ((size_t)(kb + r) * ny + y) * N;
#pragma unroll
      for (int i = 0; i < E; ++i) o[t + T * i] = v[i];
    }
  }
}

// Column pass over the K row-transformed components: strip of W columns, one
// chunk of components per group, |.|^2 summed in FP32 in registers.
template <int N, int EP, int W, bool SPLIT>
__global__ __launch_bounds__(W *(N / fft_e(N, EP))) void cols_energy(const float2 *__restrict__ inter, int nx,
                                                                     int K, int kper, const float2 *__restrict__ tw,
                                                                     float *__restrict__ out) {
  constexpr int E = FftCfg<N, EP>::E, T = FftCfg<N, EP>::T;
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  const int col = blockIdx.x * W + c;
  const bool live = col < nx;
  const int k0 = blockIdx.y * kper, k1 = (k0 + kper) < K ? (k0 + kper) : K;
  float acc[E];
#pragma unroll
  for (int i = 0; i < E; ++i) acc[i] = 0.0f;
  typedef typename std::conditional<SPLIT, float, float2>::type Slot;
  __shared__ Slot lds[(FftCfg<N, EP>::P > 1) ? W * FftCfg<N, EP>::LDSN : 1];
#pragma unroll 1
  for (int k = k0; k < k1; ++k) {
    const float2 *base = inter + (size_t)k * N * nx + (live ? col : 0);
    float2 v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = live ? base[(size_t)(t + T * i) * nx] : make_float2(0.f, 0.f);
    // the thread's position is made opaque per component, so that the compiler
    // recomputes the twiddle and LDS addresses (a few integer operations) instead
    // of holding all of them in registers across the loop
    int tk = t;
    asm volatile("" : "+v"(tk));
    if constexpr (FftCfg<N, EP>::P > 1) {
      fft_passes<N, EP, 0, SPLIT>(v, tk, tw, lds, PfColSlot<W>{c});
      __syncthreads();  // the last exchange's reads are done before the next component's writes
    } else {
      fft_passes<N, EP, 0, false>(v, tk, tw, (float2 *)nullptr, PfColSlot<W>{c});
    }
#pragma unroll
    for (int i = 0; i < E; ++i) acc[i] = fmaf(v[i].x, v[i].x, fmaf(v[i].y, v[i].y, acc[i]));
  }
  if (live) {
    float *o = out + (size_t)blockIdx.y * N * nx + col;
#pragma unroll
    for (int i = 0; i < E; ++i) o[(size_t)(t + T * i) * nx] = acc[i];
  }
}

// image[p] = sum over chunks c (in order) of part[c][p]; two pixels per thread
// (the image is 8-byte aligned)
__global__ __launch_bounds__(256) void energy_sum(const float *__restrict__ part, int chunks, long long npix,
                                                  float *__restrict__ image) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (2 * q >= npix) return;
  float2 s = reinterpret_cast<const float2 *>(part)[q];
  for (int c = 1; c < chunks; ++c) {
    const float2 a = reinterpret_cast<const float2 *>(part + (size_t)c * npix)[q];
    s.x += a.x;
    s.y += a.y;
  }
  reinterpret_cast<float2 *>(image)[q] = s;
}

// Column strip: 32 points per thread with the split exchange where the column is
// long enough (the column pass's fastest launch shape at 1024), else 16 points
// per thread; as wide as about 64 KiB of LDS allows (at most 16 columns).
template <int N>
constexpr int pf_col_ep() { return N >= 512 ? 32 : 16; }
template <int N>
constexpr int pf_col_w() {
  constexpr int T = FftCfg<N, pf_col_ep<N>()>::T;
  int w = 1024 / T;
  if (w > 16) w = 16;
  if (w < 1) w = 1;
  while (w > 1 && w * FftCfg<N, pf_col_ep<N>()>::LDSN * (N >= 512 ? 4 : 8) > 70000) w >>= 1;
  return w;
}

template <int N>
hipError_t rows_n(const Plan &pl, const uint16_t *frames, int nt, const double *V, int k_lo, int K, bool real_v,
                  float2 *inter, hipStream_t s) {
  const int groups = (K + PfRows<N>::KP - 1) / PfRows<N>::KP;
  const dim3 grid(groups * pl.ny), block(kPfThreads);
  const double2 *V2 = reinterpret_cast<const double2 *>(V);
  if (real_v)
    hipLaunchKernelGGL((proj_rows<N, false>), grid, block, 0, s, frames, nt, pl.ny, V2, k_lo, K, groups, pl.chirp_x,
                       pl.chirp_y, pl.tw_x, inter);
  else
    hipLaunchKernelGGL((proj_rows<N, true>), grid, block, 0, s, frames, nt, pl.ny, V2, k_lo, K, groups, pl.chirp_x,
                       pl.chirp_y, pl.tw_x, inter);
  return hipGetLastError();
}

template <int N>
hipError_t cols_n(const Plan &pl, const float2 *inter, int K, int chunks, int kper, float *out, hipStream_t s) {
  constexpr int EP = pf_col_ep<N>(), W = pf_col_w<N>();
  const dim3 grid((pl.nx + W - 1) / W, chunks), block(W * FftCfg<N, EP>::T);
  hipLaunchKernelGGL((cols_energy<N, EP, W, (N >= 512)>), grid, block, 0, s, inter, pl.nx, K, kper, pl.tw_y, out);
  return hipGetLastError();
}

}  // namespace

int project_frames_chunks(int nx, int ny, int K, int cus) {
  int w = 16;
  switch (ny) {  // strip width of the column pass for this column length
    case 8: w = pf_col_w<8>(); break;
    case 16: w = pf_col_w<16>(); break;
    case 32: w = pf_col_w<32>(); break;
    case 64: w = pf_col_w<64>(); break;
    case 128: w = pf_col_w<128>(); break;
    case 256: w = pf_col_w<256>(); break;
    case 512: w = pf_col_w<512>(); break;
    case 1024: w = pf_col_w<1024>(); break;
    case 2048: w = pf_col_w<2048>(); break;
    default: w = pf_col_w<4096>(); break;
  }
  const int strips = (nx + w - 1) / w;
  int chunks = (2 * cus + strips - 1) / strips;  // about two groups per compute unit
  if (chunks > kMaxEnergyChunks) chunks = kMaxEnergyChunks;
  if (chunks > K) chunks = K;
  if (chunks < 1) chunks = 1;
  const int kper = (K + chunks - 1) / chunks;
  return (K + kper - 1) / kper;
}

hipError_t launch_project_frames(const Plan &pl, const uint16_t *frames, int nt, const double *V, int k_lo, int k_hi,
                                 bool real_v, float2 *inter, float *eparts, float *image, hipStream_t s) {
  const int K = k_hi - k_lo + 1;
  const long long npix = (long long)pl.nx * pl.ny;
  hipError_t e;
  {
    ProfScope ps("proj_rows", s);
    switch (pl.nx) {
      case 8: e = rows_n<8>(pl, frames, nt, V, k_lo, K, real_v, inter, s); break;
      case 16: e = rows_n<16>(pl, frames, nt, V, k_lo, K, real_v, inter, s); break;
      case 32: e = rows_n<32>(pl, frames, nt, V, k_lo, K, real_v, inter, s); break;
      case 64: e = rows_n<64>(pl, frames, nt, V, k_lo, K, real_v, inter, s); break;
      case 128: e = rows_n<128>(pl, frames, nt, V, k_lo, K, real_v, inter, s); break;
      case 256: e = rows_n<256>(pl, frames, nt, V, k_lo, K, real_v, inter, s); break;
      case 512: e = rows_n<512>(pl, frames, nt, V, k_lo, K, real_v, inter, s); break;
      case 1024: e = rows_n<1024>(pl, frames, nt, V, k_lo, K, real_v, inter, s); break;
      case 2048: e = rows_n<2048>(pl, frames, nt, V, k_lo, K, real_v, inter, s); break;
      case 4096: e = rows_n<4096>(pl, frames, nt, V, k_lo, K, real_v, inter, s); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess) return e;
  const int chunks = project_frames_chunks(pl.nx, pl.ny, K, pl.cus);
  const int kper = (K + chunks - 1) / chunks;
  float *out = chunks == 1 ? image : eparts;
  {
    ProfScope ps("cols_energy", s);
    switch (pl.ny) {
      case 8: e = cols_n<8>(pl, inter, K, chunks, kper, out, s); break;
      case 16: e = cols_n<16>(pl, inter, K, chunks, kper, out, s); break;
      case 32: e = cols_n<32>(pl, inter, K, chunks, kper, out, s); break;
      case 64: e = cols_n<64>(pl, inter, K, chunks, kper, out, s); break;
      case 128: e = cols_n<128>(pl, inter, K, chunks, kper, out, s); break;
      case 256: e = cols_n<256>(pl, inter, K, chunks, kper, out, s); break;
      case 512: e = cols_n<512>(pl, inter, K, chunks, kper, out, s); break;
      case 1024: e = cols_n<1024>(pl, inter, K, chunks, kper, out, s); break;
      case 2048: e = cols_n<2048>(pl, inter, K, chunks, kper, out, s); break;
      case 4096: e = cols_n<4096>(pl, inter, K, chunks, kper, out, s); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess || chunks == 1) return e;
  ProfScope ps("energy_sum", s);
  const long long q = npix / 2;
  hipLaunchKernelGGL(energy_sum, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, eparts, chunks, npix, image);
  return hipGetLastError();
}

}  // namespace hh
