// Step (a), Eq. (1): Fresnel holograms = 2D FFT of (interferogram x input-plane chirp).
//
// Two kernels per frame group:
//   fresnel_rows : uint16 load -> FP32 -> chirp a[m] b[n] -> row FFT -> complex64 out
//   fresnel_cols : in-place column FFT on the row-transformed frames
// Each 1D transform is a mixed-radix Stockham FFT with 16 points per thread
// (1024 = 16 * 16 * 4: one wave per 1024-point row, 128-byte coalesced uint16
// loads), register DFTs, LDS exchanges between passes, and W_N twiddles from a
// table built in FP64 on the host.
#include "fft_common.h"
#include "hh_internal.h"

namespace hh {
namespace {

// Rows per workgroup (256 threads where possible).
template <int N>
constexpr int rows_per_wg() {
  constexpr int T = FftCfg<N>::T;
  return T >= 256 ? 1 : 256 / T;
}

// Columns per workgroup: a 128-byte strip (16 complex) where the LDS allows.
template <int N>
constexpr int cols_per_wg() {
  constexpr int T = FftCfg<N>::T;
  int w = 1024 / T;
  if (w > 16 && T > 1) w = 256 / T > 16 ? 256 / T : 16;
  if (T == 1) w = 256;
  while (w > 1 && w * FftCfg<N>::LDSN * 8 > 140000) w >>= 1;
  return w;
}

struct RowSlot {
  __device__ __forceinline__ int operator()(int e) const { return fft_pad(e); }
};
template <int W>
struct ColSlot {
  int c;
  __device__ __forceinline__ int operator()(int e) const { return fft_pad(e) * W + c; }
};

template <int N, int ROWS>
__global__ __launch_bounds__(ROWS *FftCfg<N>::T) void fresnel_rows(
    const uint16_t *__restrict__ frames, int ny, const float2 *__restrict__ chirp_x,
    const float2 *__restrict__ chirp_y, const float2 *__restrict__ tw, float2 *__restrict__ out) {
  constexpr int E = FftCfg<N>::E, T = FftCfg<N>::T;
  const int t = threadIdx.x % T;
  const int r = threadIdx.x / T;
  const int row = blockIdx.x * ROWS + r;
  const bool live = row < ny;
  const size_t base = ((size_t)blockIdx.y * ny + (live ? row : 0)) * N;

  float2 v[E];
  {
    const float2 cy = chirp_y[live ? row : 0];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int m = t + T * i;
      const float val = live ? (float)frames[base + m] : 0.0f;
      const float2 c = cmul(chirp_x[m], cy);
      v[i] = make_float2(val * c.x, val * c.y);
    }
  }
  if constexpr (FftCfg<N>::P > 1) {
    __shared__ float2 lds[ROWS * FftCfg<N>::LDSN];
    fft_passes<N, 16, 0>(v, t, tw, lds + r * FftCfg<N>::LDSN, RowSlot{});
  } else {
    fft_passes<N, 16, 0>(v, t, tw, (float2 *)nullptr, RowSlot{});
  }
  if (live) {
#pragma unroll
    for (int i = 0; i < E; ++i) out[base + t + T * i] = v[i];
  }
}

template <int N, int W>
__global__ __launch_bounds__(W *FftCfg<N>::T) void fresnel_cols(float2 *__restrict__ data, int nx,
                                                               const float2 *__restrict__ tw) {
  constexpr int E = FftCfg<N>::E, T = FftCfg<N>::T;
  const int c = threadIdx.x % W;
  const int t = threadIdx.x / W;
  const int col = blockIdx.x * W + c;
  const bool live = col < nx;
  float2 *base = data + (size_t)blockIdx.y * N * nx + (live ? col : 0);

  float2 v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = live ? base[(size_t)(t + T * i) * nx] : make_float2(0.f, 0.f);
  if constexpr (FftCfg<N>::P > 1) {
    __shared__ float2 lds[W * FftCfg<N>::LDSN];
    fft_passes<N, 16, 0>(v, t, tw, lds, ColSlot<W>{c});
  } else {
    fft_passes<N, 16, 0>(v, t, tw, (float2 *)nullptr, ColSlot<W>{c});
  }
  if (live) {
#pragma unroll
    for (int i = 0; i < E; ++i) base[(size_t)(t + T * i) * nx] = v[i];
  }
}

template <int N>
hipError_t rows_n(const Plan &pl, const uint16_t *frames, int nframes, float2 *out, hipStream_t s) {
  constexpr int R = rows_per_wg<N>();
  dim3 grid((pl.ny + R - 1) / R, nframes);
  ProfScope ps("fresnel_rows", s);
  hipLaunchKernelGGL((fresnel_rows<N, R>), grid, dim3(R * FftCfg<N>::T), 0, s, frames, pl.ny,
                     pl.chirp_x, pl.chirp_y, pl.tw_x, out);
  return hipGetLastError();
}

template <int N>
hipError_t cols_n(const Plan &pl, int nframes, float2 *data, hipStream_t s) {
  constexpr int W = cols_per_wg<N>();
  dim3 grid((pl.nx + W - 1) / W, nframes);
  ProfScope ps("fresnel_cols", s);
  hipLaunchKernelGGL((fresnel_cols<N, W>), grid, dim3(W * FftCfg<N>::T), 0, s, data, pl.nx, pl.tw_y);
  return hipGetLastError();
}

hipError_t rows_dispatch(const Plan &pl, const uint16_t *f, int n, float2 *o, hipStream_t s) {
  switch (pl.nx) {
    case 8: return rows_n<8>(pl, f, n, o, s);
    case 16: return rows_n<16>(pl, f, n, o, s);
    case 32: return rows_n<32>(pl, f, n, o, s);
    case 64: return rows_n<64>(pl, f, n, o, s);
    case 128: return rows_n<128>(pl, f, n, o, s);
    case 256: return rows_n<256>(pl, f, n, o, s);
    case 512: return rows_n<512>(pl, f, n, o, s);
    case 1024: return rows_n<1024>(pl, f, n, o, s);
    case 2048: return rows_n<2048>(pl, f, n, o, s);
    case 4096: return rows_n<4096>(pl, f, n, o, s);
  }
  return hipErrorInvalidValue;
}

hipError_t cols_dispatch(const Plan &pl, int n, float2 *d, hipStream_t s) {
  switch (pl.ny) {
    case 8: return cols_n<8>(pl, n, d, s);
    case 16: return cols_n<16>(pl, n, d, s);
    case 32: return cols_n<32>(pl, n, d, s);
    case 64: return cols_n<64>(pl, n, d, s);
    case 128: return cols_n<128>(pl, n, d, s);
    case 256: return cols_n<256>(pl, n, d, s);
    case 512: return cols_n<512>(pl, n, d, s);
    case 1024: return cols_n<1024>(pl, n, d, s);
    case 2048: return cols_n<2048>(pl, n, d, s);
    case 4096: return cols_n<4096>(pl, n, d, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

// Frames are processed in groups so that a group's row-transformed frames are
// still in the last-level cache when the column pass reads them back.
hipError_t launch_fresnel(const Plan &pl, const uint16_t *frames, int nframes, float2 *holo,
                          hipStream_t s) {
  const size_t frame_bytes = (size_t)pl.nx * pl.ny * sizeof(float2);
  int group = (int)((64u << 20) / frame_bytes);  // about 64 MiB of holograms per group
  if (group < 1) group = 1;
  for (int f0 = 0; f0 < nframes; f0 += group) {
    const int n = nframes - f0 < group ? nframes - f0 : group;
    const size_t off = (size_t)f0 * pl.nx * pl.ny;
    hipError_t e = rows_dispatch(pl, frames + off, n, holo + off, s);
    if (e != hipSuccess) return e;
    e = cols_dispatch(pl, n, holo + off, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace hh
