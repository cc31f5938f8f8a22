// Step (a), Eq. (1): Fresnel holograms = 2D FFT of (interferogram x input-plane chirp).
//
// Two kernels per frame group:
//   fresnel_rows : uint16 load -> FP32 -> chirp a[m] b[n] -> row FFT -> complex64 out
//   fresnel_cols : in-place column FFT on the row-transformed frames
// The FP16 storage form transforms the stack's temporal mean frame once (m) and
// then each frame minus that mean (R = H - m by linearity), and the column pass
// writes R scaled and rounded to FP16 instead of FP32.
// Each 1D transform is a mixed-radix Stockham FFT with 16 points per thread
// (1024 = 16 * 16 * 4: one wave per 1024-point row, 128-byte coalesced uint16
// loads), register DFTs, LDS exchanges between passes, and W_N twiddles from a
// table built in FP64 on the host.
#include <type_traits>

#include "fft_common.h"
#include "hh_internal.h"

namespace hh {
namespace {

// Rows per workgroup (256 threads where possible).
template <int N, int EP = 16>
constexpr int rows_per_wg() {
  constexpr int T = FftCfg<N, EP>::T;
  return T >= 256 ? 1 : 256 / T;
}

// Columns per workgroup: a 128-byte strip (16 complex) where the LDS allows.
template <int N, int EP = 16>
constexpr int cols_per_wg() {
  constexpr int T = FftCfg<N, EP>::T;
  int w = 1024 / T;
  if (w > 16 && T > 1) w = 256 / T > 16 ? 256 / T : 16;
  if (T == 1) w = 256;
  while (w > 1 && w * FftCfg<N, EP>::LDSN * 8 > 140000) w >>= 1;
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

// Eight floats into the LDS staging area: two 16-byte stores when the row's area
// starts 16-byte aligned (lanes 32 bytes apart then touch distinct bank groups),
// else eight 4-byte stores.
template <bool ALIGNED16>
__device__ __forceinline__ void stage8(float *dst, const float (&x)[8]) {
  if constexpr (ALIGNED16) {
    float4 *d4 = reinterpret_cast<float4 *>(dst);
    d4[0] = make_float4(x[0], x[1], x[2], x[3]);
    d4[1] = make_float4(x[4], x[5], x[6], x[7]);
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) dst[e] = x[e];
  }
}

// Input of the row pass: the uint16 frames, the frames minus a float frame
// (the stack's temporal mean), or one float frame.
enum { kInU16 = 0, kInU16MinusMean = 1, kInF32 = 2 };

template <int N, int EP, int ROWS, int IN, bool SPLIT>
__global__ __launch_bounds__(ROWS *(N / fft_e(N, EP))) void fresnel_rows(
    const void *__restrict__ src, const float *__restrict__ mean, int ny, const float2 *__restrict__ chirp_x,
    const float2 *__restrict__ chirp_y, const float2 *__restrict__ tw, float2 *__restrict__ out) {
  constexpr int E = FftCfg<N, EP>::E, T = FftCfg<N, EP>::T;
  // a row is held by T <= 64 lanes of one wave, in an LDS area of its own: the
  // exchanges need only the wave's own ordering (fft_sync)
  constexpr bool kWave = T <= 64;
  const int t = threadIdx.x % T;
  const int r = threadIdx.x / T;
  const int row = blockIdx.x * ROWS + r;
  const bool live = row < ny;
  const size_t base = ((size_t)blockIdx.y * ny + (live ? row : 0)) * N;
  const size_t mbase = (size_t)(live ? row : 0) * N;

  float2 v[E];
  const float2 cy = chirp_y[live ? row : 0];
  if constexpr (FftCfg<N, EP>::P > 1) {
    typedef typename std::conditional<SPLIT, float, float2>::type Slot;
    __shared__ __align__(16) Slot lds[ROWS * FftCfg<N, EP>::LDSN];
    // The row arrives through LDS: 16-byte coalesced loads of 8 pixels each are
    // written to the row's LDS area as floats, then every thread reads its
    // elements t + T i in FFT order (the FFT's first pass then reuses the area).
    float *stage = reinterpret_cast<float *>(lds + r * FftCfg<N, EP>::LDSN);
#pragma unroll
    for (int c = t; c < N / 8; c += T) {
      float x[8];
      if (live) {
        if constexpr (IN == kInF32) {
          const float4 *s4 = reinterpret_cast<const float4 *>(static_cast<const float *>(src) + base) + 2 * c;
          const float4 a = s4[0], b = s4[1];
          x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
          x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
        } else {
          union {
            uint4 q;
            uint16_t h[8];
          } u;
          u.q = reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(src) + base)[c];
#pragma unroll
          for (int e = 0; e < 8; ++e) x[e] = (float)u.h[e];
          if constexpr (IN == kInU16MinusMean) {
            const float4 *m4 = reinterpret_cast<const float4 *>(mean + mbase) + 2 * c;
            const float4 a = m4[0], b = m4[1];
            x[0] -= a.x; x[1] -= a.y; x[2] -= a.z; x[3] -= a.w;
            x[4] -= b.x; x[5] -= b.y; x[6] -= b.z; x[7] -= b.w;
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = 0.0f;
      }
      stage8<(FftCfg<N, EP>::LDSN * sizeof(Slot)) % 16 == 0>(stage + 8 * c, x);
    }
    fft_sync<kWave>();
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int m = t + T * i;
      const float val = stage[m];
      const float2 c = cmul(chirp_x[m], cy);
      v[i] = make_float2(val * c.x, val * c.y);
    }
    fft_sync<kWave>();
    fft_passes<N, EP, 0, SPLIT, kWave>(v, t, tw, lds + r * FftCfg<N, EP>::LDSN, RowSlot{});
  } else {
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const int m = t + T * i;
      float val = 0.0f;
      if (live) {
        if constexpr (IN == kInF32) {
          val = static_cast<const float *>(src)[base + m];
        } else {
          val = (float)static_cast<const uint16_t *>(src)[base + m];
          if constexpr (IN == kInU16MinusMean) val -= mean[mbase + m];
        }
      }
      const float2 c = cmul(chirp_x[m], cy);
      v[i] = make_float2(val * c.x, val * c.y);
    }
    fft_passes<N, EP, 0, false>(v, t, tw, (float2 *)nullptr, RowSlot{});
  }
  if (live) {
#pragma unroll
    for (int i = 0; i < E; ++i) out[base + t + T * i] = v[i];
  }
}

// R16: instead of writing the column FFT back in place, write it scaled by
// `scale` and rounded to FP16 (round to nearest even) into r16 [frames][N][nx].
// TWL: the twiddles are copied to LDS first (read there just before use, so that
// the compiler does not hold all of them in registers from the start).
template <int N, int EP, int W, bool R16, bool SPLIT, bool TWL = false>
__global__ __launch_bounds__(W *(N / fft_e(N, EP)), TWL ? 4 : 1) void fresnel_cols(float2 *__restrict__ data, int nx,
                                                               const float2 *__restrict__ tw, h2 *__restrict__ r16,
                                                               float scale) {
  constexpr int E = FftCfg<N, EP>::E, T = FftCfg<N, EP>::T;
  const int c = threadIdx.x % W;
  const int t = threadIdx.x / W;
  const int col = blockIdx.x * W + c;
  const bool live = col < nx;
  const size_t off = (size_t)blockIdx.y * N * nx + (live ? col : 0);
  float2 *base = data + off;

  float2 v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] = live ? base[(size_t)(t + T * i) * nx] : make_float2(0.f, 0.f);
  if constexpr (FftCfg<N, EP>::P > 1) {
    typedef typename std::conditional<SPLIT, float, float2>::type Slot;
    __shared__ Slot lds[W * FftCfg<N, EP>::LDSN];
    __shared__ float2 tws[TWL ? N : 1];
    if constexpr (TWL) {
      for (int i = threadIdx.x; i < N; i += W * T) tws[i] = tw[i];
      __syncthreads();
    }
    fft_passes<N, EP, 0, SPLIT>(v, t, TWL ? tws : tw, lds, ColSlot<W>{c});
  } else {
    fft_passes<N, EP, 0, false>(v, t, tw, (float2 *)nullptr, ColSlot<W>{c});
  }
  // with TWL the thread index is made opaque here, so that the store addresses are
  // formed after the transform instead of being kept in registers from the loads
  int tid = threadIdx.x;
  if constexpr (TWL) asm volatile("" : "+v"(tid));
  const int ts = tid / W, cs = blockIdx.x * W + tid % W;
  if (cs < nx) {
    const size_t offs = (size_t)blockIdx.y * N * nx + cs;
    float2 *bases = data + offs;
    if constexpr (R16) {
      h2 *ob = r16 + offs;
#pragma unroll
      for (int i = 0; i < E; ++i) {
        h2 q;
        q.x = (_Float16)(v[i].x * scale);
        q.y = (_Float16)(v[i].y * scale);
        ob[(size_t)(ts + T * i) * nx] = q;
      }
    } else {
#pragma unroll
      for (int i = 0; i < E; ++i) bases[(size_t)(ts + T * i) * nx] = v[i];
    }
  }
}

// Persistent forms of the two passes: a grid sized to what the compute units
// hold at once walks the work items (rows, or column strips of one frame) with a
// grid stride and loads the next item's data into registers while it transforms
// the current one, so memory latency overlaps the FFT.

// Raw input of one row chunk (8 pixels per 16-byte load) held in registers.
template <int IN>
struct RowIn {
  uint4 q;      // 8 uint16 (kInU16, kInU16MinusMean)
  float4 a, b;  // 8 floats (kInF32) or the mean (kInU16MinusMean)
};

template <int N, int EP, int IN>
__device__ __forceinline__ void row_load(RowIn<IN> (&in)[N / 8 / (N / fft_e(N, EP)) > 0 ? N / 8 / (N / fft_e(N, EP)) : 1],
                                         const void *src, const float *mean, size_t base, size_t mbase, int t,
                                         bool live) {
  constexpr int T = N / fft_e(N, EP), L = N / 8 / T > 0 ? N / 8 / T : 1;
#pragma unroll
  for (int l = 0; l < L; ++l) {
    const int c = t + T * l;
    (void)live;  // rows past the end load row 0 of frame 0 (a valid address) and are zeroed when staged
    if (c >= N / 8) continue;
    if constexpr (IN == kInF32) {
      const float4 *s4 = reinterpret_cast<const float4 *>(static_cast<const float *>(src) + base) + 2 * c;
      in[l].a = s4[0];
      in[l].b = s4[1];
    } else {
      in[l].q = reinterpret_cast<const uint4 *>(static_cast<const uint16_t *>(src) + base)[c];
      if constexpr (IN == kInU16MinusMean) {
        const float4 *m4 = reinterpret_cast<const float4 *>(mean + mbase) + 2 * c;
        in[l].a = m4[0];
        in[l].b = m4[1];
      }
    }
  }
}

template <int N, int EP, int ROWS, int IN, bool SPLIT>
__global__ __launch_bounds__(ROWS *(N / fft_e(N, EP))) void fresnel_rows_persist(
    const void *__restrict__ src, const float *__restrict__ mean, int ny, int nframes,
    const float2 *__restrict__ chirp_x, const float2 *__restrict__ chirp_y, const float2 *__restrict__ tw,
    float2 *__restrict__ out) {
  constexpr int E = FftCfg<N, EP>::E, T = FftCfg<N, EP>::T, L = N / 8 / T > 0 ? N / 8 / T : 1;
  // a row is held by T <= 64 lanes of one wave, in an LDS area of its own: after the
  // shared tables are loaded, the exchanges need only the wave's own ordering
  constexpr bool kWave = T <= 64;
  static_assert(FftCfg<N, EP>::P > 1 && N / 8 >= T, "persistent rows need an LDS exchange and 8 pixels per thread");
  typedef typename std::conditional<SPLIT, float, float2>::type Slot;
  __shared__ __align__(16) Slot lds[ROWS * FftCfg<N, EP>::LDSN];
  const int t = threadIdx.x % T, r = threadIdx.x / T;
  float *stage = reinterpret_cast<float *>(lds + r * FftCfg<N, EP>::LDSN);
  const int groups = (ny + ROWS - 1) / ROWS, items = groups * nframes;
  // The twiddles come from LDS (up to 2048 points): a global twiddle load issued
  // after the next item's prefetch would make the transform wait for that prefetch.
  // The row chirp, the same for every row, sits in LDS beside them.
  constexpr bool kTwLds = N <= 2048;
  __shared__ float2 tws[kTwLds ? N : 1], cxs[kTwLds ? N : 1];
  if constexpr (kTwLds) {
    for (int i = threadIdx.x; i < N; i += ROWS * T) {
      tws[i] = tw[i];
      cxs[i] = chirp_x[i];
    }
    __syncthreads();
  }
  const float2 *twp = kTwLds ? tws : tw;
  const float2 *cxp = kTwLds ? cxs : chirp_x;
  auto where = [&](int item, int &row, size_t &base, size_t &mbase) {
    const int f = item / groups;
    row = (item - f * groups) * ROWS + r;
    const bool live = row < ny;
    base = ((size_t)f * ny + (live ? row : 0)) * N;
    mbase = (size_t)(live ? row : 0) * N;
    return live;
  };
  // The loads are unconditional (an item past the end loads row 0 of frame 0, a
  // valid address): with no branch around the prefetch, the transform of the current
  // item does not wait for the next item's loads.
  RowIn<IN> cur[L], nxt[L];
  int item = blockIdx.x, row = 0;
  size_t base = 0, mbase = 0;
  bool live = item < items && where(item, row, base, mbase);
  row_load<N, EP, IN>(cur, src, mean, base, mbase, t, live);
  for (; item < items; item += gridDim.x) {
    const int item2 = item + gridDim.x;
    int row2 = 0;
    size_t base2 = 0, mbase2 = 0;
    const bool live2 = item2 < items && where(item2, row2, base2, mbase2);
    // The thread index is made opaque for each item, so that nothing derived from it
    // (the row chirp, LDS and twiddle addresses) is hoisted out of the loop and held
    // in registers across it; the column chirp is loaded before the prefetch.
    int tk = t;
    asm volatile("" : "+v"(tk));
    const float2 cy = chirp_y[live ? row : 0];
    float2 cx[E];
    if constexpr (!kTwLds) {
#pragma unroll
      for (int i = 0; i < E; ++i) cx[i] = chirp_x[tk + T * i];
    }
    row_load<N, EP, IN>(nxt, src, mean, base2, mbase2, t, live2);
#pragma unroll
    for (int l = 0; l < L; ++l) {
      const int c = t + T * l;
      float x[8];
      if constexpr (IN == kInF32) {
        x[0] = cur[l].a.x; x[1] = cur[l].a.y; x[2] = cur[l].a.z; x[3] = cur[l].a.w;
        x[4] = cur[l].b.x; x[5] = cur[l].b.y; x[6] = cur[l].b.z; x[7] = cur[l].b.w;
      } else {
        union {
          uint4 q;
          uint16_t h[8];
        } u;
        u.q = cur[l].q;
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = (float)u.h[e];
        if constexpr (IN == kInU16MinusMean) {
          x[0] -= cur[l].a.x; x[1] -= cur[l].a.y; x[2] -= cur[l].a.z; x[3] -= cur[l].a.w;
          x[4] -= cur[l].b.x; x[5] -= cur[l].b.y; x[6] -= cur[l].b.z; x[7] -= cur[l].b.w;
        }
      }
      if (!live) {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = 0.0f;
      }
      stage8<(FftCfg<N, EP>::LDSN * sizeof(Slot)) % 16 == 0>(stage + 8 * c, x);
    }
    fft_sync<kWave>();
    float2 v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) {
      const float val = stage[tk + T * i];
      const float2 c = cmul(kTwLds ? cxp[tk + T * i] : cx[i], cy);
      v[i] = make_float2(val * c.x, val * c.y);
    }
    fft_sync<kWave>();
    fft_passes<N, EP, 0, SPLIT, kWave>(v, tk, twp, lds + r * FftCfg<N, EP>::LDSN, RowSlot{});
    if (live) {
#pragma unroll
      for (int i = 0; i < E; ++i) out[base + tk + T * i] = v[i];
    }
    fft_sync<kWave>();  // the LDS is reused by the next item
#pragma unroll
    for (int l = 0; l < L; ++l) cur[l] = nxt[l];
    live = live2;
    row = row2;
    base = base2;
  }
}

template <int N, int EP, int W, bool R16, bool SPLIT>
__global__ __launch_bounds__(W *(N / fft_e(N, EP))) void fresnel_cols_persist(float2 *__restrict__ data, int nx,
                                                                       int nframes, const float2 *__restrict__ tw,
                                                                       h2 *__restrict__ r16, float scale) {
  constexpr int E = FftCfg<N, EP>::E, T = FftCfg<N, EP>::T;
  static_assert(FftCfg<N, EP>::P > 1, "persistent columns need an LDS exchange");
  typedef typename std::conditional<SPLIT, float, float2>::type Slot;
  __shared__ Slot lds[W * FftCfg<N, EP>::LDSN];
  // twiddles from LDS (up to 2048 points), so that no global load issued after the
  // next strip's prefetch makes the transform wait for it
  constexpr bool kTwLds = N <= 2048;
  __shared__ float2 tws[kTwLds ? N : 1];
  if constexpr (kTwLds) {
    for (int i = threadIdx.x; i < N; i += W * T) tws[i] = tw[i];
    __syncthreads();
  }
  const float2 *twp = kTwLds ? tws : tw;
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  const int strips = (nx + W - 1) / W, items = strips * nframes;
  auto where = [&](int item, size_t &off) {
    const int f = item / strips;
    const int col = (item - f * strips) * W + c;
    const bool live = col < nx;
    off = (size_t)f * N * nx + (live ? col : 0);
    return live;
  };
  // Loads are unconditional (a dead column loads column 0 of its frame; past the
  // last item the prefetch repeats the current strip), so no branch separates the
  // prefetch from the transform.
  float2 cur[E], nxt[E];
  int item = blockIdx.x;
  size_t off = 0;
  bool live = item < items && where(item, off);
#pragma unroll
  for (int i = 0; i < E; ++i) cur[i] = data[off + (size_t)(t + T * i) * nx];
  for (; item < items; item += gridDim.x) {
    const int item2 = item + gridDim.x;
    size_t off2 = off;
    const bool live2 = item2 < items && where(item2, off2);
#pragma unroll
    for (int i = 0; i < E; ++i) nxt[i] = data[off2 + (size_t)(t + T * i) * nx];
    // the thread's position is made opaque per strip, so that the compiler
    // recomputes the twiddle and LDS addresses instead of holding them in registers
    int tk = t;
    asm volatile("" : "+v"(tk));
    fft_passes<N, EP, 0, SPLIT>(cur, tk, twp, lds, ColSlot<W>{c});
    if (live) {
      if constexpr (R16) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          h2 q;
          q.x = (_Float16)(cur[i].x * scale);
          q.y = (_Float16)(cur[i].y * scale);
          r16[off + (size_t)(t + T * i) * nx] = q;
        }
      } else {
#pragma unroll
        for (int i = 0; i < E; ++i) data[off + (size_t)(t + T * i) * nx] = cur[i];
      }
    }
    __syncthreads();  // the LDS is reused by the next item
#pragma unroll
    for (int i = 0; i < E; ++i) cur[i] = nxt[i];
    live = live2;
    off = off2;
  }
}

// mean[p] = (1 / nt) sum_t frames[t][p]: four pixels per thread
__global__ __launch_bounds__(256) void frame_mean(const uint16_t *__restrict__ frames, int nt, long long npix,
                                                  float *__restrict__ mean) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (4 * q >= npix) return;
  const ushort4 *f4 = reinterpret_cast<const ushort4 *>(frames);
  const long long nq = npix / 4;
  unsigned s0 = 0, s1 = 0, s2 = 0, s3 = 0;  // exact: nt * 65535 < 2^32
  for (int t = 0; t < nt; ++t) {
    const ushort4 a = f4[(long long)t * nq + q];
    s0 += a.x;
    s1 += a.y;
    s2 += a.z;
    s3 += a.w;
  }
  const float inv = 1.0f / (float)nt;
  reinterpret_cast<float4 *>(mean)[q] = make_float4((float)s0 * inv, (float)s1 * inv, (float)s2 * inv, (float)s3 * inv);
}

// Launch shapes the autotuner chooses between (index = FftShape::rows / ::cols);
// sizes below kTunedMinN have only shape 0.
constexpr int kTunedMinN = 512;

template <int N, int EP, int R, bool SPLIT = false>
hipError_t rows_launch(const Plan &pl, int in_mode, const void *src, const float *mean, int nframes, float2 *out,
                       hipStream_t s) {
  dim3 grid((pl.ny + R - 1) / R, nframes), block(R * FftCfg<N, EP>::T);
  if (in_mode == kInU16)
    hipLaunchKernelGGL((fresnel_rows<N, EP, R, kInU16, SPLIT>), grid, block, 0, s, src, mean, pl.ny, pl.chirp_x,
                       pl.chirp_y, pl.tw_x, out);
  else if (in_mode == kInU16MinusMean)
    hipLaunchKernelGGL((fresnel_rows<N, EP, R, kInU16MinusMean, SPLIT>), grid, block, 0, s, src, mean, pl.ny, pl.chirp_x,
                       pl.chirp_y, pl.tw_x, out);
  else
    hipLaunchKernelGGL((fresnel_rows<N, EP, R, kInF32, SPLIT>), grid, block, 0, s, src, mean, pl.ny, pl.chirp_x,
                       pl.chirp_y, pl.tw_x, out);
  return hipGetLastError();
}

template <int N, int EP, int R, bool SPLIT = false>
hipError_t rows_persist_launch(const Plan &pl, int in_mode, const void *src, const float *mean, int nframes,
                               float2 *out, hipStream_t s) {
  const int items = (pl.ny + R - 1) / R * nframes;
  // as many groups as the compute units hold at once (LDS, registers)
  static int per_cu = 0;
  if (per_cu == 0) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fresnel_rows_persist<N, EP, R, kInU16, SPLIT>,
                                                     R * FftCfg<N, EP>::T, 0) != hipSuccess || occ < 1)
      occ = 1;
    per_cu = occ;
  }
  const int resident = per_cu * pl.cus;
  const int grid = items < resident ? items : resident;
  dim3 g(grid), block(R * FftCfg<N, EP>::T);
  if (in_mode == kInU16)
    hipLaunchKernelGGL((fresnel_rows_persist<N, EP, R, kInU16, SPLIT>), g, block, 0, s, src, mean, pl.ny, nframes,
                       pl.chirp_x, pl.chirp_y, pl.tw_x, out);
  else if (in_mode == kInU16MinusMean)
    hipLaunchKernelGGL((fresnel_rows_persist<N, EP, R, kInU16MinusMean, SPLIT>), g, block, 0, s, src, mean, pl.ny,
                       nframes, pl.chirp_x, pl.chirp_y, pl.tw_x, out);
  else
    hipLaunchKernelGGL((fresnel_rows_persist<N, EP, R, kInF32, SPLIT>), g, block, 0, s, src, mean, pl.ny, nframes,
                       pl.chirp_x, pl.chirp_y, pl.tw_x, out);
  return hipGetLastError();
}

template <int N>
hipError_t rows_n(const Plan &pl, int shape, int in_mode, const void *src, const float *mean, int nframes,
                  float2 *out, hipStream_t s) {
  ProfScope ps("fresnel_rows", s);
  if constexpr (N >= kTunedMinN) {
    if (shape == 6) return rows_persist_launch<N, 16, 1>(pl, in_mode, src, mean, nframes, out, s);
    if (shape == 7) return rows_persist_launch<N, 32, 2>(pl, in_mode, src, mean, nframes, out, s);
    if (shape == 8) return rows_persist_launch<N, 16, 4, true>(pl, in_mode, src, mean, nframes, out, s);
    if (shape == 9) return rows_persist_launch<N, 16, 2>(pl, in_mode, src, mean, nframes, out, s);
    if (shape == 1) return rows_launch<N, 32, rows_per_wg<N, 32>()>(pl, in_mode, src, mean, nframes, out, s);
    if (shape == 2) return rows_launch<N, 32, 2>(pl, in_mode, src, mean, nframes, out, s);
    if (shape == 3) return rows_launch<N, 16, 1>(pl, in_mode, src, mean, nframes, out, s);
    if (shape == 4) return rows_launch<N, 32, 2, true>(pl, in_mode, src, mean, nframes, out, s);
    if (shape == 5) return rows_launch<N, 16, rows_per_wg<N, 16>(), true>(pl, in_mode, src, mean, nframes, out, s);
  }
  return rows_launch<N, 16, rows_per_wg<N, 16>()>(pl, in_mode, src, mean, nframes, out, s);
}

template <int N, int EP, int W, bool SPLIT = false, bool TWL = false>
hipError_t cols_launch(const Plan &pl, int nframes, float2 *data, h2 *r16, float scale, hipStream_t s) {
  dim3 grid((pl.nx + W - 1) / W, nframes), block(W * FftCfg<N, EP>::T);
  if (r16)
    hipLaunchKernelGGL((fresnel_cols<N, EP, W, true, SPLIT, TWL>), grid, block, 0, s, data, pl.nx, pl.tw_y, r16,
                       scale);
  else
    hipLaunchKernelGGL((fresnel_cols<N, EP, W, false, SPLIT, TWL>), grid, block, 0, s, data, pl.nx, pl.tw_y, r16,
                       scale);
  return hipGetLastError();
}

template <int N, int EP, int W, bool SPLIT = false>
hipError_t cols_persist_launch(const Plan &pl, int nframes, float2 *data, h2 *r16, float scale, hipStream_t s) {
  const int items = (pl.nx + W - 1) / W * nframes;
  // as many groups as the compute units hold at once (LDS, registers)
  static int per_cu = 0;
  if (per_cu == 0) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fresnel_cols_persist<N, EP, W, false, SPLIT>,
                                                     W * FftCfg<N, EP>::T, 0) != hipSuccess || occ < 1)
      occ = 1;
    per_cu = occ;
  }
  const int resident = per_cu * pl.cus;
  const int grid = items < resident ? items : resident;
  dim3 g(grid), block(W * FftCfg<N, EP>::T);
  if (r16)
    hipLaunchKernelGGL((fresnel_cols_persist<N, EP, W, true, SPLIT>), g, block, 0, s, data, pl.nx, nframes, pl.tw_y,
                       r16, scale);
  else
    hipLaunchKernelGGL((fresnel_cols_persist<N, EP, W, false, SPLIT>), g, block, 0, s, data, pl.nx, nframes, pl.tw_y,
                       r16, scale);
  return hipGetLastError();
}

template <int N>
hipError_t cols_n(const Plan &pl, int shape, int nframes, float2 *data, h2 *r16, float scale, hipStream_t s) {
  ProfScope ps(r16 ? "fresnel_cols_r16" : "fresnel_cols", s);
  if constexpr (N >= kTunedMinN) {
    if (shape == 5) return cols_persist_launch<N, 16, cols_per_wg<N, 16>()>(pl, nframes, data, r16, scale, s);
    if (shape == 6) return cols_persist_launch<N, 16, cols_per_wg<N, 16>(), true>(pl, nframes, data, r16, scale, s);
    if (shape == 7)
      return cols_launch<N, 32, cols_per_wg<N, 32>(), true, (N <= 2048)>(pl, nframes, data, r16, scale, s);
    constexpr int Wh = cols_per_wg<N, 16>() / 2 > 0 ? cols_per_wg<N, 16>() / 2 : 1;
    if (shape == 1) return cols_launch<N, 16, Wh>(pl, nframes, data, r16, scale, s);
    if (shape == 2) return cols_launch<N, 32, cols_per_wg<N, 32>()>(pl, nframes, data, r16, scale, s);
    if (shape == 3) return cols_launch<N, 16, cols_per_wg<N, 16>(), true>(pl, nframes, data, r16, scale, s);
    if (shape == 4) return cols_launch<N, 32, cols_per_wg<N, 32>(), true>(pl, nframes, data, r16, scale, s);
  }
  return cols_launch<N, 16, cols_per_wg<N, 16>()>(pl, nframes, data, r16, scale, s);
}

hipError_t rows_dispatch(const Plan &pl, int sh, int in_mode, const void *f, const float *mean, int n, float2 *o,
                         hipStream_t s) {
  switch (pl.nx) {
    case 8: return rows_n<8>(pl, sh, in_mode, f, mean, n, o, s);
    case 16: return rows_n<16>(pl, sh, in_mode, f, mean, n, o, s);
    case 32: return rows_n<32>(pl, sh, in_mode, f, mean, n, o, s);
    case 64: return rows_n<64>(pl, sh, in_mode, f, mean, n, o, s);
    case 128: return rows_n<128>(pl, sh, in_mode, f, mean, n, o, s);
    case 256: return rows_n<256>(pl, sh, in_mode, f, mean, n, o, s);
    case 512: return rows_n<512>(pl, sh, in_mode, f, mean, n, o, s);
    case 1024: return rows_n<1024>(pl, sh, in_mode, f, mean, n, o, s);
    case 2048: return rows_n<2048>(pl, sh, in_mode, f, mean, n, o, s);
    case 4096: return rows_n<4096>(pl, sh, in_mode, f, mean, n, o, s);
  }
  return hipErrorInvalidValue;
}

hipError_t cols_dispatch(const Plan &pl, int sh, int n, float2 *d, h2 *r16, float scale, hipStream_t s) {
  switch (pl.ny) {
    case 8: return cols_n<8>(pl, sh, n, d, r16, scale, s);
    case 16: return cols_n<16>(pl, sh, n, d, r16, scale, s);
    case 32: return cols_n<32>(pl, sh, n, d, r16, scale, s);
    case 64: return cols_n<64>(pl, sh, n, d, r16, scale, s);
    case 128: return cols_n<128>(pl, sh, n, d, r16, scale, s);
    case 256: return cols_n<256>(pl, sh, n, d, r16, scale, s);
    case 512: return cols_n<512>(pl, sh, n, d, r16, scale, s);
    case 1024: return cols_n<1024>(pl, sh, n, d, r16, scale, s);
    case 2048: return cols_n<2048>(pl, sh, n, d, r16, scale, s);
    case 4096: return cols_n<4096>(pl, sh, n, d, r16, scale, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

// Frames are processed in groups so that a group's row-transformed frames are
// still in the last-level cache when the column pass reads them back: about
// 64 MiB of FP32 holograms by default, or the tuned count.
int fresnel_group_frames(int nx, int ny, int nframes, int tuned) {
  int g = tuned;
  if (g <= 0) g = (int)((64u << 20) / ((size_t)nx * ny * sizeof(float2)));
  if (g < 1) g = 1;
  return g < nframes ? g : nframes;
}

hipError_t launch_fresnel(const Plan &pl, const Tune &tu, const uint16_t *frames, int nframes, float2 *holo,
                          hipStream_t s) {
  const int group = fresnel_group_frames(pl.nx, pl.ny, nframes, tu.group);
  for (int f0 = 0; f0 < nframes; f0 += group) {
    const int n = nframes - f0 < group ? nframes - f0 : group;
    const size_t off = (size_t)f0 * pl.nx * pl.ny;
    hipError_t e = rows_dispatch(pl, tu.rows, kInU16, frames + off, nullptr, n, holo + off, s);
    if (e != hipSuccess) return e;
    e = cols_dispatch(pl, tu.cols, n, holo + off, nullptr, 0.f, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fresnel_r16(const Plan &pl, const Tune &tu, const uint16_t *frames, int nframes, float *mean,
                              float2 *m, float2 *group_buf, h2 *r16, float scale, hipStream_t s) {
  const long long npix = (long long)pl.nx * pl.ny;
  {
    ProfScope ps("frame_mean", s);
    hipLaunchKernelGGL(frame_mean, dim3((unsigned)((npix / 4 + 255) / 256)), dim3(256), 0, s, frames, nframes, npix,
                       mean);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = rows_dispatch(pl, tu.rows, kInF32, mean, nullptr, 1, m, s);
  if (e == hipSuccess) e = cols_dispatch(pl, tu.cols, 1, m, nullptr, 0.f, s);
  // the group buffer holds the default group: larger tuned groups are clamped to it
  const int dflt = fresnel_group_frames(pl.nx, pl.ny, nframes, 0);
  const int group = fresnel_group_frames(pl.nx, pl.ny, nframes, tu.group < dflt ? tu.group : dflt);
  for (int f0 = 0; f0 < nframes && e == hipSuccess; f0 += group) {
    const int n = nframes - f0 < group ? nframes - f0 : group;
    const size_t off = (size_t)f0 * npix;
    e = rows_dispatch(pl, tu.rows, kInU16MinusMean, frames + off, mean, n, group_buf, s);
    if (e == hipSuccess) e = cols_dispatch(pl, tu.cols, n, group_buf, r16 + off, scale, s);
  }
  return e;
}

}  // namespace hh
