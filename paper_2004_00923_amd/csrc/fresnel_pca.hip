// Steps (a)-(e) of one stack in the FP32 form as three passes over one
// hologram-sized buffer: Eq. (1) is split so that the covariance of Eq. (4) and
// the image of Eqs. (6)-(7) are both formed from transforms that finish in LDS,
// and the holograms H themselves are never written to memory.
//
// Eq. (1) with the separable chirp c[y][x] = a[x] b[y] is the 2D DFT of z = c I.
// With Q = nx / 4, x = x' + Q g and u = 4 u' + q (x', u' < Q; g, q < 4), one
// radix-4 decimation-in-frequency step of the x transform gives
//   H[v][4u'+q] = sum_{x'} W_Q^{x'u'} Bhat_q[v][x'],
//   B_q[y][x']  = b[y] sum_g A_q[x'][g] I[y][x'+Qg],  A_q[x'][g] = W_nx^{x'q} (-i)^{gq} a[x'+Qg],
// with Bhat_q the full y transform of B_q.  So:
//   pass 1, qcols   : uint16 frames -> B_q -> y transform -> T[t][v][q][x'] (complex64)
//   pass 2, qgram   : for each (v, q) the Q-point transforms of the quarter row of
//                     every frame, then the covariance partials on FP32 MFMA from LDS
//                     (same split as the split-K Gram: H = m 1^T + R, m = frame 0)
//   pass 3, qproject: after the eigensolver, the same transforms (same code, so the
//                     same H), the projection onto the eigenvectors and |.|^2.
// HBM traffic per stack: the frames once, T written once and read twice, the image
// once -- the algorithmic bytes of the path, with T in place of H.
#include <type_traits>

#include "fft_common.h"
#include "hh_internal.h"

namespace hh {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

// LDS slot of element e of column transform c of W (split exchange)
template <int W>
struct ColSlotW {
  int c;
  __device__ __forceinline__ int operator()(int e) const { return fft_pad(e) * W + c; }
};

// Rank of this group in a persistent grid of G groups: the first G / 8 ranks go to
// XCD 0, the next to XCD 1, and so on (groups are dealt to the XCDs in turn), when G
// is a multiple of 8, so that consecutive work items run on one XCD.
__device__ __forceinline__ int xcd_rank(int G) {
  return (G & 7) == 0 ? (int)((blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3)) : (int)blockIdx.x;
}

// ---------------------------------------------------------------- pass 1 ----
// One group: W = 16 consecutive x' of one q of one frame (16 column transforms of
// length NY, 16 points per thread, NY threads), so that every output row is one
// full 128-byte line (measured: half-line rows written by two groups cost about
// as much as the whole transform).  The input is NY rows x 4 groups g x 16 uint16
// (32 bytes per row and g), read with 16-byte loads (8 chunks per thread, all
// issued at the start), staged in LDS half the rows at a time (chunk c at byte
// c * 16 of the half tile, row-major [y][g][16]) and combined from there; the
// transforms then exchange through the same area.  Sixteen consecutive groups (4
// strips x 4 q) read the same 128-byte input lines; groups are dealt to the XCDs
// in turn and the rank below puts consecutive ranks on one XCD.
template <int NY, int Q>
struct P1Cfg {
  static constexpr int EP = 16, E = FftCfg<NY, EP>::E, T = FftCfg<NY, EP>::T, W = 16, NTH = W * T, S = Q / 16;
  static constexpr int HALFB = NY * 64;                      // bytes of half the input tile
  static constexpr int XCHB = W * FftCfg<NY, EP>::LDSN * 4;  // bytes of the split exchange
  static constexpr int AREA = HALFB > XCHB ? HALFB : XCHB;
  static constexpr int CH = NY * 8 / NTH;                    // 16-byte chunks per thread
  static_assert(NTH == NY && E == 16 && S % 4 == 0 && CH == 8 && T * 8 == NY / 2, "pass 1 shape");
};

template <int NY, int Q>
__global__ __launch_bounds__(NY) void qcols_u16(const uint16_t *__restrict__ frames,
                                                 const float2 *__restrict__ chirp_x,
                                                 const float2 *__restrict__ chirp_y,
                                                 const float2 *__restrict__ tw_x,
                                                 const float2 *__restrict__ tw_y, float2 *__restrict__ out) {
  using C = P1Cfg<NY, Q>;
  constexpr int NX = 4 * Q, E = C::E, T = C::T, W = C::W, S = C::S;
  __shared__ __align__(16) unsigned char area[C::AREA];
  __shared__ float2 tws[NY];
  const int b = xcd_rank(gridDim.x);
  const int f = b / (4 * S), r = b - f * (4 * S);
  const int q = (r >> 2) & 3, s = (r >> 4) * 4 + (r & 3);
  // chunk k of thread x: chunk c = x + NTH k, row y = c / 8, group g = (c / 2) % 4,
  // half h = c % 2; chunks 0..3 hold the first half of the rows, 4..7 the second.
  // (Named registers: an array of the chunks is placed in scratch memory.)
  uint4 r0_, r1_, r2_, r3_, r4_, r5_, r6_, r7_;
  {
    constexpr size_t KS = (size_t)(C::NTH / 8) * NX;
    const uint16_t *bp = frames + (size_t)f * NY * NX + 16 * s + (size_t)(threadIdx.x >> 3) * NX +
                         Q * ((threadIdx.x >> 1) & 3) + 8 * (threadIdx.x & 1);
    r0_ = *reinterpret_cast<const uint4 *>(bp);
    r1_ = *reinterpret_cast<const uint4 *>(bp + KS);
    r2_ = *reinterpret_cast<const uint4 *>(bp + 2 * KS);
    r3_ = *reinterpret_cast<const uint4 *>(bp + 3 * KS);
    r4_ = *reinterpret_cast<const uint4 *>(bp + 4 * KS);
    r5_ = *reinterpret_cast<const uint4 *>(bp + 5 * KS);
    r6_ = *reinterpret_cast<const uint4 *>(bp + 6 * KS);
    r7_ = *reinterpret_cast<const uint4 *>(bp + 7 * KS);
  }
  for (int i = threadIdx.x; i < NY; i += C::NTH) tws[i] = tw_y[i];
  const int j = threadIdx.x % W, t = threadIdx.x / W;
  const int xp = 16 * s + j;
  float2 A[4];  // A_q[x'][g], g = 0..3
  {
    const float2 wq = tw_x[xp * q];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const float2 c = cmul(wq, chirp_x[xp + Q * g]);
      const int rot = (g * q) & 3;  // (-i)^{gq}
      A[g] = rot == 0 ? c : rot == 1 ? make_float2(c.y, -c.x) : rot == 2 ? make_float2(-c.x, -c.y)
                                                                        : make_float2(-c.y, c.x);
    }
  }
  float2 v[E];
  const uint16_t *tile = reinterpret_cast<const uint16_t *>(area);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    {
      uint4 *dst = reinterpret_cast<uint4 *>(area) + threadIdx.x;
      dst[0] = h ? r4_ : r0_;
      dst[C::NTH] = h ? r5_ : r1_;
      dst[2 * C::NTH] = h ? r6_ : r2_;
      dst[3 * C::NTH] = h ? r7_ : r3_;
    }
    __syncthreads();
    // points i = 8h .. 8h+7 have rows y = t + T i in this half (T * 8 = NY / 2)
#pragma unroll
    for (int i = 0; i < E / 2; ++i) {
      const int yl = t + T * i, y = yl + h * (NY / 2);
      const uint16_t *rw = tile + yl * 64 + j;
      const float i0 = rw[0], i1 = rw[16], i2 = rw[32], i3 = rw[48];
      const float re = A[0].x * i0 + A[1].x * i1 + A[2].x * i2 + A[3].x * i3;
      const float im = A[0].y * i0 + A[1].y * i1 + A[2].y * i2 + A[3].y * i3;
      const float2 by = chirp_y[y];
      v[8 * h + i] = make_float2(re * by.x - im * by.y, re * by.y + im * by.x);
    }
    __syncthreads();  // tile reads done: the area is reused
  }
  int tk = t;
  asm volatile("" : "+v"(tk));
  fft_passes<NY, C::EP, 0, true>(v, tk, tws, reinterpret_cast<float *>(area), ColSlotW<W>{j});
  float2 *o = out + ((size_t)f * NY * 4 + q) * Q + xp;
#pragma unroll
  for (int i = 0; i < E; ++i) o[(size_t)(tk + T * i) * (4 * Q)] = v[i];
}

// ----------------------------------------------------------- passes 2, 3 ----
// A unit is (v, q): the quarter row T[t][v][q][0..Q) of every frame, u = 4 v + q
// (its offset in a frame of T is u Q).  The 32 frame slots (frames >= nt are zero)
// each get T = Q/16 threads of 16 points; the transform exchanges through LDS (real
// and imaginary parts in turn), after which the unit's values are staged in LDS,
// half a row at a time, as X[pixel][frame] (swizzled, below).
// Staging layout: row r (a pixel) holds the 32 frame slots, column c of row r at
// r * 32 + (c ^ swz(r)).  The XOR swizzle makes the three access patterns free of
// bank conflicts (64-bit accesses, 32 lanes per LDS cycle): the transform threads'
// stores (a half-wave covers 32 / T frames x T consecutive rows), the MFMA operand
// loads (16 consecutive frames of two rows, whose swizzles differ in bit 4) and the
// projection loads (four frames of eight consecutive rows).
__device__ __forceinline__ int swz(int r) {
  return (16 * (r & 1)) ^ (4 * ((r >> 1) & 3)) ^ (2 * ((r >> 3) & 1)) ^ ((r >> 4) & 1);
}
__device__ __forceinline__ int sidx(int r, int c) { return r * 32 + (c ^ swz(r)); }
constexpr int kQPitch = 32;

template <int Q>
struct QCfg {
  static constexpr int E = 16, T = Q / 16, NTH = 32 * T, NW = NTH / 64, HALF = Q / 2;
  static constexpr int LDSN = FftCfg<Q, 16>::LDSN;
  static constexpr int XCH = (32 * LDSN > 2 * HALF * kQPitch) ? 32 * LDSN : 2 * HALF * kQPitch;  // floats
  static_assert(T * 8 == HALF && NW * 32 == Q, "unit shape");
};

struct Row1 {
  __device__ __forceinline__ int operator()(int e) const { return fft_pad(e); }
};

// Q-point transform of this thread's frame slot of one unit, staged afterwards
// by the caller.  Shared by passes 2 and 3 so that both see the same H.  A frame's
// T = Q / 16 <= 64 threads lie in one wave and exchange through the frame's own LDS
// area, so the exchanges need only the wave's own ordering.
template <int Q>
__device__ __forceinline__ void quarter_fft(float2 (&v)[16], int t, const float2 *tws, float *xch, int f) {
  static_assert(QCfg<Q>::T <= 64, "a frame's transform within one wave");
  fft_passes<Q, 16, 0, true, true>(v, t, tws, xch + f * QCfg<Q>::LDSN, Row1{});
}

template <int Q, bool PF>
__global__ __launch_bounds__(QCfg<Q>::NTH, PF ? 2 : 4) void qgram(const float2 *__restrict__ tin, int nt, int ny,
                                                      const float2 *__restrict__ tw_x,
                                                      double *__restrict__ partial) {
  using C = QCfg<Q>;
  constexpr int D = 32, E = C::E, T = C::T, NW = C::NW;
  __shared__ __align__(16) float xch[C::XCH];
  __shared__ float2 tws[Q];
  __shared__ double red[2 * D * D];
  const int tid = threadIdx.x;
  const int f = tid / T, t = tid % T;
  const int lane = tid & 63, wave = tid >> 6, fi = lane & 15, kk = lane >> 4;
  for (int i = tid; i < Q; i += C::NTH) tws[i] = tw_x[4 * i];  // W_Q^i = W_nx^{4i}
  for (int i = tid; i < 2 * D * D; i += C::NTH) red[i] = 0.0;
  __syncthreads();

  const int units = 4 * ny, G = gridDim.x;
  const bool fv = f < nt, v0 = fi < nt, v1 = 16 + fi < nt;
  const float2 *fsrc = tin + (size_t)(fv ? f : 0) * ((size_t)units * Q) + t;
  float2 *st = reinterpret_cast<float2 *>(xch);

  v4f S00 = {0.f, 0.f, 0.f, 0.f}, S01 = S00, S11 = S00, Q00 = S00, Q01 = S00, Q10 = S00, Q11 = S00;
  double2 a0 = make_double2(0.0, 0.0), a1 = a0;
  double mm = 0.0;
  auto flush = [&]() {  // fixed wave order
    for (int w = 0; w < NW; ++w) {
      if (wave == w) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 4 * kk + r, j = fi;  // 16x16 accumulator layout
          red[i * D + j] += (double)S00[r];
          red[i * D + 16 + j] += (double)S01[r];
          red[(16 + i) * D + 16 + j] += (double)S11[r];
          red[D * D + i * D + j] += (double)Q00[r];
          red[D * D + i * D + 16 + j] += (double)Q01[r];
          red[D * D + (16 + i) * D + j] += (double)Q10[r];
          red[D * D + (16 + i) * D + 16 + j] += (double)Q11[r];
        }
      }
      __syncthreads();
    }
  };

  // Loads are unconditional (a slot past nt reads frame 0 and is zeroed; the
  // prefetch past the last unit repeats the current one).
  // PF: the next unit's loads are issued before this unit's transform (registers
  // for two units); else one unit's loads at a time, overlapped by other groups.
  const int u0 = xcd_rank(G);
  float2 v[E], nxt[PF ? E : 1];
  if constexpr (PF) {
    const float2 *p = fsrc + (size_t)(u0 < units ? u0 : 0) * Q;
#pragma unroll
    for (int i = 0; i < E; ++i) nxt[i] = p[T * i];
  }
  for (int u = u0; u < units; u += G) {
    if constexpr (PF) {
      const int u2 = u + G < units ? u + G : u;
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = nxt[i];
      const float2 *p = fsrc + (size_t)u2 * Q;
#pragma unroll
      for (int i = 0; i < E; ++i) nxt[i] = p[T * i];
    } else {
      const float2 *p = fsrc + (size_t)u * Q;
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = p[T * i];
    }
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = fv ? v[i] : make_float2(0.f, 0.f);
    int tk = t;
    asm volatile("" : "+v"(tk));
    quarter_fft<Q>(v, tk, tws, xch, f);
    __syncthreads();  // exchange reads done: the area becomes the staging area
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int i = 0; i < 8; ++i) st[sidx(tk + T * i, f)] = v[8 * h + i];
      __syncthreads();
      float a0r = 0.f, a0i = 0.f, a1r = 0.f, a1i = 0.f, mmf = 0.f;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int px = 4 * (4 * wave + ks) + kk;
        const float2 m = st[sidx(px, 0)];
        float2 x0 = st[sidx(px, fi)], x1 = st[sidx(px, 16 + fi)];
        x0 = v0 ? make_float2(x0.x - m.x, x0.y - m.y) : make_float2(0.f, 0.f);
        x1 = v1 ? make_float2(x1.x - m.x, x1.y - m.y) : make_float2(0.f, 0.f);
        mmf += m.x * m.x + m.y * m.y;
        a0r += m.x * x0.x + m.y * x0.y;
        a0i += m.x * x0.y - m.y * x0.x;
        a1r += m.x * x1.x + m.y * x1.y;
        a1i += m.x * x1.y - m.y * x1.x;
        S00 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.x, x0.x, S00, 0, 0, 0);
        S00 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.y, x0.y, S00, 0, 0, 0);
        Q00 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.x, x0.y, Q00, 0, 0, 0);
        S01 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.x, x1.x, S01, 0, 0, 0);
        S01 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.y, x1.y, S01, 0, 0, 0);
        S11 = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.x, x1.x, S11, 0, 0, 0);
        S11 = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.y, x1.y, S11, 0, 0, 0);
        Q01 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.x, x1.y, Q01, 0, 0, 0);
        Q10 = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.x, x0.y, Q10, 0, 0, 0);
        Q11 = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.x, x1.y, Q11, 0, 0, 0);
      }
      a0.x += a0r;
      a0.y += a0i;
      a1.x += a1r;
      a1.y += a1i;
      mm += mmf;
      __syncthreads();  // staging reads done before the next writes
    }
  }
  // the launch gives each group at most 16 units: FP32 sums over at most 512 pixels
  // per accumulator, then FP64
  flush();

  // fixed-order FP64 sums of the rank-one terms, then one store of the partial
  double2 *ared = reinterpret_cast<double2 *>(xch);  // [NW][4][D]
  double *mmred = reinterpret_cast<double *>(ared + NW * 4 * D);
  static_assert((NW * 4 * D * 16 + NW * 4 * 8) <= C::XCH * 4, "rank-one reduction fits the staging area");
  ared[(wave * 4 + kk) * D + fi] = a0;
  ared[(wave * 4 + kk) * D + 16 + fi] = a1;
  if (fi == 0) mmred[wave * 4 + kk] = mm;
  __syncthreads();
  double *o = partial + (size_t)blockIdx.x * partial_len(D);
  for (int i = tid; i < 2 * D * D; i += C::NTH) o[i] = red[i];
  if (tid < D) {
    double ar = 0.0, ai = 0.0;
    for (int w = 0; w < NW * 4; ++w) {
      ar += ared[w * D + tid].x;
      ai += ared[w * D + tid].y;
    }
    o[2 * D * D + tid] = ar;
    o[2 * D * D + D + tid] = ai;
  }
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < NW * 4; ++w) s += mmred[w];
    o[2 * D * D + 2 * D] = s;
    o[2 * D * D + 2 * D + 1] = 0.0;
  }
}

#ifndef HH_FUSED_PF
#define HH_FUSED_PF 0
#endif
constexpr bool kFusedPF = HH_FUSED_PF != 0;  // prefetch form of passes 2 and 3

struct QList {
  int n;
  int k[32];
};

// Pass 3.  Thread (p, c) of a half row: pixel p, lane c of four.  The list holds
// the kept components, or the dropped ones when COMPL: the image is then
// sum_t |h_t|^2 - sum over dropped |h . v_k|^2, exact because V is unitary, in
// FP64 as the kernels on stored holograms.  Short complement lists (<= 8): lane c
// sums frames t = c mod 4 for every component and the lanes' sums are combined;
// otherwise lane c takes components a = c mod 4 over every frame and the lanes'
// values are added.
template <int Q, int KMAX, bool COMPL, bool PF>
__global__ __launch_bounds__(QCfg<Q>::NTH, PF ? 2 : 4) void qproject(const float2 *__restrict__ tin, int nt, int ny,
                                                         const float2 *__restrict__ tw_x,
                                                         const double2 *__restrict__ V, QList kl,
                                                         float *__restrict__ image) {
  using C = QCfg<Q>;
  constexpr int E = C::E, T = C::T, KPT = (KMAX + 3) / 4, NX = 4 * Q;
  typedef typename std::conditional<COMPL, double, float>::type R;
  __shared__ __align__(16) float xch[C::XCH];
  __shared__ float2 tws[Q];
  __shared__ double2 vl[32 * KMAX];
  const int tid = threadIdx.x;
  const int f = tid / T, t = tid % T;
  const int p = tid >> 2, c = tid & 3;
  for (int i = tid; i < Q; i += C::NTH) tws[i] = tw_x[4 * i];
  for (int i = tid; i < 32 * KMAX; i += C::NTH) {
    const int tt = i / KMAX, a = i - tt * KMAX;
    vl[i] = (tt < nt && a < kl.n) ? V[tt * nt + kl.k[a]] : make_double2(0.0, 0.0);
  }
  __syncthreads();

  const int units = 4 * ny, G = gridDim.x;
  const bool fv = f < nt;
  const float2 *fsrc = tin + (size_t)(fv ? f : 0) * ((size_t)units * Q) + t;
  float2 *st = reinterpret_cast<float2 *>(xch);
  const int u0 = xcd_rank(G);
  float2 v[E], nxt[PF ? E : 1];
  if constexpr (PF) {
    const float2 *pp = fsrc + (size_t)(u0 < units ? u0 : 0) * Q;
#pragma unroll
    for (int i = 0; i < E; ++i) nxt[i] = pp[T * i];
  }
  for (int u = u0; u < units; u += G) {
    if constexpr (PF) {
      const int u2 = u + G < units ? u + G : u;
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = nxt[i];
      const float2 *pp = fsrc + (size_t)u2 * Q;
#pragma unroll
      for (int i = 0; i < E; ++i) nxt[i] = pp[T * i];
    } else {
      const float2 *pp = fsrc + (size_t)u * Q;
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] = pp[T * i];
    }
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = fv ? v[i] : make_float2(0.f, 0.f);
    int tk = t;
    asm volatile("" : "+v"(tk));
    quarter_fft<Q>(v, tk, tws, xch, f);
    __syncthreads();
    const int vrow = u >> 2, q = u & 3;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int i = 0; i < 8; ++i) st[sidx(tk + T * i, f)] = v[8 * h + i];
      __syncthreads();
      R val;
      if constexpr (COMPL && KMAX <= 8) {
        // lane c: frames t = c mod 4, every listed (dropped) component; the four
        // lanes' partial sums are combined before the squares
        double nrm = 0.0, zr[KMAX], zi[KMAX];
#pragma unroll
        for (int a = 0; a < KMAX; ++a) zr[a] = zi[a] = 0.0;
        for (int tt = c; tt < nt; tt += 4) {
          const float2 hv = st[sidx(p, tt)];
          const double hr = hv.x, hi = hv.y;
          nrm += hr * hr + hi * hi;
#pragma unroll
          for (int a = 0; a < KMAX; ++a) {
            const double2 vv = vl[tt * KMAX + a];
            zr[a] += hr * vv.x - hi * vv.y;
            zi[a] += hr * vv.y + hi * vv.x;
          }
        }
        nrm += __shfl_xor(nrm, 1);
        nrm += __shfl_xor(nrm, 2);
        double e = 0.0;
#pragma unroll
        for (int a = 0; a < KMAX; ++a) {
          if (a < kl.n) {
            double xr = zr[a], xi = zi[a];
            xr += __shfl_xor(xr, 1);
            xi += __shfl_xor(xi, 1);
            xr += __shfl_xor(xr, 2);
            xi += __shfl_xor(xi, 2);
            e += xr * xr + xi * xi;
          }
        }
        val = nrm - e;
      } else {
        // lane c: components a = c mod 4 of the list, every frame (and, with COMPL,
        // the |h|^2 terms of frames t = c mod 4)
        R nrm = 0, zr[KPT], zi[KPT];
#pragma unroll
        for (int bb = 0; bb < KPT; ++bb) zr[bb] = zi[bb] = 0;
        for (int tt = 0; tt < nt; ++tt) {
          const float2 hv = st[sidx(p, tt)];
          const R hr = hv.x, hi = hv.y;
          if (COMPL) nrm += ((tt & 3) == c) ? hr * hr + hi * hi : R(0);
#pragma unroll
          for (int bb = 0; bb < KPT; ++bb) {
            const double2 vv = vl[tt * KMAX + (c + 4 * bb < KMAX ? c + 4 * bb : 0)];
            const R vr = (R)vv.x, vi = (R)vv.y;
            zr[bb] += hr * vr - hi * vi;
            zi[bb] += hr * vi + hi * vr;
          }
        }
        R e = 0;
#pragma unroll
        for (int bb = 0; bb < KPT; ++bb)
          if (c + 4 * bb < kl.n) e += zr[bb] * zr[bb] + zi[bb] * zi[bb];
        val = COMPL ? nrm - e : e;
        val += __shfl_xor(val, 1);
        val += __shfl_xor(val, 2);
      }
      if (c == 0) image[(size_t)vrow * NX + 4 * (h * C::HALF + p) + q] = (float)val;
      __syncthreads();
    }
  }
}

// as many groups as the compute units hold at once (occupancy queried once per kernel)
int persistent_grid(const void *kernel, int threads, int cus, int units, int &per_cu) {
  if (per_cu == 0) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0) != hipSuccess || occ < 1) occ = 1;
    per_cu = occ;
  }
  int g = per_cu * cus;
  if (g > units) g = units;
  if (g >= 8) g &= ~7;
  return g;
}

template <int NY, int Q>
hipError_t qcols_launch(const Plan &pl, const uint16_t *frames, int nt, float2 *tbuf, hipStream_t s) {
  using C = P1Cfg<NY, Q>;
  ProfScope ps("qcols_u16", s);
  hipLaunchKernelGGL((qcols_u16<NY, Q>), dim3(nt * 4 * C::S), dim3(C::NTH), 0, s, frames, pl.chirp_x, pl.chirp_y,
                     pl.tw_x, pl.tw_y, tbuf);
  return hipGetLastError();
}

template <int Q, bool PF>
hipError_t qgram_launch(const Plan &pl, const float2 *tbuf, int nt, int max_groups, double *partial, int *groups,
                        hipStream_t s) {
  static int per_cu = 0;
  const int units = 4 * pl.ny;
  int g = persistent_grid(reinterpret_cast<const void *>(&qgram<Q, PF>), QCfg<Q>::NTH, pl.cus, units, per_cu);
  // at most 16 units per group (the FP32 partial sums' length); the extra groups
  // of a small device simply wait for a free compute unit
  const int need = ((units + 15) / 16 + 7) & ~7;
  if (g < need) g = need;
  if (g > max_groups) g = max_groups >= 8 ? (max_groups & ~7) : max_groups;
  *groups = g;
  ProfScope ps("qgram", s);
  hipLaunchKernelGGL((qgram<Q, PF>), dim3(g), dim3(QCfg<Q>::NTH), 0, s, tbuf, nt, pl.ny, pl.tw_x, partial);
  return hipGetLastError();
}

template <int Q, int KMAX, bool COMPL, bool PF>
hipError_t qproject_one(const Plan &pl, const float2 *tbuf, int nt, const double2 *V, const QList &kl, float *image,
                        hipStream_t s) {
  static int per_cu = 0;
  const int units = 4 * pl.ny;
  const int g = persistent_grid(reinterpret_cast<const void *>(&qproject<Q, KMAX, COMPL, PF>), QCfg<Q>::NTH,
                                pl.cus, units, per_cu);
  hipLaunchKernelGGL((qproject<Q, KMAX, COMPL, PF>), dim3(g), dim3(QCfg<Q>::NTH), 0, s, tbuf, nt, pl.ny, pl.tw_x, V,
                     kl, image);
  return hipGetLastError();
}

template <int Q, bool COMPL>
hipError_t qproject_k(const Plan &pl, const float2 *tbuf, int nt, const double2 *V, const QList &kl, float *image,
                      hipStream_t s) {
  ProfScope ps(COMPL ? "qproject_complement" : "qproject_direct", s);
  if (kl.n <= 4) return qproject_one<Q, 4, COMPL, kFusedPF>(pl, tbuf, nt, V, kl, image, s);
  if (kl.n <= 8) return qproject_one<Q, 8, COMPL, kFusedPF>(pl, tbuf, nt, V, kl, image, s);
  if (kl.n <= 16) return qproject_one<Q, 16, COMPL, kFusedPF>(pl, tbuf, nt, V, kl, image, s);
  return qproject_one<Q, 32, COMPL, kFusedPF>(pl, tbuf, nt, V, kl, image, s);
}

}  // namespace

bool fused_supported(int nx, int ny, int nt) {
  return nt >= 1 && nt <= 32 && (nx == 512 || nx == 1024 || nx == 2048) && (ny == 512 || ny == 1024);
}

hipError_t launch_fused_front(const Plan &pl, const uint16_t *frames, int nt, float2 *tbuf, int max_groups,
                              double *partial, int *groups, hipStream_t s) {
  hipError_t e = hipErrorInvalidValue;
  switch (pl.nx * 4 + pl.ny / 512) {  // (nx, ny) pairs
#define HH_QCOLS(NX_, NY_) \
  case NX_ * 4 + NY_ / 512: e = qcols_launch<NY_, NX_ / 4>(pl, frames, nt, tbuf, s); break;
    HH_QCOLS(512, 512) HH_QCOLS(512, 1024)
    HH_QCOLS(1024, 512) HH_QCOLS(1024, 1024)
    HH_QCOLS(2048, 512) HH_QCOLS(2048, 1024)
#undef HH_QCOLS
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  switch (pl.nx) {
    case 512: return qgram_launch<128, false>(pl, tbuf, nt, max_groups, partial, groups, s);
    case 1024: return qgram_launch<256, false>(pl, tbuf, nt, max_groups, partial, groups, s);
    case 2048: return qgram_launch<512, false>(pl, tbuf, nt, max_groups, partial, groups, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_fused_back(const Plan &pl, const float2 *tbuf, int nt, const double *V, int k_lo, int k_hi,
                             int mode, float *image, hipStream_t s) {
  const int kept = k_hi - k_lo + 1, dropped = nt - kept;
  const bool compl_ = mode == HH_PROJ_COMPLEMENT || (mode == HH_PROJ_AUTO && dropped <= kept);
  QList kl{};
  for (int k = 0; k < nt; ++k)
    if (compl_ ? (k < k_lo || k > k_hi) : (k >= k_lo && k <= k_hi)) kl.k[kl.n++] = k;
  const double2 *V2 = reinterpret_cast<const double2 *>(V);
  switch (pl.nx) {
    case 512:
      return compl_ ? qproject_k<128, true>(pl, tbuf, nt, V2, kl, image, s)
                    : qproject_k<128, false>(pl, tbuf, nt, V2, kl, image, s);
    case 1024:
      return compl_ ? qproject_k<256, true>(pl, tbuf, nt, V2, kl, image, s)
                    : qproject_k<256, false>(pl, tbuf, nt, V2, kl, image, s);
    case 2048:
      return compl_ ? qproject_k<512, true>(pl, tbuf, nt, V2, kl, image, s)
                    : qproject_k<512, false>(pl, tbuf, nt, V2, kl, image, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace hh
