// Steps (d)+(e), Eqs. (6)-(7): M[p] = sum over kept k of |sum_t H[p][t] V[t][k]|^2,
// with the projection fused into the |.|^2 sum (the components are never stored).
//
// Two evaluations of the same quantity:
//   direct     : the kept components in FP32;
//   complement : sum_t |H[p][t]|^2 - sum over dropped k of |.|^2 in FP64, exact because
//                V is unitary (Eq. (5)); cheap when few components are dropped, and
//                FP64 because the kept energy can be a small part of the total.
// One thread handles two neighbouring pixels (one 16-byte load per frame); V is
// wave-uniform and is read through the scalar cache.
#include <type_traits>

#include "hh_internal.h"

namespace hh {
namespace {

struct KList {
  int n;
  int k[64];
};

// Frame t of the two pixels of pair q, as (re, im, re, im).
struct LoadF32 {  // complex64 hologram [nt][npix]
  const float4 *H;
  long long npair;
  __device__ __forceinline__ float4 operator()(int t, long long q) const { return H[(long long)t * npair + q]; }
};
struct LoadR16 {  // FP16 storage form: H = m + R / s
  const uint2 *R;
  const float4 *M;
  long long npair;
  float inv_s;
  __device__ __forceinline__ float4 operator()(int t, long long q) const {
    union {
      uint2 u;
      h2 h[2];
    } x;
    x.u = R[(long long)t * npair + q];
    const float4 m = M[q];
    return make_float4(m.x + (float)x.h[0].x * inv_s, m.y + (float)x.h[0].y * inv_s, m.z + (float)x.h[1].x * inv_s,
                       m.w + (float)x.h[1].y * inv_s);
  }
};

template <int KMAX, class Load>
__global__ __launch_bounds__(256) void project_direct(Load H, int nt, long long npair,
                                                      const double2 *__restrict__ V, KList kl,
                                                      float2 *__restrict__ image) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= npair) return;
  float2 z0[KMAX], z1[KMAX];
#pragma unroll
  for (int a = 0; a < KMAX; ++a) z0[a] = z1[a] = make_float2(0.f, 0.f);
  for (int t = 0; t < nt; ++t) {
    const float4 h = H(t, q);
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
      if (a < kl.n) {
        const double2 vd = V[t * nt + kl.k[a]];
        const float vr = (float)vd.x, vi = (float)vd.y;
        z0[a].x += h.x * vr - h.y * vi;
        z0[a].y += h.x * vi + h.y * vr;
        z1[a].x += h.z * vr - h.w * vi;
        z1[a].y += h.z * vi + h.w * vr;
      }
    }
  }
  float m0 = 0.f, m1 = 0.f;
#pragma unroll
  for (int a = 0; a < KMAX; ++a) {
    if (a < kl.n) {
      m0 += z0[a].x * z0[a].x + z0[a].y * z0[a].y;
      m1 += z1[a].x * z1[a].x + z1[a].y * z1[a].y;
    }
  }
  image[q] = make_float2(m0, m1);
}

template <int KMAX, class Load>
__global__ __launch_bounds__(256) void project_complement(Load H, int nt, long long npair,
                                                          const double2 *__restrict__ V, KList kl,
                                                          float2 *__restrict__ image) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= npair) return;
  double n0 = 0.0, n1 = 0.0;
  double2 z0[KMAX > 0 ? KMAX : 1], z1[KMAX > 0 ? KMAX : 1];
#pragma unroll
  for (int a = 0; a < KMAX; ++a) z0[a] = z1[a] = make_double2(0.0, 0.0);
  for (int t = 0; t < nt; ++t) {
    const float4 h = H(t, q);
    const double r0 = h.x, i0 = h.y, r1 = h.z, i1 = h.w;
    n0 += r0 * r0 + i0 * i0;
    n1 += r1 * r1 + i1 * i1;
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
      if (a < kl.n) {
        const double2 v = V[t * nt + kl.k[a]];
        z0[a].x += r0 * v.x - i0 * v.y;
        z0[a].y += r0 * v.y + i0 * v.x;
        z1[a].x += r1 * v.x - i1 * v.y;
        z1[a].y += r1 * v.y + i1 * v.x;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < KMAX; ++a) {
    if (a < kl.n) {
      n0 -= z0[a].x * z0[a].x + z0[a].y * z0[a].y;
      n1 -= z1[a].x * z1[a].x + z1[a].y * z1[a].y;
    }
  }
  image[q] = make_float2((float)n0, (float)n1);
}

template <bool COMPL, int KMAX, class Load>
void launch_one(dim3 grid, const Load &H, int nt, long long npair, const double2 *V, const KList &kl, float2 *img,
                hipStream_t s) {
  if constexpr (COMPL)
    hipLaunchKernelGGL((project_complement<KMAX, Load>), grid, dim3(256), 0, s, H, nt, npair, V, kl, img);
  else
    hipLaunchKernelGGL((project_direct<KMAX, Load>), grid, dim3(256), 0, s, H, nt, npair, V, kl, img);
}

template <bool COMPL, class Load>
hipError_t launch_k(int kcount, const Load &H, int nt, long long npair, const double2 *V, const KList &kl,
                    float2 *img, hipStream_t s, const char *name) {
  const dim3 grid((unsigned)((npair + 255) / 256));
  ProfScope ps(name, s);
  if (kcount <= 2) launch_one<COMPL, 2>(grid, H, nt, npair, V, kl, img, s);
  else if (kcount <= 4) launch_one<COMPL, 4>(grid, H, nt, npair, V, kl, img, s);
  else if (kcount <= 8) launch_one<COMPL, 8>(grid, H, nt, npair, V, kl, img, s);
  else if (kcount <= 16) launch_one<COMPL, 16>(grid, H, nt, npair, V, kl, img, s);
  else if (kcount <= 32) launch_one<COMPL, 32>(grid, H, nt, npair, V, kl, img, s);
  else launch_one<COMPL, 64>(grid, H, nt, npair, V, kl, img, s);
  return hipGetLastError();
}

// SVD-filtered stack, Eq. (3): Hf = H V I_f V^H, i.e. per pixel
//   Hf[p][t] = sum over kept k of c_k conj(V[t][k]),      c_k = sum_s H[p][s] V[s][k]   (direct, FP32)
//            = H[p][t] - sum over dropped k of c_k conj(V[t][k])                         (complement, FP64 c_k)
// Two passes over the pixel's frames: the coefficients, then one output frame at a
// time (the second read of H comes mostly from cache).  Two pixels per thread.
template <bool COMPL, int KMAX>
__global__ __launch_bounds__(256) void svd_filter_k(const float4 *__restrict__ H, int nt, long long npair,
                                                    const double2 *__restrict__ V, KList kl,
                                                    float4 *__restrict__ out) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= npair) return;
  typedef typename std::conditional<COMPL, double, float>::type T;
  T c0r[KMAX], c0i[KMAX], c1r[KMAX], c1i[KMAX];
#pragma unroll
  for (int a = 0; a < KMAX; ++a) c0r[a] = c0i[a] = c1r[a] = c1i[a] = T(0);
  for (int t = 0; t < nt; ++t) {
    const float4 h = H[(long long)t * npair + q];
    const T r0 = h.x, i0 = h.y, r1 = h.z, i1 = h.w;
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
      if (a < kl.n) {
        const double2 vd = V[t * nt + kl.k[a]];
        const T vr = (T)vd.x, vi = (T)vd.y;
        c0r[a] += r0 * vr - i0 * vi;
        c0i[a] += r0 * vi + i0 * vr;
        c1r[a] += r1 * vr - i1 * vi;
        c1i[a] += r1 * vi + i1 * vr;
      }
    }
  }
  for (int t = 0; t < nt; ++t) {
    T o0r = 0, o0i = 0, o1r = 0, o1i = 0;
#pragma unroll
    for (int a = 0; a < KMAX; ++a) {
      if (a < kl.n) {
        const double2 vd = V[t * nt + kl.k[a]];  // times conj(v)
        const T vr = (T)vd.x, vi = (T)vd.y;
        o0r += c0r[a] * vr + c0i[a] * vi;
        o0i += c0i[a] * vr - c0r[a] * vi;
        o1r += c1r[a] * vr + c1i[a] * vi;
        o1i += c1i[a] * vr - c1r[a] * vi;
      }
    }
    float4 o;
    if constexpr (COMPL) {
      const float4 h = H[(long long)t * npair + q];
      o = make_float4((float)((T)h.x - o0r), (float)((T)h.y - o0i), (float)((T)h.z - o1r), (float)((T)h.w - o1i));
    } else {
      o = make_float4(o0r, o0i, o1r, o1i);
    }
    out[(long long)t * npair + q] = o;
  }
}

template <bool COMPL>
hipError_t launch_filter(int kcount, const float4 *H, int nt, long long npair, const double2 *V, const KList &kl,
                         float4 *out, hipStream_t s) {
  const dim3 grid((unsigned)((npair + 255) / 256)), b(256);
  ProfScope ps(COMPL ? "svd_filter_complement" : "svd_filter_direct", s);
  if (kcount <= 2) hipLaunchKernelGGL((svd_filter_k<COMPL, 2>), grid, b, 0, s, H, nt, npair, V, kl, out);
  else if (kcount <= 4) hipLaunchKernelGGL((svd_filter_k<COMPL, 4>), grid, b, 0, s, H, nt, npair, V, kl, out);
  else if (kcount <= 8) hipLaunchKernelGGL((svd_filter_k<COMPL, 8>), grid, b, 0, s, H, nt, npair, V, kl, out);
  else if (kcount <= 16) hipLaunchKernelGGL((svd_filter_k<COMPL, 16>), grid, b, 0, s, H, nt, npair, V, kl, out);
  else if (kcount <= 32) hipLaunchKernelGGL((svd_filter_k<COMPL, 32>), grid, b, 0, s, H, nt, npair, V, kl, out);
  else hipLaunchKernelGGL((svd_filter_k<COMPL, 64>), grid, b, 0, s, H, nt, npair, V, kl, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The direct projection on MFMA (precision forms): M[p] = sum over kept k of
// |z_k|^2 with z = h V restated as a real product.  Each pixel is split as
// h = m + r, m its temporal mean (FP32), so z_k = m s_k + sum_t r_t V[t][k] with
// s_k = sum_t V[t][k]: only r (a few per cent of h) goes through the low-precision
// format, m s_k is added in FP32.  With c = 2a + part (a = position in the kept
// list, part 0/1 = real/imaginary) and kk = 2t + part' (frame t),
//   Z[c][p] = sum_kk A[c][kk] B[kk][p],  A = [[Re V, -Im V], [Im V, Re V]] per (a, t),
//   B[2t][p] = Re r_t(p), B[2t+1][p] = Im r_t(p),
// a 64 x 64 by 64 x 16 product per 16 pixels on v_mfma_f32_16x16x32_{bf16,f16} or
// _fp8_fp8 (4 row tiles x 2 k-steps), with FP32 accumulation.  A (from V, a
// 64 x 64 matrix shared by every pixel) is always kept as hi + lo and both parts
// are multiplied with B (two products); SPLIT also splits B (the streamed
// residual) and adds the hi*lo' product (three).  B is scaled per pixel by a power of two (FP16, FP8)
// so that its largest entry fits the format, and A by 2^8 for FP8 (|V| <= 1); the
// scales are undone exactly in the epilogue.  One wave takes 16 pixels at a time:
// lane (n, g), n = lane % 16 the pixel, g = lane / 16 the k-block, holds frames
// 16 j + 4 g .. + 3 of k-step j (8 values: re, im of four frames).
enum { kPjBF16 = 0, kPjFP16 = 1, kPjFP8 = 2 };

typedef __bf16 pv8bf __attribute__((ext_vector_type(8)));
typedef _Float16 pv8h __attribute__((ext_vector_type(8)));
typedef float pv4f __attribute__((ext_vector_type(4)));

template <int FMT>
struct PjOp;
template <>
struct PjOp<kPjBF16> {
  typedef pv8bf vec;
  typedef __bf16 elt;
  static constexpr float kLim = 0.f;  // no scale
  __device__ static elt cvt(float x) { return (__bf16)x; }
  __device__ static float back(elt x) { return (float)x; }
  __device__ static pv4f mma(const vec &a, const vec &b, pv4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct PjOp<kPjFP16> {
  typedef pv8h vec;
  typedef _Float16 elt;
  static constexpr float kLim = 16384.f;  // headroom for the lo residual and the sums
  __device__ static elt cvt(float x) { return (_Float16)x; }
  __device__ static float back(elt x) { return (float)x; }
  __device__ static pv4f mma(const vec &a, const vec &b, pv4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct PjOp<kPjFP8> {
  typedef long vec;
  typedef unsigned char elt;
  static constexpr float kLim = 448.f;  // OCP e4m3 maximum
  __device__ static elt cvt(float x) { return (unsigned char)(__builtin_amdgcn_cvt_pk_fp8_f32(x, 0.f, 0, false) & 0xFF); }
  __device__ static float back(elt x) { return __builtin_amdgcn_cvt_f32_fp8((int)x, 0); }
  __device__ static pv4f mma(const vec &a, const vec &b, pv4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0);
  }
};

template <int FMT, bool SPLIT>
__global__ __launch_bounds__(256, 3) void project_mfma(const float2 *__restrict__ H, int nt, long long npix,
                                                    const double2 *__restrict__ V, KList kl,
                                                    float *__restrict__ image) {
  typedef PjOp<FMT> Op;
  typedef typename Op::elt elt;
  typedef typename Op::vec vec;
  union Frag {
    vec v;
    elt e[8];
  };
  constexpr float kAScale = FMT == kPjFP8 ? 256.f : 1.f;
  // rows padded to 72 elements: the 16 lanes of an LDS phase (rows n, 16-byte fragments)
  // then fall on distinct banks
  constexpr int LA = 72;
  __shared__ __align__(16) elt Ahi[64 * LA], Alo[64 * LA];
  __shared__ float2 ssum[32];
  const int tid = threadIdx.x, lane = tid & 63;
  const int n = lane & 15, g = lane >> 4;
  const float inv_nt = 1.f / (float)nt;
  // A (rows c = 2a + part, columns kk = 2t + part'), hi and lo parts
  for (int i = tid; i < 64 * 64; i += 256) {
    const int c = i >> 6, kk = i & 63, a = c >> 1, t = kk >> 1;
    float x = 0.f;
    if (a < kl.n && t < nt) {
      const double2 v = V[t * nt + kl.k[a]];
      const int pp = ((c & 1) << 1) | (kk & 1);
      x = (float)(pp == 0 ? v.x : pp == 1 ? -v.y : pp == 2 ? v.y : v.x) * kAScale;
    }
    const elt h = Op::cvt(x);
    Ahi[c * LA + kk] = h;
    Alo[c * LA + kk] = Op::cvt(x - Op::back(h));
  }
  if (tid < 32) {
    double sr = 0.0, si = 0.0;
    if (tid < kl.n)
      for (int t = 0; t < nt; ++t) {
        const double2 v = V[t * nt + kl.k[tid]];
        sr += v.x;
        si += v.y;
      }
    ssum[tid] = make_float2((float)sr, (float)si);
  }
  __syncthreads();
  // this lane's components (rows 16 rt + 4 g + r): a = 8 rt + 2 g + r / 2, with their
  // column sums in registers (zero past the kept set, whose rows of A are zero too,
  // so that those rows add nothing and the epilogue needs no branch); the A
  // fragments are read from LDS where they are used (one 8-element vector each)
  float2 sv[4][2];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int u = 0; u < 2; ++u) sv[rt][u] = ssum[8 * rt + 2 * g + u];
  int an = n;  // made opaque per pair below (BF16, FP16), so that the fragment reads are not hoisted
              // into registers
  auto afrag = [&](const elt *A, int rt, int j) {
    return *reinterpret_cast<const vec *>(A + (16 * rt + an) * LA + 32 * j + 8 * g);
  };
  // Two 16-pixel tiles at a time: lane (n, g) loads pixels 2n and 2n + 1 of the pair
  // (one 16-byte load per frame), which are column n of the first and of the second
  // tile.  Each wave takes a contiguous range of pairs, so that its 32 frame streams
  // are read sequentially.  npix is a multiple of 64: every pair is whole.
  const long long pairs = npix / 32;
  const long long waves = (long long)gridDim.x * 4, per = (pairs + waves - 1) / waves;
  const long long t_begin = ((long long)blockIdx.x * 4 + (tid >> 6)) * per;
  const long long t_end = t_begin + per < pairs ? t_begin + per : pairs;
  // the eight frames of this lane for one pair; the next pair's are loaded before
  // this pair is converted and multiplied (unconditional loads from a valid address)
  auto load = [&](long long tp, float4 (&d)[2][4]) {
    const long long pc = tp < t_end ? tp * 32 + 2 * n : 0;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t = 16 * j + 4 * g + i;
        d[j][i] = *reinterpret_cast<const float4 *>(H + (long long)(t < nt ? t : 0) * npix + pc);
      }
  };
  // one tile: the pixel's temporal mean split off, the per-pixel scale, the MFMA
  // products, the |.|^2 sum over the components (all four lanes of the pixel get it)
  auto tile = [&](const float2 (&hin)[2][4]) {
    float2 h[2][4];
    float mr = 0.f, mi = 0.f;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        h[j][i] = hin[j][i];
        if (16 * j + 4 * g + i < nt) {
          mr += h[j][i].x;
          mi += h[j][i].y;
        }
      }
    mr += __shfl_xor(mr, 16);
    mi += __shfl_xor(mi, 16);
    mr += __shfl_xor(mr, 32);
    mi += __shfl_xor(mi, 32);
    mr *= inv_nt;
    mi *= inv_nt;
    float mx = 0.f;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const bool on = 16 * j + 4 * g + i < nt;
        h[j][i] = on ? make_float2(h[j][i].x - mr, h[j][i].y - mi) : make_float2(0.f, 0.f);
        mx = fmaxf(mx, fmaxf(fabsf(h[j][i].x), fabsf(h[j][i].y)));
      }
    float sc = 1.f;
    if constexpr (Op::kLim > 0.f) {
      mx = fmaxf(mx, __shfl_xor(mx, 16));
      mx = fmaxf(mx, __shfl_xor(mx, 32));
      if (mx > 0.f) {
        int ex;
        frexpf(Op::kLim / mx, &ex);  // kLim / mx = f 2^ex, f in [0.5, 1)
        sc = ldexpf(1.f, ex - 1);
      }
    }
    Frag bh[2], bl[2];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const float x = (q ? h[j][i].y : h[j][i].x) * sc;
          const elt hi = Op::cvt(x);
          bh[j].e[2 * i + q] = hi;
          if constexpr (SPLIT) bl[j].e[2 * i + q] = Op::cvt(x - Op::back(hi));
        }
    const float inv = 1.f / (sc * kAScale);  // powers of two: exact
    float e = 0.f;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      pv4f acc = pv4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc = Op::mma(afrag(Ahi, rt, j), bh[j].v, acc);
        acc = Op::mma(afrag(Alo, rt, j), bh[j].v, acc);
        if constexpr (SPLIT) acc = Op::mma(afrag(Ahi, rt, j), bl[j].v, acc);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const float2 s = sv[rt][u];
        const float zr = acc[2 * u] * inv + (mr * s.x - mi * s.y);
        const float zi = acc[2 * u + 1] * inv + (mr * s.y + mi * s.x);
        e += zr * zr + zi * zi;
      }
    }
    e += __shfl_xor(e, 16);
    e += __shfl_xor(e, 32);
    return e;
  };
  float4 nx_[2][4];
  load(t_begin, nx_);
  for (long long tp = t_begin; tp < t_end; ++tp) {
    float2 h0[2][4], h1[2][4];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        h0[j][i] = make_float2(nx_[j][i].x, nx_[j][i].y);
        h1[j][i] = make_float2(nx_[j][i].z, nx_[j][i].w);
      }
    load(tp + 1, nx_);
    an = n;
    if constexpr (FMT != kPjFP8) asm volatile("" : "+v"(an));  // FP8 fragments (8 bytes) stay in registers
    const float e0 = tile(h0);
    __builtin_amdgcn_sched_barrier(0);  // one tile's work at a time (registers)
    const float e1 = tile(h1);
    if (g == 0) *reinterpret_cast<float2 *>(image + tp * 32 + 2 * n) = make_float2(e0, e1);
  }
}

template <int FMT, bool SPLIT>
hipError_t launch_pmfma(const float2 *H, int nt, long long npix, const double2 *V, const KList &kl, float *image,
                        hipStream_t s) {
  // every group builds the operand table of the kept components first: about sixteen
  // pairs of tiles per wave amortise it (at most 512 groups, two per compute unit)
  const long long pairs = npix / 32;      // pairs of 16-pixel tiles (npix is a multiple of 64)
  long long groups = (pairs + 63) / 64;
  if (groups < 1) groups = 1;
  if (groups > 512) groups = 512;
  hipLaunchKernelGGL((project_mfma<FMT, SPLIT>), dim3((unsigned)groups), dim3(256), 0, s, H, nt, npix, V, kl, image);
  return hipGetLastError();
}

// FP32 direct projection, Eq. (6) as written (the kept components, no complement),
// on v_mfma_f32_32x32x2f32: D[c][n] = sum_kk A[c][kk] B[kk][n] with rows c = 2a + part
// (component a of the kept list), columns n = 32 pixels, kk = 2t + part over the
// frames, A the real 2x2 form of V[t][k_a] and B = H minus the pixel's temporal mean
// m (the mean's contribution m s_a, s_a = sum_t V[t][k_a], is added in the epilogue,
// as in the low-precision forms).  Lane (j, h) of a wave holds pixel j of the tile:
// all its frames (the two lanes j and 32 + j load the same 8 bytes), the real parts
// as B operand for h = 0, the imaginary parts for h = 1.  RB row blocks of 32: one
// when at most 16 components are kept (the direct mode chosen automatically), two
// for up to 32.  n_t <= 32.
__device__ __forceinline__ int acc32_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

typedef float pv16f __attribute__((ext_vector_type(16)));

template <int RB>
__global__ __launch_bounds__(256, 2) void project_mfma32(const float2 *__restrict__ H, int nt, long long npix,
                                                      const double2 *__restrict__ V, KList kl,
                                                      float *__restrict__ image) {
  __shared__ float Af[64 * 65];
  __shared__ float2 ssum[32];
  const int tid = threadIdx.x, lane = tid & 63, j = lane & 31, h = lane >> 5;
  for (int i = tid; i < 64 * 64; i += 256) {
    const int c = i >> 6, kk = i & 63, a = c >> 1, t = kk >> 1;
    float x = 0.f;
    if (a < kl.n && t < nt) {
      const double2 v = V[t * nt + kl.k[a]];
      const int pp = ((c & 1) << 1) | (kk & 1);
      x = (float)(pp == 0 ? v.x : pp == 1 ? -v.y : pp == 2 ? v.y : v.x);
    }
    Af[c * 65 + kk] = x;
  }
  if (tid < 32) {
    double sr = 0.0, si = 0.0;
    if (tid < kl.n)
      for (int t = 0; t < nt; ++t) {
        const double2 v = V[t * nt + kl.k[tid]];
        sr += v.x;
        si += v.y;
      }
    ssum[tid] = make_float2((float)sr, (float)si);
  }
  __syncthreads();
  // A operand of K-step s for row block rb: A[32 rb + j][2 s + h]
  float av[RB][32];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int s = 0; s < 32; ++s) av[rb][s] = Af[(32 * rb + j) * 65 + 2 * s + h];
  // this lane's components: rows 32 rb + 8 q + 4 h + u, u = 0..3 -> components
  // 16 rb + 4 q + 2 h (u = 0, 1) and that + 1 (u = 2, 3); their column sums
  float2 sv[RB][4][2];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int u = 0; u < 2; ++u) sv[rb][q][u] = ssum[16 * rb + 4 * q + 2 * h + u];
  const float inv_nt = 1.f / (float)nt;
  const long long tiles = npix / 32;  // npix is a multiple of 64
  for (long long tl = blockIdx.x * 4 + (tid >> 6); tl < tiles; tl += (long long)gridDim.x * 4) {
    const long long p = tl * 32 + j;
    float2 x[32];
#pragma unroll
    for (int t = 0; t < 32; ++t) x[t] = H[(long long)(t < nt ? t : 0) * npix + p];
    float mr = 0.f, mi = 0.f;
#pragma unroll
    for (int t = 0; t < 32; ++t)
      if (t < nt) {
        mr += x[t].x;
        mi += x[t].y;
      }
    mr *= inv_nt;
    mi *= inv_nt;
    pv16f acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[rb][r] = 0.f;
#pragma unroll
    for (int s = 0; s < 32; ++s) {
      const float b = s < nt ? (h ? x[s].y - mi : x[s].x - mr) : 0.f;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) acc[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rb][s], b, acc[rb], 0, 0, 0);
    }
    float e = 0.f;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const float2 sa = sv[rb][q][u];
          const float zr = acc[rb][4 * q + 2 * u] + (mr * sa.x - mi * sa.y);
          const float zi = acc[rb][4 * q + 2 * u + 1] + (mr * sa.y + mi * sa.x);
          e += zr * zr + zi * zi;
        }
    e += __shfl_xor(e, 32);
    if (h == 0) image[p] = e;
  }
}

hipError_t launch_pmfma32(const float2 *H, int nt, long long npix, const double2 *V, const KList &kl, float *image,
                          hipStream_t s) {
  const long long tiles = npix / 32;
  long long groups = (tiles + 31) / 32;  // about eight tiles per wave
  if (groups < 1) groups = 1;
  if (groups > 1024) groups = 1024;
  if (kl.n <= 16)
    hipLaunchKernelGGL((project_mfma32<1>), dim3((unsigned)groups), dim3(256), 0, s, H, nt, npix, V, kl, image);
  else
    hipLaunchKernelGGL((project_mfma32<2>), dim3((unsigned)groups), dim3(256), 0, s, H, nt, npix, V, kl, image);
  return hipGetLastError();
}

// kept / dropped component lists of the selector I_f
bool select_list(int nt, int k_lo, int k_hi, int mode, KList &kl) {
  const int kept = k_hi - k_lo + 1, dropped = nt - kept;
  const bool complement = mode == HH_PROJ_COMPLEMENT || (mode == HH_PROJ_AUTO && dropped <= kept);
  kl = KList{};
  for (int k = 0; k < nt; ++k)
    if (complement ? (k < k_lo || k > k_hi) : (k >= k_lo && k <= k_hi)) kl.k[kl.n++] = k;
  return complement;
}

}  // namespace

hipError_t launch_svd_filter(const float2 *holo, int nt, long long npix, const double *V, int k_lo, int k_hi,
                             int mode, float2 *out, hipStream_t s) {
  KList kl;
  const bool complement = select_list(nt, k_lo, k_hi, mode, kl);
  const long long npair = npix / 2;
  const float4 *H4 = reinterpret_cast<const float4 *>(holo);
  const double2 *V2 = reinterpret_cast<const double2 *>(V);
  float4 *o4 = reinterpret_cast<float4 *>(out);
  if (complement) return launch_filter<true>(kl.n, H4, nt, npair, V2, kl, o4, s);
  return launch_filter<false>(kl.n, H4, nt, npair, V2, kl, o4, s);
}

hipError_t launch_project(const float2 *holo, int nt, long long npix, const double *V, int k_lo, int k_hi,
                          int mode, float *image, hipStream_t s, int precision) {
  KList kl;
  if (precision >= HH_BF16 && precision <= HH_FP8E4M3 && nt <= 32 && mode != HH_PROJ_COMPLEMENT) {
    // precision forms: the kept components on MFMA in the form's operand format
    select_list(nt, k_lo, k_hi, HH_PROJ_DIRECT, kl);
    const double2 *V2 = reinterpret_cast<const double2 *>(V);
    ProfScope ps("project_mfma", s);
    switch (precision) {
      case HH_BF16: return launch_pmfma<kPjBF16, false>(holo, nt, npix, V2, kl, image, s);
      case HH_BF16X3: return launch_pmfma<kPjBF16, true>(holo, nt, npix, V2, kl, image, s);
      case HH_FP16: return launch_pmfma<kPjFP16, false>(holo, nt, npix, V2, kl, image, s);
      case HH_FP16X3: return launch_pmfma<kPjFP16, true>(holo, nt, npix, V2, kl, image, s);
      default: return launch_pmfma<kPjFP8, false>(holo, nt, npix, V2, kl, image, s);
    }
  }
  const bool complement = select_list(nt, k_lo, k_hi, mode, kl);
  const long long npair = npix / 2;
  const LoadF32 H{reinterpret_cast<const float4 *>(holo), npair};
  const double2 *V2 = reinterpret_cast<const double2 *>(V);
  float2 *img = reinterpret_cast<float2 *>(image);
  if (complement) return launch_k<true>(kl.n, H, nt, npair, V2, kl, img, s, "project_complement");
  if (nt <= 32 && npix % 64 == 0) {  // the kept components on FP32 MFMA
    ProfScope ps("project_direct", s);
    return launch_pmfma32(holo, nt, npix, V2, kl, image, s);
  }
  return launch_k<false>(kl.n, H, nt, npair, V2, kl, img, s, "project_direct");
}

hipError_t launch_project_r16(const h2 *r16, const float2 *m, float inv_s, int nt, long long npix, const double *V,
                              int k_lo, int k_hi, int mode, float *image, hipStream_t s) {
  KList kl;
  const bool complement = select_list(nt, k_lo, k_hi, mode, kl);
  const long long npair = npix / 2;
  const LoadR16 H{reinterpret_cast<const uint2 *>(r16), reinterpret_cast<const float4 *>(m), npair, inv_s};
  const double2 *V2 = reinterpret_cast<const double2 *>(V);
  float2 *img = reinterpret_cast<float2 *>(image);
  if (complement) return launch_k<true>(kl.n, H, nt, npair, V2, kl, img, s, "project_r16_complement");
  return launch_k<false>(kl.n, H, nt, npair, V2, kl, img, s, "project_r16_direct");
}

}  // namespace hh
