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
                          int mode, float *image, hipStream_t s) {
  KList kl;
  const bool complement = select_list(nt, k_lo, k_hi, mode, kl);
  const long long npair = npix / 2;
  const LoadF32 H{reinterpret_cast<const float4 *>(holo), npair};
  const double2 *V2 = reinterpret_cast<const double2 *>(V);
  float2 *img = reinterpret_cast<float2 *>(image);
  if (complement) return launch_k<true>(kl.n, H, nt, npair, V2, kl, img, s, "project_complement");
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
