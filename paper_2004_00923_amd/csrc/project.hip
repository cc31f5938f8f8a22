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
#include "hh_internal.h"

namespace hh {
namespace {

struct KList {
  int n;
  int k[64];
};

template <int KMAX>
__global__ __launch_bounds__(256) void project_direct(const float4 *__restrict__ H, int nt, long long npair,
                                                      const double2 *__restrict__ V, KList kl,
                                                      float2 *__restrict__ image) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= npair) return;
  float2 z0[KMAX], z1[KMAX];
#pragma unroll
  for (int a = 0; a < KMAX; ++a) z0[a] = z1[a] = make_float2(0.f, 0.f);
  for (int t = 0; t < nt; ++t) {
    const float4 h = H[(long long)t * npair + q];
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

template <int KMAX>
__global__ __launch_bounds__(256) void project_complement(const float4 *__restrict__ H, int nt, long long npair,
                                                          const double2 *__restrict__ V, KList kl,
                                                          float2 *__restrict__ image) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= npair) return;
  double n0 = 0.0, n1 = 0.0;
  double2 z0[KMAX > 0 ? KMAX : 1], z1[KMAX > 0 ? KMAX : 1];
#pragma unroll
  for (int a = 0; a < KMAX; ++a) z0[a] = z1[a] = make_double2(0.0, 0.0);
  for (int t = 0; t < nt; ++t) {
    const float4 h = H[(long long)t * npair + q];
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

template <bool COMPL, int KMAX>
void launch_one(dim3 grid, const float4 *H, int nt, long long npair, const double2 *V, const KList &kl, float2 *img,
                hipStream_t s) {
  if constexpr (COMPL)
    hipLaunchKernelGGL(project_complement<KMAX>, grid, dim3(256), 0, s, H, nt, npair, V, kl, img);
  else
    hipLaunchKernelGGL(project_direct<KMAX>, grid, dim3(256), 0, s, H, nt, npair, V, kl, img);
}

template <bool COMPL>
hipError_t launch_k(int kcount, const float4 *H, int nt, long long npair, const double2 *V, const KList &kl,
                    float2 *img, hipStream_t s) {
  const dim3 grid((unsigned)((npair + 255) / 256));
  ProfScope ps(COMPL ? "project_complement" : "project_direct", s);
  if (kcount <= 2) launch_one<COMPL, 2>(grid, H, nt, npair, V, kl, img, s);
  else if (kcount <= 4) launch_one<COMPL, 4>(grid, H, nt, npair, V, kl, img, s);
  else if (kcount <= 8) launch_one<COMPL, 8>(grid, H, nt, npair, V, kl, img, s);
  else if (kcount <= 16) launch_one<COMPL, 16>(grid, H, nt, npair, V, kl, img, s);
  else if (kcount <= 32) launch_one<COMPL, 32>(grid, H, nt, npair, V, kl, img, s);
  else launch_one<COMPL, 64>(grid, H, nt, npair, V, kl, img, s);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_project(const float2 *holo, int nt, long long npix, const double *V, int k_lo, int k_hi,
                          int mode, float *image, hipStream_t s) {
  const int kept = k_hi - k_lo + 1, dropped = nt - kept;
  const bool complement = mode == HH_PROJ_COMPLEMENT || (mode == HH_PROJ_AUTO && dropped <= kept);
  KList kl{};
  if (complement) {
    for (int k = 0; k < nt; ++k)
      if (k < k_lo || k > k_hi) kl.k[kl.n++] = k;
  } else {
    for (int k = k_lo; k <= k_hi; ++k) kl.k[kl.n++] = k;
  }
  const long long npair = npix / 2;
  const float4 *H4 = reinterpret_cast<const float4 *>(holo);
  const double2 *V2 = reinterpret_cast<const double2 *>(V);
  float2 *img = reinterpret_cast<float2 *>(image);
  if (complement) return launch_k<true>(kl.n, H4, nt, npair, V2, kl, img, s);
  return launch_k<false>(kl.n, H4, nt, npair, V2, kl, img, s);
}

}  // namespace hh
