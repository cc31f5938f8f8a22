// Step (b), Eq. (4): C = H^{t*} H as a tall-skinny split-K Gram on FP32 MFMA.
//
// With R = A + iB (A, B real, one column per frame):
//   Re R^H R = A^T A + B^T B,   Im (R^H R)[s][t] = (A^T B)[s][t] - (A^T B)[t][s].
// Each wave streams its own pixel range straight from HBM in MFMA operand layout
// (lanes = frames, MFMA k-slots = pixels); there is no LDS or barrier in the
// main loop.
//
// Accuracy: the stack is dominated by its temporal mean (the static speckle),
// so C is dominated by one eigenvalue while the components the image keeps sit
// ~1e-3 below it.  FP32 sums of raw products would leave errors of ~1e-8 of the
// top eigenvalue, enough to tilt the kept subspace when the boundary gap is
// small.  Each pixel is therefore split exactly as H = m 1^T + R, m the pixel's
// temporal mean (any m works: R is formed as H - m), and
//   C = (m^H m) 1 1^T + 1 a^T + conj(a) 1^T + R^H R,   a_t = sum_p conj(m_p) R[p][t],
// with R^H R on MFMA (FP32 sums over at most 512 products per accumulator) and
// the rank-one terms carried to FP64 every 8 pixels.  Partials are combined in
// FP64 in a fixed order (waves, then workgroups in two levels), so the result is
// deterministic.
#include "hh_internal.h"

namespace hh {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Output of accumulator register r on lane l of a 32x32 MFMA block.
__device__ __forceinline__ int acc_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// Length (doubles) of one workgroup partial: S, Q (D x D each), a (re, im), m^H m, pad.
__host__ __device__ constexpr int partial_len(int D) { return 2 * D * D + 2 * D + 2; }

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
// Sum over the 16 lanes of a DPP row (butterfly: every lane gets the same bits).
__device__ __forceinline__ float sum16(float v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  return v;
}
// Sum over the 32 lanes of each half-wave: the 16-lane sum plus one swizzle (XOR 16).
__device__ __forceinline__ float sum32(float v) {
  v = sum16(v);
  return v + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
}

// n_t <= 32 path on v_mfma_f32_16x16x4f32: lane (f, k), f = lane % 16, k = lane / 16,
// holds frames f and 16 + f of pixel slot k.  A 16-byte load of lane k covers
// pixels 8j + 2k, 8j + 2k + 1, so one load instruction reads 64 contiguous bytes
// of each of 16 frames, and the two MFMA steps of a load take pixels
// {8j, 8j+2, 8j+4, 8j+6} and {8j+1, 8j+3, 8j+5, 8j+7}.  The 32-frame mean of a
// pixel is a 16-lane sum of the two values (DPP).  S needs the upper 16x16
// blocks 00, 01, 11 only; Q all four.  TWO = false when n_t <= 16.
template <bool TWO>
__global__ __launch_bounds__(256) void gram_partial16(const float2 *__restrict__ H, int nt, long long npix,
                                                      double *__restrict__ partial) {
  constexpr int D = 32;
  constexpr int G4 = 4;  // 16-byte loads per stream per iteration (32 pixels of the wave)
  __shared__ double red[2 * D * D];
  __shared__ double2 ared[4][4][D];
  __shared__ double mmred[4][4];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int f = lane & 15, k = lane >> 4;
  const float inv_nt = 1.0f / (float)nt;

  v4f S00 = {0.f, 0.f, 0.f, 0.f}, S01 = S00, S11 = S00, Q00 = S00, Q01 = S00, Q10 = S00, Q11 = S00;
  double2 a0 = make_double2(0.0, 0.0), a1 = a0;
  double mm = 0.0;

  const long long p0 = ((long long)blockIdx.x * 4 + wave) * kGramPxPerWave;  // first pixel of this wave
  const bool v0 = f < nt, v1 = TWO && (16 + f) < nt;
  const float4 *s0p = reinterpret_cast<const float4 *>(H + (long long)(v0 ? f : 0) * npix + p0) + k;
  const float4 *s1p = reinterpret_cast<const float4 *>(H + (long long)(v1 ? 16 + f : 0) * npix + p0) + k;

  for (int q0 = 0; q0 < kGramPxPerWave; q0 += 8 * G4) {
    float4 h0[G4], h1[G4];
#pragma unroll
    for (int g = 0; g < G4; ++g) {
      const bool in = p0 + q0 + 8 * g + 2 * k < npix;
      h0[g] = (v0 && in) ? s0p[(q0 >> 1) + 4 * g] : make_float4(0.f, 0.f, 0.f, 0.f);
      h1[g] = (v1 && in) ? s1p[(q0 >> 1) + 4 * g] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float a0r = 0.f, a0i = 0.f, a1r = 0.f, a1i = 0.f, mmf = 0.f;  // FP32 sums over 8 pixels per lane
#pragma unroll
    for (int g = 0; g < G4; ++g) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        float2 x0 = e ? make_float2(h0[g].z, h0[g].w) : make_float2(h0[g].x, h0[g].y);
        float2 x1 = e ? make_float2(h1[g].z, h1[g].w) : make_float2(h1[g].x, h1[g].y);
        const float mr = sum16(x0.x + x1.x) * inv_nt, mi = sum16(x0.y + x1.y) * inv_nt;
        mmf += mr * mr + mi * mi;
        if (v0) {
          x0.x -= mr;
          x0.y -= mi;
        }
        if (v1) {
          x1.x -= mr;
          x1.y -= mi;
        }
        a0r += mr * x0.x + mi * x0.y;
        a0i += mr * x0.y - mi * x0.x;
        S00 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.x, x0.x, S00, 0, 0, 0);
        S00 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.y, x0.y, S00, 0, 0, 0);
        Q00 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.x, x0.y, Q00, 0, 0, 0);
        if constexpr (TWO) {
          a1r += mr * x1.x + mi * x1.y;
          a1i += mr * x1.y - mi * x1.x;
          S01 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.x, x1.x, S01, 0, 0, 0);
          S01 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.y, x1.y, S01, 0, 0, 0);
          S11 = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.x, x1.x, S11, 0, 0, 0);
          S11 = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.y, x1.y, S11, 0, 0, 0);
          Q01 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.x, x1.y, Q01, 0, 0, 0);
          Q10 = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.x, x0.y, Q10, 0, 0, 0);
          Q11 = __builtin_amdgcn_mfma_f32_16x16x4f32(x1.x, x1.y, Q11, 0, 0, 0);
        }
      }
    }
    a0.x += a0r;
    a0.y += a0i;
    a1.x += a1r;
    a1.y += a1i;
    mm += mmf;
  }

  // fixed-order FP64 combination of the four waves, then one store
  for (int i = tid; i < 2 * D * D; i += 256) red[i] = 0.0;
  ared[wave][k][f] = a0;
  ared[wave][k][16 + f] = a1;
  if (f == 0) mmred[wave][k] = mm;
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * k + r, j = f;  // 16x16 accumulator layout
        red[i * D + j] += (double)S00[r];
        red[D * D + i * D + j] += (double)Q00[r];
        if constexpr (TWO) {
          red[i * D + 16 + j] += (double)S01[r];
          red[(16 + i) * D + 16 + j] += (double)S11[r];
          red[D * D + i * D + 16 + j] += (double)Q01[r];
          red[D * D + (16 + i) * D + j] += (double)Q10[r];
          red[D * D + (16 + i) * D + 16 + j] += (double)Q11[r];
        }
      }
    }
    __syncthreads();
  }
  double *out = partial + (size_t)blockIdx.x * partial_len(D);
  for (int i = tid; i < 2 * D * D; i += 256) out[i] = red[i];
  if (tid < D) {
    double ar = 0.0, ai = 0.0;
    for (int w = 0; w < 4; ++w)
      for (int q = 0; q < 4; ++q) {
        ar += ared[w][q][tid].x;
        ai += ared[w][q][tid].y;
      }
    out[2 * D * D + tid] = ar;
    out[2 * D * D + D + tid] = ai;
  }
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < 4; ++w)
      for (int q = 0; q < 4; ++q) t += mmred[w][q];
    out[2 * D * D + 2 * D] = t;
    out[2 * D * D + 2 * D + 1] = 0.0;
  }
}

// 32 < n_t <= 64 path on v_mfma_f32_32x32x2f32: lane (fr, half) holds frames fr and
// 32 + fr; the two half-waves take one half of the wave's pixels each.
__global__ __launch_bounds__(256) void gram_partial64(const float2 *__restrict__ H, int nt, long long npix,
                                                      double *__restrict__ partial) {
  constexpr int D = 64;
  constexpr int HALF = kGramPxPerWave / 2;  // pixels per half-wave
  constexpr int G4 = 4;
  __shared__ double red[2 * D * D];
  __shared__ double2 ared[4][2][D];
  __shared__ double mmred[4][2];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int fr = lane & 31, half = lane >> 5;
  const float inv_nt = 1.0f / (float)nt;

  v16f S[3], Q[4];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) S[b][r] = 0.f;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) Q[b][r] = 0.f;
  double2 a_acc[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
  double mm_acc = 0.0;

  const long long p0 = ((long long)blockIdx.x * 4 + wave) * kGramPxPerWave + (long long)half * HALF;
  const float4 *src[2];
  bool valid[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int t = 32 * b + fr;
    valid[b] = t < nt;
    src[b] = reinterpret_cast<const float4 *>(H + (long long)(valid[b] ? t : 0) * npix + p0);
  }

  for (int s0 = 0; s0 < HALF; s0 += 2 * G4) {
    float4 h[2][G4];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int g = 0; g < G4; ++g) {
        const long long px = p0 + s0 + 2 * g;
        h[b][g] = (valid[b] && px < npix) ? src[b][s0 / 2 + g] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
    for (int g = 0; g < G4; ++g) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        float2 x[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) x[b] = e ? make_float2(h[b][g].z, h[b][g].w) : make_float2(h[b][g].x, h[b][g].y);
        const float mr = sum32(x[0].x + x[1].x) * inv_nt, mi = sum32(x[0].y + x[1].y) * inv_nt;
        const double dmr = mr, dmi = mi;
        mm_acc += dmr * dmr + dmi * dmi;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          if (valid[b]) {
            x[b].x -= mr;
            x[b].y -= mi;
          }
          const double rr = x[b].x, ri = x[b].y;
          a_acc[b].x += dmr * rr + dmi * ri;
          a_acc[b].y += dmr * ri - dmi * rr;
        }
        S[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[0].x, x[0].x, S[0], 0, 0, 0);
        S[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[0].y, x[0].y, S[0], 0, 0, 0);
        S[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[0].x, x[1].x, S[1], 0, 0, 0);
        S[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[0].y, x[1].y, S[1], 0, 0, 0);
        S[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[1].x, x[1].x, S[2], 0, 0, 0);
        S[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[1].y, x[1].y, S[2], 0, 0, 0);
        Q[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[0].x, x[0].y, Q[0], 0, 0, 0);
        Q[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[0].x, x[1].y, Q[1], 0, 0, 0);
        Q[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[1].x, x[0].y, Q[2], 0, 0, 0);
        Q[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[1].x, x[1].y, Q[3], 0, 0, 0);
      }
    }
  }

  for (int i = tid; i < 2 * D * D; i += 256) red[i] = 0.0;
#pragma unroll
  for (int b = 0; b < 2; ++b) ared[wave][half][32 * b + fr] = a_acc[b];
  if (fr == 0) mmred[wave][half] = mm_acc;
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const int bi = b == 2 ? 1 : 0, bj = b == 0 ? 0 : 1;
#pragma unroll
        for (int r = 0; r < 16; ++r) red[(32 * bi + acc_row(lane, r)) * D + 32 * bj + fr] += (double)S[b][r];
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int bi = b / 2, bj = b % 2;
#pragma unroll
        for (int r = 0; r < 16; ++r)
          red[D * D + (32 * bi + acc_row(lane, r)) * D + 32 * bj + fr] += (double)Q[b][r];
      }
    }
    __syncthreads();
  }
  double *out = partial + (size_t)blockIdx.x * partial_len(D);
  for (int i = tid; i < 2 * D * D; i += 256) out[i] = red[i];
  if (tid < D) {
    double ar = 0.0, ai = 0.0;
    for (int w = 0; w < 4; ++w)
      for (int h2 = 0; h2 < 2; ++h2) {
        ar += ared[w][h2][tid].x;
        ai += ared[w][h2][tid].y;
      }
    out[2 * D * D + tid] = ar;
    out[2 * D * D + D + tid] = ai;
  }
  if (tid == 0) {
    double t = 0.0;
    for (int w = 0; w < 4; ++w)
      for (int h2 = 0; h2 < 2; ++h2) t += mmred[w][h2];
    out[2 * D * D + 2 * D] = t;
    out[2 * D * D + 2 * D + 1] = 0.0;
  }
}

// out[g2][l] = sum over g in segment g2 of in[g][l], segments in increasing g.
__global__ __launch_bounds__(256) void gram_reduce(const double *__restrict__ in, int G, int L, int G2,
                                                   double *__restrict__ out) {
  const int l = blockIdx.x * 256 + threadIdx.x;
  const int g2 = blockIdx.y;
  if (l >= L) return;
  const int g0 = (int)((long long)g2 * G / G2), g1 = (int)((long long)(g2 + 1) * G / G2);
  double s = 0.0;
#pragma unroll 8
  for (int g = g0; g < g1; ++g) s += in[(size_t)g * L + l];
  out[(size_t)g2 * L + l] = s;
}

// Assemble the Hermitian C = (m^H m) 1 1^T + 1 a^T + conj(a) 1^T + R^H R from the
// summed partials (S = Re R^H R upper blocks, Q = A^T B of R = A + iB).
__global__ __launch_bounds__(256) void gram_finalize(const double *__restrict__ in2, int G2, int D, int nt,
                                                     double2 *__restrict__ cov) {
  const size_t L = partial_len(D);
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nt * nt) return;
  const int s = e / nt, t = e % nt;
  const int lo = s < t ? s : t, hi = s < t ? t : s;
  double re = 0.0, qst = 0.0, qts = 0.0, mm = 0.0, alo = 0.0, ahi = 0.0, ais = 0.0, ait = 0.0;
#pragma unroll 4
  for (int g = 0; g < G2; ++g) {
    const double *p = in2 + g * L;
    re += p[lo * D + hi];
    qst += p[(size_t)D * D + s * D + t];
    qts += p[(size_t)D * D + t * D + s];
    alo += p[2 * D * D + lo];
    ahi += p[2 * D * D + hi];
    ais += p[2 * D * D + D + s];
    ait += p[2 * D * D + D + t];
    mm += p[2 * D * D + 2 * D];
  }
  cov[e] = make_double2((re + mm) + (alo + ahi), (qst - qts) + (ait - ais));
}

}  // namespace

GramLayout gram_layout(int nt, long long npix) {
  GramLayout L;
  L.nb = nt <= 32 ? 1 : 2;
  L.D = 32 * L.nb;
  L.chunks = (npix + kGramPxPerWave - 1) / kGramPxPerWave;  // one chunk per wave
  L.groups = (int)((L.chunks + 3) / 4);
  L.groups2 = L.groups < 16 ? L.groups : 16;
  L.partial_bytes = (size_t)L.groups * partial_len(L.D) * sizeof(double);
  L.partial2_bytes = (size_t)L.groups2 * partial_len(L.D) * sizeof(double);
  return L;
}

hipError_t launch_gram(const GramLayout &L, const float2 *holo, int nt, long long npix, double *partial,
                       double *partial2, double *cov, hipStream_t s) {
  {
    ProfScope ps("gram_partial", s);
    if (nt <= 16)
      hipLaunchKernelGGL(gram_partial16<false>, dim3(L.groups), dim3(256), 0, s, holo, nt, npix, partial);
    else if (nt <= 32)
      hipLaunchKernelGGL(gram_partial16<true>, dim3(L.groups), dim3(256), 0, s, holo, nt, npix, partial);
    else
      hipLaunchKernelGGL(gram_partial64, dim3(L.groups), dim3(256), 0, s, holo, nt, npix, partial);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int Lw = partial_len(L.D);
  {
    ProfScope ps("gram_reduce", s);
    hipLaunchKernelGGL(gram_reduce, dim3((Lw + 255) / 256, L.groups2), dim3(256), 0, s, partial, L.groups, Lw,
                       L.groups2, partial2);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  {
    ProfScope ps("gram_finalize", s);
    hipLaunchKernelGGL(gram_finalize, dim3((nt * nt + 255) / 256), dim3(256), 0, s, partial2, L.groups2, L.D, nt,
                       reinterpret_cast<double2 *>(cov));
  }
  return hipGetLastError();
}

}  // namespace hh
