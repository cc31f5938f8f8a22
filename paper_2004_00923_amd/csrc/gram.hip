// Step (b), Eq. (4): C = H^{t*} H as a tall-skinny split-K Gram on FP32 MFMA.
//
// With R = A + iB (A, B real, one column per frame) and M = A^T B:
//   Re R^H R = A^T A + B^T B = (A + B)^T (A + B) - M - M^T,
//   Im (R^H R)[s][t] = M[s][t] - M[t][s],
// so the FP32 forms take three real products per block pair (N = (A + B)^T (A + B)
// on the upper blocks, M on all of them) and form Re in FP64 from the summed N, M.
// Each wave streams its own pixel range straight from HBM in MFMA operand layout
// (lanes = frames, MFMA k-slots = pixels); there is no LDS or barrier in the
// main loop.
//
// Accuracy: the stack is dominated by its temporal mean (the static speckle),
// so C is dominated by one eigenvalue while the components the image keeps sit
// ~1e-3 below it.  FP32 sums of raw products would leave errors of ~1e-8 of the
// top eigenvalue, enough to tilt the kept subspace when the boundary gap is
// small.  Each pixel is therefore split exactly as H = m 1^T + R, m a reference
// value of the pixel (any m works: R is formed as H - m): its temporal mean, or
// its frame-0 value, which removes the static part as well and costs one DPP
// row broadcast instead of a 16-lane sum; and
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
typedef double v4d __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Output of accumulator register r on lane l of a 32x32 MFMA block.
__device__ __forceinline__ int acc_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// second-level partial count (the first level is summed in this many segments)
constexpr int kGroups2 = 16;

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

// The real part of R^H R from N = (A + B)^T (A + B) and M = A^T B (R = A + iB):
//   A^T A + B^T B = N - M - M^T,
// three real products per block pair instead of four.  red holds N's upper blocks
// in [0, D*D) and M in [D*D, 2*D*D), summed in FP64; the upper triangle of the
// first area becomes S = Re R^H R (the part the assembly reads).  Each thread
// rewrites entries it alone reads and writes, then the block synchronises.
template <int D>
__device__ __forceinline__ void n_to_s(double *red, int tid) {
  for (int e = tid; e < D * D; e += 256) {
    const int i = e / D, j = e % D;
    if (i <= j) red[e] = red[e] - red[D * D + i * D + j] - red[D * D + j * D + i];
  }
  __syncthreads();
}

// n_t <= 32 path on v_mfma_f32_16x16x4f32: lane (f, k), f = lane % 16, k = lane / 16,
// holds frames f and 16 + f of pixel slot k.  A 16-byte load of lane k covers
// pixels 8j + 2k, 8j + 2k + 1, so one load instruction reads 64 contiguous bytes
// of each of 16 frames, and the two MFMA steps of a load take pixels
// {8j, 8j+2, 8j+4, 8j+6} and {8j+1, 8j+3, 8j+5, 8j+7}.  MEAN: the reference is
// the temporal mean, a 16-lane sum of the two values (DPP); else frame 0's value,
// broadcast from lane f = 0 of the row.  S needs the upper 16x16 blocks 00, 01,
// 11 only; Q all four.  TWO = false when n_t <= 16.
template <bool TWO, bool MEAN>
__global__ __launch_bounds__(256) void gram_partial16(const float2 *__restrict__ H, int nt, long long npix,
                                                      int pxw, double *__restrict__ partial) {
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

  const long long p0 = ((long long)blockIdx.x * 4 + wave) * pxw;  // first pixel of this wave
  const bool v0 = f < nt, v1 = TWO && (16 + f) < nt;
  const float4 *f0 = reinterpret_cast<const float4 *>(H + (long long)(v0 ? f : 0) * npix);
  const float4 *f1 = reinterpret_cast<const float4 *>(H + (long long)(v1 ? 16 + f : 0) * npix);
  // Loads are unconditional (past the end they read the frame's first pixels, and
  // the prefetch after the last chunk reads that chunk again) and masked when the
  // chunk is taken up, so the next chunk's loads stay in flight while the current
  // one is summed.  A chunk is held in vector registers (16 floats per frame
  // stream), which the compiler keeps out of scratch across iterations.
  v16f h0, h1, n0, n1;
  unsigned hmask = 0, nmask = 0;  // bit g: pixel pair g of the chunk is inside the frame
#pragma unroll
  for (int g = 0; g < G4; ++g) {
    const long long px = p0 + 8 * g + 2 * k;
    const bool in = px < npix;
    hmask |= in ? (1u << g) : 0u;
    const float4 a = f0[in ? (px >> 1) : 0], b = f1[in ? (px >> 1) : 0];
    h0[4 * g] = a.x; h0[4 * g + 1] = a.y; h0[4 * g + 2] = a.z; h0[4 * g + 3] = a.w;
    h1[4 * g] = b.x; h1[4 * g + 1] = b.y; h1[4 * g + 2] = b.z; h1[4 * g + 3] = b.w;
  }
  for (int q0 = 0; q0 < pxw; q0 += 8 * G4) {
    const int qn = (q0 + 8 * G4 < pxw) ? q0 + 8 * G4 : q0;
    nmask = 0;
#pragma unroll
    for (int g = 0; g < G4; ++g) {
      const long long px = p0 + qn + 8 * g + 2 * k;
      const bool in = px < npix;
      nmask |= in ? (1u << g) : 0u;
      const float4 a = f0[in ? (px >> 1) : 0], b = f1[in ? (px >> 1) : 0];
      n0[4 * g] = a.x; n0[4 * g + 1] = a.y; n0[4 * g + 2] = a.z; n0[4 * g + 3] = a.w;
      n1[4 * g] = b.x; n1[4 * g + 1] = b.y; n1[4 * g + 2] = b.z; n1[4 * g + 3] = b.w;
    }
    float4 hc0[G4], hc1[G4];  // the current chunk, masked
#pragma unroll
    for (int g = 0; g < G4; ++g) {
      const bool in = (hmask >> g) & 1u;
      const bool i0 = v0 && in, i1 = v1 && in;
      hc0[g] = make_float4(i0 ? h0[4 * g] : 0.f, i0 ? h0[4 * g + 1] : 0.f, i0 ? h0[4 * g + 2] : 0.f,
                           i0 ? h0[4 * g + 3] : 0.f);
      hc1[g] = make_float4(i1 ? h1[4 * g] : 0.f, i1 ? h1[4 * g + 1] : 0.f, i1 ? h1[4 * g + 2] : 0.f,
                           i1 ? h1[4 * g + 3] : 0.f);
    }
    float a0r = 0.f, a0i = 0.f, a1r = 0.f, a1i = 0.f, mmf = 0.f;  // FP32 sums over 8 pixels per lane
#pragma unroll
    for (int g = 0; g < G4; ++g) {
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        float2 x0 = e ? make_float2(hc0[g].z, hc0[g].w) : make_float2(hc0[g].x, hc0[g].y);
        float2 x1 = e ? make_float2(hc1[g].z, hc1[g].w) : make_float2(hc1[g].x, hc1[g].y);
        float mr, mi;
        if constexpr (MEAN) {
          mr = sum16(x0.x + x1.x) * inv_nt;
          mi = sum16(x0.y + x1.y) * inv_nt;
        } else {
          mr = dpp<0x150>(x0.x);  // row_newbcast:0 (lane f = 0 holds frame 0)
          mi = dpp<0x150>(x0.y);
        }
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
        // S holds N = (A + B)^T (A + B): one product per block instead of two
        const float u0 = x0.x + x0.y;
        S00 = __builtin_amdgcn_mfma_f32_16x16x4f32(u0, u0, S00, 0, 0, 0);
        Q00 = __builtin_amdgcn_mfma_f32_16x16x4f32(x0.x, x0.y, Q00, 0, 0, 0);
        if constexpr (TWO) {
          a1r += mr * x1.x + mi * x1.y;
          a1i += mr * x1.y - mi * x1.x;
          const float u1 = x1.x + x1.y;
          S01 = __builtin_amdgcn_mfma_f32_16x16x4f32(u0, u1, S01, 0, 0, 0);
          S11 = __builtin_amdgcn_mfma_f32_16x16x4f32(u1, u1, S11, 0, 0, 0);
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
    h0 = n0;
    h1 = n1;
    hmask = nmask;
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
  n_to_s<D>(red, tid);
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
// 32 + fr; the two half-waves take one half of the wave's pixels each.  MEAN: the
// reference is the temporal mean (a 32-lane sum); else frame 0's value, read from
// lane 0 of each half-wave.
template <bool MEAN>
__global__ __launch_bounds__(256, 2) void gram_partial64(const float2 *__restrict__ H, int nt, long long npix,
                                                      int pxw, double *__restrict__ partial) {
  constexpr int D = 64;
  const int HALF = pxw / 2;  // pixels per half-wave
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

  const long long p0 = ((long long)blockIdx.x * 4 + wave) * pxw + (long long)half * HALF;
  const float4 *src[2];
  bool valid[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int t = 32 * b + fr;
    valid[b] = t < nt;
    src[b] = reinterpret_cast<const float4 *>(H + (long long)(valid[b] ? t : 0) * npix);
  }
  // Loads are unconditional (past the end they read the frame's first pixels; the
  // prefetch after the last chunk reads that chunk again) and masked when the chunk
  // is taken up, so the next chunk's loads stay in flight while the current one is
  // summed.  Chunk: 8 pixels of each of the lane's two frames, 16 floats each.
  v16f h0, h1, n0, n1;
  unsigned hmask = 0, nmask = 0;  // bit g: pixel pair g of the chunk is inside the frame
  auto load = [&](int s, v16f &c0, v16f &c1, unsigned &mask) {
    mask = 0;
#pragma unroll
    for (int g = 0; g < G4; ++g) {
      const long long px = p0 + s + 2 * g;
      const bool in = px < npix;
      mask |= in ? (1u << g) : 0u;
      const float4 x = src[0][in ? (px >> 1) : 0], y = src[1][in ? (px >> 1) : 0];
      c0[4 * g] = x.x; c0[4 * g + 1] = x.y; c0[4 * g + 2] = x.z; c0[4 * g + 3] = x.w;
      c1[4 * g] = y.x; c1[4 * g + 1] = y.y; c1[4 * g + 2] = y.z; c1[4 * g + 3] = y.w;
    }
  };
  load(0, h0, h1, hmask);
  for (int s0 = 0; s0 < HALF; s0 += 2 * G4) {
    load(s0 + 2 * G4 < HALF ? s0 + 2 * G4 : s0, n0, n1, nmask);
#pragma unroll
    for (int g = 0; g < G4; ++g) {
      const bool in = (hmask >> g) & 1u;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        float2 x[2];
        x[0] = (in && valid[0]) ? make_float2(h0[4 * g + 2 * e], h0[4 * g + 2 * e + 1]) : make_float2(0.f, 0.f);
        x[1] = (in && valid[1]) ? make_float2(h1[4 * g + 2 * e], h1[4 * g + 2 * e + 1]) : make_float2(0.f, 0.f);
        float mr, mi;
        if constexpr (MEAN) {
          mr = sum32(x[0].x + x[1].x) * inv_nt;
          mi = sum32(x[0].y + x[1].y) * inv_nt;
        } else {  // lanes 0 and 32 hold frame 0 of their half-wave's pixel
          const int lo_r = __builtin_amdgcn_readlane(__float_as_int(x[0].x), 0);
          const int lo_i = __builtin_amdgcn_readlane(__float_as_int(x[0].y), 0);
          const int hi_r = __builtin_amdgcn_readlane(__float_as_int(x[0].x), 32);
          const int hi_i = __builtin_amdgcn_readlane(__float_as_int(x[0].y), 32);
          mr = __int_as_float(half ? hi_r : lo_r);
          mi = __int_as_float(half ? hi_i : lo_i);
        }
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
        // S holds N = (A + B)^T (A + B): one product per block instead of two
        const float u0 = x[0].x + x[0].y, u1 = x[1].x + x[1].y;
        S[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(u0, u0, S[0], 0, 0, 0);
        S[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(u0, u1, S[1], 0, 0, 0);
        S[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(u1, u1, S[2], 0, 0, 0);
        Q[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[0].x, x[0].y, Q[0], 0, 0, 0);
        Q[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[0].x, x[1].y, Q[1], 0, 0, 0);
        Q[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[1].x, x[0].y, Q[2], 0, 0, 0);
        Q[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[1].x, x[1].y, Q[3], 0, 0, 0);
      }
    }
    h0 = n0;
    h1 = n1;
    hmask = nmask;
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
  n_to_s<D>(red, tid);
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


// ---------------------------------------------------------------------------
// Low-precision forms of the R^H R contraction (n_t <= 32).  R = H - m is formed
// in FP32 exactly as above (the rank-one terms stay FP32/FP64), then rounded to
// the operand format, and R^H R runs on v_mfma_f32_16x16x32_{bf16,f16} or
// v_mfma_f32_16x16x32_fp8_fp8 with FP32 accumulation.  SPLIT keeps r = hi + lo
// and sums hi*hi' + hi*lo' + lo*hi' (the lo*lo' term is dropped).  FP16 uses a
// power-of-two scale per wave and FP8 (OCP e4m3, max 448) one per wave and
// frame, both chosen from a first pass over the wave's pixels so that the
// largest |Re|, |Im| fits; the scales are undone exactly when the partial sums
// are converted to FP64.
// Lane (f, kq) holds frames f and 16 + f of 8 pixels per 32-pixel step: element e
// is pixel 8 (e / 2) + 2 kq + (e % 2), so each 16-byte load instruction covers 64
// contiguous bytes of 16 frames.
enum { kLpBF16 = 0, kLpFP16 = 1, kLpFP8 = 2 };

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));


template <int FMT>
struct LpOp;
template <>
struct LpOp<kLpBF16> {
  typedef v8bf vec;
  union U {
    vec v;
    __bf16 s[8];
  };
  // hardware round to nearest even (v_cvt_pk_bf16_f32)
  __device__ static float put(U &u, int e, float x) {
    const __bf16 b = (__bf16)x;
    u.s[e] = b;
    return (float)b;
  }
  __device__ static v4f mma(const vec &a, const vec &b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <>
struct LpOp<kLpFP16> {
  typedef v8h vec;
  union U {
    vec v;
    _Float16 s[8];
  };
  __device__ static float put(U &u, int e, float x) {
    const _Float16 h = (_Float16)x;
    u.s[e] = h;
    return (float)h;
  }
  __device__ static v4f mma(const vec &a, const vec &b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0); }
};
template <>
struct LpOp<kLpFP8> {
  typedef long vec;
  union U {
    long v;
    unsigned char s[8];
  };
  // OCP e4m3 round-to-nearest-even of a value already scaled into [-448, 448]
  __device__ static float put(U &u, int e, float x) {
    const int pk = __builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false);
    u.s[e] = (unsigned char)(pk & 0xFF);
    return __builtin_amdgcn_cvt_f32_fp8(pk, 0);
  }
  __device__ static v4f mma(const vec &a, const vec &b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0); }
};

__device__ __forceinline__ float max16(float v) {
  v = fmaxf(v, dpp<0xB1>(v));
  v = fmaxf(v, dpp<0x4E>(v));
  v = fmaxf(v, dpp<0x141>(v));
  v = fmaxf(v, dpp<0x140>(v));
  return v;
}
// max over the four 16-lane rows (lanes f, f+16, f+32, f+48)
__device__ __forceinline__ float max_rows(float v) {
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F)));  // xor 16
  v = fmaxf(v, __shfl_xor(v, 32));
  return v;
}
// power of two s with max * s <= lim (1 for max == 0)
__device__ __forceinline__ float pow2_scale(float mx, float lim) {
  if (!(mx > 0.f)) return 1.f;
  int e;
  frexpf(lim / mx, &e);  // lim/mx = f * 2^e, f in [0.5, 1)
  return ldexpf(1.f, e - 1);
}

template <int FMT, bool SPLIT>
__global__ __launch_bounds__(256) void gram_partial_lp(const float2 *__restrict__ H, int nt, long long npix,
                                                       int pxw, double *__restrict__ partial) {
  constexpr int D = 32;
  typedef LpOp<FMT> Op;
  typedef typename Op::U U;
  __shared__ double red[2 * D * D];
  __shared__ double2 ared[4][4][D];
  __shared__ double mmred[4][4];
  __shared__ float fscale[4][D];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int f = lane & 15, kq = lane >> 4;
  const float inv_nt = 1.0f / (float)nt;
  const long long p0 = ((long long)blockIdx.x * 4 + wave) * pxw;
  const bool v0 = f < nt, v1 = (16 + f) < nt;
  const float4 *s0p = reinterpret_cast<const float4 *>(H + (long long)(v0 ? f : 0) * npix);
  const float4 *s1p = reinterpret_cast<const float4 *>(H + (long long)(v1 ? 16 + f : 0) * npix);

  // One step: pixels 8g + 2kq, 8g + 2kq + 1 (g < 4) of the wave's 32, of frames f and
  // 16 + f.  Loads are unconditional (past the end they read the frame's first
  // pixels) and masked when the step is unpacked, so that a prefetched step's loads
  // stay in flight while the current step is summed; a step is held in vector
  // registers (16 floats per frame stream).
  auto load_raw = [&](int j, v16f &c0, v16f &c1, unsigned &mask) {
    mask = 0;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const long long px = p0 + 32 * j + 8 * g + 2 * kq;
      const bool in = px < npix;
      mask |= in ? (1u << g) : 0u;
      const float4 a = s0p[in ? (px >> 1) : 0], b = s1p[in ? (px >> 1) : 0];
      c0[4 * g] = a.x; c0[4 * g + 1] = a.y; c0[4 * g + 2] = a.z; c0[4 * g + 3] = a.w;
      c1[4 * g] = b.x; c1[4 * g + 1] = b.y; c1[4 * g + 2] = b.z; c1[4 * g + 3] = b.w;
    }
  };
  auto unpack = [&](const v16f &c0, const v16f &c1, unsigned mask, float2 (&x0)[8], float2 (&x1)[8]) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const bool in = (mask >> g) & 1u;
      const bool i0 = v0 && in, i1 = v1 && in;
      x0[2 * g] = i0 ? make_float2(c0[4 * g], c0[4 * g + 1]) : make_float2(0.f, 0.f);
      x0[2 * g + 1] = i0 ? make_float2(c0[4 * g + 2], c0[4 * g + 3]) : make_float2(0.f, 0.f);
      x1[2 * g] = i1 ? make_float2(c1[4 * g], c1[4 * g + 1]) : make_float2(0.f, 0.f);
      x1[2 * g + 1] = i1 ? make_float2(c1[4 * g + 2], c1[4 * g + 3]) : make_float2(0.f, 0.f);
    }
  };
  const int STEPS = pxw / 32;

  // pass A (FP16, FP8): largest |Re|, |Im| of R, per wave or per wave and frame
  float sc0 = 1.f, sc1 = 1.f;
  if constexpr (FMT != kLpBF16) {
    float m0 = 0.f, m1 = 0.f;
    for (int j = 0; j < STEPS; ++j) {
      v16f c0, c1;
      unsigned mask;
      load_raw(j, c0, c1, mask);
      float2 x0[8], x1[8];
      unpack(c0, c1, mask, x0, x1);
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float mr = sum16(x0[e].x + x1[e].x) * inv_nt, mi = sum16(x0[e].y + x1[e].y) * inv_nt;
        if (v0) m0 = fmaxf(m0, fmaxf(fabsf(x0[e].x - mr), fabsf(x0[e].y - mi)));
        if (v1) m1 = fmaxf(m1, fmaxf(fabsf(x1[e].x - mr), fabsf(x1[e].y - mi)));
      }
    }
    m0 = max_rows(m0);
    m1 = max_rows(m1);
    if constexpr (FMT == kLpFP16) {
      const float mw = max16(fmaxf(m0, m1));  // whole wave
      sc0 = sc1 = pow2_scale(mw, 16384.f);     // headroom for the hi/lo residual and partial sums
    } else {
      sc0 = pow2_scale(m0, 448.f);
      sc1 = pow2_scale(m1, 448.f);
    }
  }
  if (kq == 0) {
    fscale[wave][f] = sc0;
    fscale[wave][16 + f] = sc1;
  }

  v4f S00 = {0.f, 0.f, 0.f, 0.f}, S01 = S00, S11 = S00, Q00 = S00, Q01 = S00, Q10 = S00, Q11 = S00;
  double2 a0 = make_double2(0.0, 0.0), a1 = a0;
  double mm = 0.0;
  v16f h0, h1, n0, n1;
  unsigned hmask = 0, nmask = 0;
  load_raw(0, h0, h1, hmask);
  for (int j = 0; j < STEPS; ++j) {
    load_raw(j + 1 < STEPS ? j + 1 : j, n0, n1, nmask);  // the last prefetch repeats the step
    float2 x0[8], x1[8];
    unpack(h0, h1, hmask, x0, x1);
    U r0h, i0h, r1h, i1h, r0l, i0l, r1l, i1l;
    float a0r = 0.f, a0i = 0.f, a1r = 0.f, a1i = 0.f, mmf = 0.f;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float mr = sum16(x0[e].x + x1[e].x) * inv_nt, mi = sum16(x0[e].y + x1[e].y) * inv_nt;
      mmf += mr * mr + mi * mi;
      float2 q0 = x0[e], q1 = x1[e];
      if (v0) {
        q0.x -= mr;
        q0.y -= mi;
      }
      if (v1) {
        q1.x -= mr;
        q1.y -= mi;
      }
      a0r += mr * q0.x + mi * q0.y;
      a0i += mr * q0.y - mi * q0.x;
      a1r += mr * q1.x + mi * q1.y;
      a1i += mr * q1.y - mi * q1.x;
      const float hr0 = Op::put(r0h, e, q0.x * sc0), hi0 = Op::put(i0h, e, q0.y * sc0);
      const float hr1 = Op::put(r1h, e, q1.x * sc1), hi1 = Op::put(i1h, e, q1.y * sc1);
      if constexpr (SPLIT) {
        Op::put(r0l, e, q0.x * sc0 - hr0);
        Op::put(i0l, e, q0.y * sc0 - hi0);
        Op::put(r1l, e, q1.x * sc1 - hr1);
        Op::put(i1l, e, q1.y * sc1 - hi1);
      }
    }
    a0.x += a0r;
    a0.y += a0i;
    a1.x += a1r;
    a1.y += a1i;
    mm += mmf;
    auto prod = [&](const U &xh, const U &xl, const U &yh, const U &yl, v4f acc) {
      acc = Op::mma(xh.v, yh.v, acc);
      if constexpr (SPLIT) {
        acc = Op::mma(xh.v, yl.v, acc);
        acc = Op::mma(xl.v, yh.v, acc);
      }
      return acc;
    };
    S00 = prod(r0h, r0l, r0h, r0l, S00);
    S00 = prod(i0h, i0l, i0h, i0l, S00);
    Q00 = prod(r0h, r0l, i0h, i0l, Q00);
    S01 = prod(r0h, r0l, r1h, r1l, S01);
    S01 = prod(i0h, i0l, i1h, i1l, S01);
    S11 = prod(r1h, r1l, r1h, r1l, S11);
    S11 = prod(i1h, i1l, i1h, i1l, S11);
    Q01 = prod(r0h, r0l, i1h, i1l, Q01);
    Q10 = prod(r1h, r1l, i0h, i0l, Q10);
    Q11 = prod(r1h, r1l, i1h, i1l, Q11);
    h0 = n0;
    h1 = n1;
    hmask = nmask;
  }

  for (int i = tid; i < 2 * D * D; i += 256) red[i] = 0.0;
  ared[wave][kq][f] = a0;
  ared[wave][kq][16 + f] = a1;
  if (f == 0) mmred[wave][kq] = mm;
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * kq + r, jj = f;  // 16x16 accumulator layout
        auto un = [&](int a, int b) { return 1.0 / ((double)fscale[w][a] * (double)fscale[w][b]); };
        red[i * D + jj] += (double)S00[r] * un(i, jj);
        red[D * D + i * D + jj] += (double)Q00[r] * un(i, jj);
        red[i * D + 16 + jj] += (double)S01[r] * un(i, 16 + jj);
        red[(16 + i) * D + 16 + jj] += (double)S11[r] * un(16 + i, 16 + jj);
        red[D * D + i * D + 16 + jj] += (double)Q01[r] * un(i, 16 + jj);
        red[D * D + (16 + i) * D + jj] += (double)Q10[r] * un(16 + i, jj);
        red[D * D + (16 + i) * D + 16 + jj] += (double)Q11[r] * un(16 + i, 16 + jj);
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


// FP16 storage form (n_t <= 32): the stack arrives split as H = m 1^T + R with m
// (complex64, one per pixel) and R stored as FP16(s R), s a power of two.  R^H R
// runs on v_mfma_f32_16x16x32_f16 straight from the stored halves (no conversion),
// unscaled by 1/s^2 exactly at the flush; the rank-one terms use m and R / s in
// FP32 over 8 pixels, then FP64.  Lane (f, kq) holds frames f and 16 + f of the 8
// pixels 8 kq .. 8 kq + 7 of each 32-pixel step (two 16-byte loads per frame).
__global__ __launch_bounds__(256) void gram_partial_r16(const h2 *__restrict__ R, const float2 *__restrict__ M,
                                                         int nt, long long npix, int pxw, float inv_s,
                                                         double *__restrict__ partial) {
  constexpr int D = 32;
  __shared__ double red[2 * D * D];
  __shared__ double2 ared[4][4][D];
  __shared__ double mmred[4][4];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int f = lane & 15, kq = lane >> 4;
  const long long p0 = ((long long)blockIdx.x * 4 + wave) * pxw;
  const bool v0 = f < nt, v1 = (16 + f) < nt;
  const uint4 *r0p = reinterpret_cast<const uint4 *>(R + (long long)(v0 ? f : 0) * npix + p0) + 2 * kq;
  const uint4 *r1p = reinterpret_cast<const uint4 *>(R + (long long)(v1 ? 16 + f : 0) * npix + p0) + 2 * kq;
  const float4 *mp = reinterpret_cast<const float4 *>(M + p0) + 4 * kq;
  union U8 {
    uint4 q[2];
    h2 h[8];
  };

  v4f S00 = {0.f, 0.f, 0.f, 0.f}, S01 = S00, S11 = S00, Q00 = S00, Q01 = S00, Q10 = S00, Q11 = S00;
  double2 a0 = make_double2(0.0, 0.0), a1 = a0;
  double mm = 0.0;
  const int STEPS = pxw / 32;
  for (int j = 0; j < STEPS; ++j) {
    const bool in = p0 + 32 * j + 8 * kq < npix;  // npix is a multiple of 8
    U8 x0, x1;
    float4 mq[4];
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      x0.q[g] = (v0 && in) ? r0p[8 * j + g] : make_uint4(0u, 0u, 0u, 0u);
      x1.q[g] = (v1 && in) ? r1p[8 * j + g] : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) mq[g] = in ? mp[16 * j + g] : make_float4(0.f, 0.f, 0.f, 0.f);
    v8h re0, im0, re1, im1;
    float a0r = 0.f, a0i = 0.f, a1r = 0.f, a1i = 0.f, mmf = 0.f;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      re0[e] = x0.h[e].x;
      im0[e] = x0.h[e].y;
      re1[e] = x1.h[e].x;
      im1[e] = x1.h[e].y;
      const float mr = (e & 1) ? mq[e >> 1].z : mq[e >> 1].x;
      const float mi = (e & 1) ? mq[e >> 1].w : mq[e >> 1].y;
      const float r0r = (float)x0.h[e].x * inv_s, r0i = (float)x0.h[e].y * inv_s;
      const float r1r = (float)x1.h[e].x * inv_s, r1i = (float)x1.h[e].y * inv_s;
      mmf += mr * mr + mi * mi;
      a0r += mr * r0r + mi * r0i;
      a0i += mr * r0i - mi * r0r;
      a1r += mr * r1r + mi * r1i;
      a1i += mr * r1i - mi * r1r;
    }
    a0.x += a0r;
    a0.y += a0i;
    a1.x += a1r;
    a1.y += a1i;
    mm += mmf;
    S00 = __builtin_amdgcn_mfma_f32_16x16x32_f16(re0, re0, S00, 0, 0, 0);
    S00 = __builtin_amdgcn_mfma_f32_16x16x32_f16(im0, im0, S00, 0, 0, 0);
    Q00 = __builtin_amdgcn_mfma_f32_16x16x32_f16(re0, im0, Q00, 0, 0, 0);
    S01 = __builtin_amdgcn_mfma_f32_16x16x32_f16(re0, re1, S01, 0, 0, 0);
    S01 = __builtin_amdgcn_mfma_f32_16x16x32_f16(im0, im1, S01, 0, 0, 0);
    S11 = __builtin_amdgcn_mfma_f32_16x16x32_f16(re1, re1, S11, 0, 0, 0);
    S11 = __builtin_amdgcn_mfma_f32_16x16x32_f16(im1, im1, S11, 0, 0, 0);
    Q01 = __builtin_amdgcn_mfma_f32_16x16x32_f16(re0, im1, Q01, 0, 0, 0);
    Q10 = __builtin_amdgcn_mfma_f32_16x16x32_f16(re1, im0, Q10, 0, 0, 0);
    Q11 = __builtin_amdgcn_mfma_f32_16x16x32_f16(re1, im1, Q11, 0, 0, 0);
  }

  const double un = (double)inv_s * (double)inv_s;
  for (int i = tid; i < 2 * D * D; i += 256) red[i] = 0.0;
  ared[wave][kq][f] = a0;
  ared[wave][kq][16 + f] = a1;
  if (f == 0) mmred[wave][kq] = mm;
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 4 * kq + r, jj = f;  // 16x16 accumulator layout
        red[i * D + jj] += (double)S00[r] * un;
        red[D * D + i * D + jj] += (double)Q00[r] * un;
        red[i * D + 16 + jj] += (double)S01[r] * un;
        red[(16 + i) * D + 16 + jj] += (double)S11[r] * un;
        red[D * D + i * D + 16 + jj] += (double)Q01[r] * un;
        red[D * D + (16 + i) * D + jj] += (double)Q10[r] * un;
        red[D * D + (16 + i) * D + 16 + jj] += (double)Q11[r] * un;
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


// The same exact Gram on integer MFMA (n_t <= 32).  Each 16-bit value is written
// with two signed 8-bit digits around the offset o = 32896 = 128 * 257:
//   x = 256 h + l + o,   h = (x >> 8) - 128,   l = (x & 255) - 128   (both in [-128, 127]),
// so that, summed over the pixels of a chunk (P of them),
//   sum x_s x_t = 2^16 (h^T h) + 2^8 (h^T l + l^T h) + (l^T l) + o (S_s + S_t) + P o^2,
// with S_s = sum (x_s - o).  Pixels past the end load as x = 0 and drop out of the
// identity exactly.  h^T h and l^T l (blocks a <= b) and h^T l (all blocks) run on
// v_mfma_i32_16x16x64_i8; every int32 sum stays below 2^31 (at most pxw products of
// magnitude <= 2^14 each), and the combination in FP64 is exact (integers below
// 2^53), so the result equals the FP64 kernel's bit for bit.  As bytes, l and h are
// the low and high bytes of x with the top bit flipped.  Lane (f, kq) holds frames
// f + 16 b of the 16 pixels 16 kq .. 16 kq + 15 of each 64-pixel step (two 16-byte
// loads per frame); the 32-bit 16x16 accumulator layout puts row 4 kq + r, column f
// in register r of lane (f, kq).
template <int NB>
__global__ __launch_bounds__(256) void gram_partial_u16_i8(const uint16_t *__restrict__ I, int nt, long long npix,
                                                            int pxw, double npix_d, double *__restrict__ partial) {
  static_assert(NB == 1 || NB == 2, "integer form for n_t <= 32");
  constexpr int D = 32;
  constexpr int NSYM = NB * (NB + 1) / 2, NCROSS = NB * NB;
  constexpr double kOff = 32896.0;
  __shared__ double red[D * D];
  __shared__ double ssum[D];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int f = lane & 15, kq = lane >> 4;
  const long long p0 = ((long long)blockIdx.x * 4 + wave) * pxw;
  const uint4 *src[NB];  // frame start (frame 0 for frames past nt)
  bool valid[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    valid[b] = 16 * b + f < nt;
    src[b] = reinterpret_cast<const uint4 *>(I + (long long)(valid[b] ? 16 * b + f : 0) * npix);
  }
  v4i hh[NSYM], ll[NSYM], hl[NCROSS];
#pragma unroll
  for (int q = 0; q < NSYM; ++q) hh[q] = ll[q] = v4i{0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < NCROSS; ++q) hl[q] = v4i{0, 0, 0, 0};
  int xsum[NB];  // sum of this lane's raw values per frame block
#pragma unroll
  for (int b = 0; b < NB; ++b) xsum[b] = 0;
  // Loads are unconditional (past the end they read the frame's first pixels; the
  // prefetch after the last step repeats that step) and masked when the step is
  // taken up, so the next step's loads stay in flight during the MFMAs; a step's
  // raw words sit in vector registers (8 dwords per frame block).
  typedef unsigned v8u __attribute__((ext_vector_type(8)));
  const int steps = pxw / 64;
  v8u cur[NB], nxt[NB];
  bool cin = p0 + 16 * kq < npix, nin = cin;  // npix is a multiple of 64
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const long long idx = cin ? (p0 + 16 * kq) / 8 : 0;
    const uint4 w0 = src[b][idx], w1 = src[b][idx + 1];
    cur[b] = v8u{w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
  }
  for (int j = 0; j < steps; ++j) {
    const int jn = j + 1 < steps ? j + 1 : j;
    nin = p0 + 64 * jn + 16 * kq < npix;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const long long idx = nin ? (p0 + 64 * jn + 16 * kq) / 8 : 0;
      const uint4 w0 = src[b][idx], w1 = src[b][idx + 1];
      nxt[b] = v8u{w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
    }
    v4i H[NB], L[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const bool ok = valid[b] && cin;
      unsigned u[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) u[e] = ok ? cur[b][e] : 0u;
      int h4[4], l4[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        // bytes of u[2q], u[2q+1]: lo0 hi0 lo1 hi1 | lo2 hi2 lo3 hi3, top bits flipped
        const unsigned a = u[2 * q] ^ 0x80808080u, c = u[2 * q + 1] ^ 0x80808080u;
        l4[q] = (int)__builtin_amdgcn_perm(c, a, 0x06040200u);  // lo0 lo1 lo2 lo3
        h4[q] = (int)__builtin_amdgcn_perm(c, a, 0x07050301u);  // hi0 hi1 hi2 hi3
        xsum[b] += (int)((u[2 * q] & 0xffffu) + (u[2 * q] >> 16) + (u[2 * q + 1] & 0xffffu) + (u[2 * q + 1] >> 16));
      }
      H[b] = v4i{h4[0], h4[1], h4[2], h4[3]};
      L[b] = v4i{l4[0], l4[1], l4[2], l4[3]};
    }
    int q = 0;
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = a; b < NB; ++b, ++q) {
        hh[q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(H[a], H[b], hh[q], 0, 0, 0);
        ll[q] = __builtin_amdgcn_mfma_i32_16x16x64_i8(L[a], L[b], ll[q], 0, 0, 0);
      }
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        hl[a * NB + b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(H[a], L[b], hl[a * NB + b], 0, 0, 0);
#pragma unroll
    for (int b = 0; b < NB; ++b) cur[b] = nxt[b];
    cin = nin;
  }
  // per-frame sums over the wave: the four lanes kq of frame f
  double fs[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    int v = xsum[b];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    fs[b] = (double)v;
  }
  // fixed-order combination of the four waves (exact: integer-valued doubles), then one store
  for (int i = tid; i < D * D; i += 256) red[i] = 0.0;
  if (tid < D) ssum[tid] = 0.0;
  __syncthreads();
#pragma unroll 1
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
      int q = 0;
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = a; b < NB; ++b, ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * a + 4 * kq + r, jj = 16 * b + f;
            const double v = 65536.0 * (double)hh[q][r] + (double)ll[q][r];
            red[i * D + jj] += v;
            if (a != b) red[jj * D + i] += v;
          }
      // h^T l counts at (i, j) and mirrored at (j, i): h^T l + l^T h
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * a + 4 * kq + r, jj = 16 * b + f;
            const double v = 256.0 * (double)hl[a * NB + b][r];
            red[i * D + jj] += v;
            red[jj * D + i] += v;
          }
      if (kq == 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b) ssum[16 * b + f] += fs[b];
      }
    }
    __syncthreads();
  }
  // + o (S_s + S_t) + P o^2 with S = (sum of x) - o P, P = the block's 4 pxw pixels
  const double P = 4.0 * (double)pxw;
  double *out = partial + (size_t)blockIdx.x * partial_len(D);
  for (int i = tid; i < partial_len(D); i += 256) {
    double v = 0.0;
    if (i < D * D) {
      const int s_ = i / D, t_ = i - (i / D) * D;
      const double Ss = ssum[s_] - kOff * P, St = ssum[t_] - kOff * P;
      v = (red[i] + kOff * (Ss + St) + P * kOff * kOff) * npix_d;
    }
    out[i] = v;
  }
}

// Exact covariance from the frames (n_t <= 64): because the input chirp has unit
// modulus and the unnormalised DFT satisfies F^H F = N_pix I, C = H^H H of Eq. (4)
// equals N_pix I^T I for the real interferogram matrix I, an integer Gram.  Its
// products (< 2^32) and sums (< 2^53 up to 2^21 pixels) are exact in FP64, so
// v_mfma_f64_16x16x4f64 computes it exactly; N_pix is a power of two.  Lane (f, kq)
// holds frames f + 16 b (b < NB) of the 8 pixels 8 kq .. 8 kq + 7 of each 32-pixel
// step (one 16-byte load per frame); MFMA step e takes pixel 8 kq + e of every kq.
// Only the blocks (a, b), a <= b, are accumulated; the rest follow by symmetry.
template <int NB>
__global__ __launch_bounds__(256) void gram_partial_u16(const uint16_t *__restrict__ I, int nt, long long npix,
                                                         int pxw, double npix_d, double *__restrict__ partial) {
  constexpr int D = NB <= 2 ? 32 : 64;
  constexpr int NBLK = NB * (NB + 1) / 2;
  __shared__ double red[D * D];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int f = lane & 15, kq = lane >> 4;
  const long long p0 = ((long long)blockIdx.x * 4 + wave) * pxw;
  const uint4 *src[NB];
  bool valid[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    valid[b] = 16 * b + f < nt;
    src[b] = reinterpret_cast<const uint4 *>(I + (long long)(valid[b] ? 16 * b + f : 0) * npix + p0) + kq;
  }
  v4d acc[NBLK];
#pragma unroll
  for (int q = 0; q < NBLK; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
  const int steps = pxw / 32;
  for (int j = 0; j < steps; ++j) {
    const bool in = p0 + 32 * j + 8 * kq < npix;  // npix is a multiple of 8
    union {
      uint4 q;
      unsigned short h[8];
    } x[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) x[b].q = (valid[b] && in) ? src[b][4 * j] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      double v[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) v[b] = (double)x[b].h[e];
      int q = 0;
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = a; b < NB; ++b, ++q) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[a], v[b], acc[q], 0, 0, 0);
    }
  }
  // fixed-order combination of the four waves (exact: integer-valued doubles), then one store
  for (int i = tid; i < D * D; i += 256) red[i] = 0.0;
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
      int q = 0;
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = a; b < NB; ++b, ++q)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            // FP64 16x16 accumulator layout: register r of lane (f, kq) holds row kq + 4 r, column f
            const int i = 16 * a + kq + 4 * r, jj = 16 * b + f;
            red[i * D + jj] += acc[q][r];
            if (a != b) red[jj * D + i] += acc[q][r];
          }
    }
    __syncthreads();
  }
  double *out = partial + (size_t)blockIdx.x * partial_len(D);
  for (int i = tid; i < partial_len(D); i += 256) out[i] = i < D * D ? red[i] * npix_d : 0.0;
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
#pragma unroll
  for (int g = 0; g < kGroups2; ++g) {  // all loads in flight at once
    if (g >= G2) break;
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

GramLayout gram_layout(int nt, long long npix, int pxw) {
  GramLayout L;
  L.nb = nt <= 32 ? 1 : 2;
  L.D = 32 * L.nb;
  L.pxw = pxw;
  L.chunks = (npix + pxw - 1) / pxw;  // one chunk per wave
  L.groups = (int)((L.chunks + 3) / 4);
  L.groups2 = L.groups < kGroups2 ? L.groups : kGroups2;
  L.partial_bytes = (size_t)L.groups * partial_len(L.D) * sizeof(double);
  L.partial2_bytes = (size_t)L.groups2 * partial_len(L.D) * sizeof(double);
  return L;
}

namespace {
hipError_t gram_tail(const GramLayout &L, int nt, double *partial, double *partial2, double *cov, hipStream_t s,
                     bool finalize);
}

hipError_t launch_gram_tail(const GramLayout &L, int nt, double *partial, double *partial2, double *cov,
                            hipStream_t s, bool finalize) {
  return gram_tail(L, nt, partial, partial2, cov, s, finalize);
}

hipError_t launch_gram(const GramLayout &L, const float2 *holo, int nt, long long npix, double *partial,
                       double *partial2, double *cov, hipStream_t s, int precision, bool finalize) {
  if (precision != HH_FP32 && nt <= 32) {
    ProfScope ps("gram_partial_lp", s);
    const dim3 g(L.groups), b(256);
    switch (precision) {
      case HH_BF16: hipLaunchKernelGGL((gram_partial_lp<kLpBF16, false>), g, b, 0, s, holo, nt, npix, L.pxw, partial); break;
      case HH_BF16X3: hipLaunchKernelGGL((gram_partial_lp<kLpBF16, true>), g, b, 0, s, holo, nt, npix, L.pxw, partial); break;
      case HH_FP16: hipLaunchKernelGGL((gram_partial_lp<kLpFP16, false>), g, b, 0, s, holo, nt, npix, L.pxw, partial); break;
      case HH_FP16X3: hipLaunchKernelGGL((gram_partial_lp<kLpFP16, true>), g, b, 0, s, holo, nt, npix, L.pxw, partial); break;
      default: hipLaunchKernelGGL((gram_partial_lp<kLpFP8, false>), g, b, 0, s, holo, nt, npix, L.pxw, partial); break;
    }
  } else {
    ProfScope ps("gram_partial", s);
    const dim3 g(L.groups), b(256);
    if (nt <= 16) {
      if (L.ref) hipLaunchKernelGGL((gram_partial16<false, false>), g, b, 0, s, holo, nt, npix, L.pxw, partial);
      else hipLaunchKernelGGL((gram_partial16<false, true>), g, b, 0, s, holo, nt, npix, L.pxw, partial);
    } else if (nt <= 32) {
      if (L.ref) hipLaunchKernelGGL((gram_partial16<true, false>), g, b, 0, s, holo, nt, npix, L.pxw, partial);
      else hipLaunchKernelGGL((gram_partial16<true, true>), g, b, 0, s, holo, nt, npix, L.pxw, partial);
    }
    else {
      if (L.ref) hipLaunchKernelGGL((gram_partial64<false>), dim3(L.groups), dim3(256), 0, s, holo, nt, npix, L.pxw, partial);
      else hipLaunchKernelGGL((gram_partial64<true>), dim3(L.groups), dim3(256), 0, s, holo, nt, npix, L.pxw, partial);
    }
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return gram_tail(L, nt, partial, partial2, cov, s, finalize);
}

hipError_t launch_gram_r16(const GramLayout &L, const h2 *r16, const float2 *m, int nt, long long npix, float inv_s,
                           double *partial, double *partial2, double *cov, hipStream_t s, bool finalize) {
  {
    ProfScope ps("gram_partial_r16", s);
    hipLaunchKernelGGL(gram_partial_r16, dim3(L.groups), dim3(256), 0, s, r16, m, nt, npix, L.pxw, inv_s, partial);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return gram_tail(L, nt, partial, partial2, cov, s, finalize);
}

hipError_t launch_gram_u16(const GramLayout &L, const uint16_t *frames, int nt, long long npix, double *partial,
                           double *partial2, double *cov, hipStream_t s, bool finalize) {
  {
    ProfScope ps("gram_partial_u16", s);
    const dim3 g(L.groups), b(256);
    const double nd = (double)npix;
    if (nt <= 16) hipLaunchKernelGGL(gram_partial_u16_i8<1>, g, b, 0, s, frames, nt, npix, L.pxw, nd, partial);
    else if (nt <= 32) hipLaunchKernelGGL(gram_partial_u16_i8<2>, g, b, 0, s, frames, nt, npix, L.pxw, nd, partial);
    else if (nt <= 48) hipLaunchKernelGGL(gram_partial_u16<3>, g, b, 0, s, frames, nt, npix, L.pxw, nd, partial);
    else hipLaunchKernelGGL(gram_partial_u16<4>, g, b, 0, s, frames, nt, npix, L.pxw, nd, partial);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return gram_tail(L, nt, partial, partial2, cov, s, finalize);
}

namespace {
// fixed-order reduction of the workgroup partials and Hermitian assembly
hipError_t gram_tail(const GramLayout &L, int nt, double *partial, double *partial2, double *cov, hipStream_t s,
                     bool finalize) {
  hipError_t e;
  const int Lw = partial_len(L.D);
  {
    ProfScope ps("gram_reduce", s);
    hipLaunchKernelGGL(gram_reduce, dim3((Lw + 255) / 256, L.groups2), dim3(256), 0, s, partial, L.groups, Lw,
                       L.groups2, partial2);
  }
  e = hipGetLastError();
  if (e != hipSuccess || !finalize) return e;
  {
    ProfScope ps("gram_finalize", s);
    hipLaunchKernelGGL(gram_finalize, dim3((nt * nt + 255) / 256), dim3(256), 0, s, partial2, L.groups2, L.D, nt,
                       reinterpret_cast<double2 *>(cov));
  }
  return hipGetLastError();
}
}  // namespace

}  // namespace hh
