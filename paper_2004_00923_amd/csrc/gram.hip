// Step (b), Eq. (4): C = H^{t*} H as a tall-skinny split-K Gram on FP32 MFMA.
//
// With H = A + iB (A, B real, one column per frame):
//   Re C = A^T A + B^T B,   Im C[s][t] = (A^T B)[s][t] - (A^T B)[t][s].
// Each workgroup stages 128-pixel x n_t tiles of H in LDS (coalesced loads) and
// feeds v_mfma_f32_32x32x2f32 with one frame per lane (32 lanes) and two pixels
// per instruction (the two half-waves).
//
// Accuracy: the stack is dominated by its temporal mean (the static speckle),
// so C is dominated by one eigenvalue while the components the image keeps sit
// ~1e-3 below it.  FP32 sums of raw products would leave errors of ~1e-8 of the
// top eigenvalue, enough to tilt the kept subspace when the boundary gap is
// small.  Each tile therefore splits H exactly as H = m 1^T + R, m the per-pixel
// temporal mean (any m works: R is formed as H - m), and
//   C = (m^H m) 1 1^T + 1 a^T + conj(a) 1^T + R^H R,   a_t = sum_p conj(m_p) R[p][t],
// with R^H R on MFMA (FP32 sums over at most 512 pixels) and the rank-one terms
// in FP64.  Partials are combined in FP64 in a fixed order (waves, then
// workgroups in two levels), so the result is deterministic.
#include "hh_internal.h"

namespace hh {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kLD = kGramChunk + 1;  // padded LDS row (complex): bank spread across frames

// Output of accumulator register r on lane l of a 32x32 MFMA block.
__device__ __forceinline__ int acc_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

// Length (doubles) of one workgroup partial: S, Q (D x D each), a (re, im), m^H m, pad.
__host__ __device__ constexpr int partial_len(int D) { return 2 * D * D + 2 * D + 2; }

template <int NB>
__global__ __launch_bounds__(256) void gram_partial(const float2 *__restrict__ H, int nt, long long npix,
                                                    long long nchunks, double *__restrict__ partial) {
  constexpr int D = 32 * NB;
  constexpr int NS = NB == 1 ? 1 : 3;  // S blocks: 00 | 00, 01, 11
  constexpr int NQ = NB * NB;          // Q blocks: all
  constexpr int PAIRS = kGramChunk / 2;           // float4 (2 pixels) per tile row
  constexpr int LOADS = D * PAIRS / 256;          // float4 per thread per tile
  __shared__ float2 tile[D * kLD];
  __shared__ float2 msum[2][kGramChunk];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int fr = lane & 31, half = lane >> 5;
  const float inv_nt = 1.0f / (float)nt;

  v16f S[NS], Q[NQ];
#pragma unroll
  for (int b = 0; b < NS; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) S[b][r] = 0.f;
#pragma unroll
  for (int b = 0; b < NQ; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) Q[b][r] = 0.f;
  double2 a_acc[LOADS];  // sum of conj(m_p) R[f][p] over this thread's (frame f, pixel) slots
#pragma unroll
  for (int l = 0; l < LOADS; ++l) a_acc[l] = make_double2(0.0, 0.0);
  double mm_acc = 0.0;   // sum of |m_p|^2 (threads 0..127, one pixel column each)

  const long long c0 = (long long)blockIdx.x * kGramChunksPerWG;
  const long long c1 = c0 + kGramChunksPerWG < nchunks ? c0 + kGramChunksPerWG : nchunks;
  const float4 *H4 = reinterpret_cast<const float4 *>(H);
  const long long npix2 = npix / 2;

  for (long long c = c0; c < c1; ++c) {
    float4 buf[LOADS];
#pragma unroll
    for (int l = 0; l < LOADS; ++l) {
      const int f4 = tid + 256 * l;
      const int frame = f4 / PAIRS, pr = f4 % PAIRS;
      const long long pp = c * PAIRS + pr;  // pixel-pair index
      buf[l] = (frame < nt && pp < npix2) ? H4[(long long)frame * npix2 + pp] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();  // previous tile fully consumed
#pragma unroll
    for (int l = 0; l < LOADS; ++l) {
      const int f4 = tid + 256 * l;
      const int frame = f4 / PAIRS, pr = f4 % PAIRS;
      tile[frame * kLD + 2 * pr] = make_float2(buf[l].x, buf[l].y);
      tile[frame * kLD + 2 * pr + 1] = make_float2(buf[l].z, buf[l].w);
    }
    __syncthreads();
    {  // per-pixel frame sums, two interleaved halves per pixel
      const int px = tid & (kGramChunk - 1), h = tid >> 7;
      float2 sm = make_float2(0.f, 0.f);
      for (int t = h; t < nt; t += 2) {
        const float2 v = tile[t * kLD + px];
        sm.x += v.x;
        sm.y += v.y;
      }
      msum[h][px] = sm;
    }
    __syncthreads();
    // R = H - m on this thread's own slots; a_t += conj(m) R in FP64
#pragma unroll
    for (int l = 0; l < LOADS; ++l) {
      const int f4 = tid + 256 * l;
      const int frame = f4 / PAIRS, pr = f4 % PAIRS;
      if (frame < nt) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int px = 2 * pr + e;
          const float2 m = make_float2((msum[0][px].x + msum[1][px].x) * inv_nt,
                                       (msum[0][px].y + msum[1][px].y) * inv_nt);
          float2 r = tile[frame * kLD + px];
          r.x -= m.x;
          r.y -= m.y;
          tile[frame * kLD + px] = r;
          const double mr = m.x, mi = m.y, rr = r.x, ri = r.y;
          a_acc[l].x += mr * rr + mi * ri;
          a_acc[l].y += mr * ri - mi * rr;
        }
      }
    }
    if (tid < kGramChunk) {
      const double mr = (double)((msum[0][tid].x + msum[1][tid].x) * inv_nt);
      const double mi = (double)((msum[0][tid].y + msum[1][tid].y) * inv_nt);
      mm_acc += mr * mr + mi * mi;
    }
    __syncthreads();
    // wave w owns pixels [32w, 32w+32) of the tile: 16 MFMA steps of 2 pixels
#pragma unroll 4
    for (int st = 0; st < 16; ++st) {
      const int px = 32 * wave + 2 * st + half;
      const float2 x0 = tile[fr * kLD + px];
      if constexpr (NB == 1) {
        S[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.x, x0.x, S[0], 0, 0, 0);
        S[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.y, x0.y, S[0], 0, 0, 0);
        Q[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.x, x0.y, Q[0], 0, 0, 0);
      } else {
        const float2 x1 = tile[(32 + fr) * kLD + px];
        S[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.x, x0.x, S[0], 0, 0, 0);
        S[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.y, x0.y, S[0], 0, 0, 0);
        S[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.x, x1.x, S[1], 0, 0, 0);
        S[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.y, x1.y, S[1], 0, 0, 0);
        S[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.x, x1.x, S[2], 0, 0, 0);
        S[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.y, x1.y, S[2], 0, 0, 0);
        Q[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.x, x0.y, Q[0], 0, 0, 0);
        Q[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(x0.x, x1.y, Q[1], 0, 0, 0);
        Q[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.x, x0.y, Q[2], 0, 0, 0);
        Q[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(x1.x, x1.y, Q[3], 0, 0, 0);
      }
    }
  }

  // Fixed-order FP64 combination of the four waves in LDS, then one store.
  __syncthreads();
  double *acc = reinterpret_cast<double *>(tile);  // [2][D][D] doubles (fits in the tile)
  for (int i = tid; i < 2 * D * D; i += 256) acc[i] = 0.0;
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int b = 0; b < NS; ++b) {
        const int bi = (NB == 1) ? 0 : (b == 2 ? 1 : 0);
        const int bj = (NB == 1) ? 0 : (b == 0 ? 0 : 1);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = 32 * bi + acc_row(lane, r), j = 32 * bj + fr;
          acc[i * D + j] += (double)S[b][r];
        }
      }
#pragma unroll
      for (int b = 0; b < NQ; ++b) {
        const int bi = b / NB, bj = b % NB;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int i = 32 * bi + acc_row(lane, r), j = 32 * bj + fr;
          acc[D * D + i * D + j] += (double)Q[b][r];
        }
      }
    }
    __syncthreads();
  }
  double *out = partial + (size_t)blockIdx.x * partial_len(D);
  for (int i = tid; i < 2 * D * D; i += 256) out[i] = acc[i];
  __syncthreads();
  // rank-one terms: thread slots -> per-frame a_t (fixed order over the 64 owners), and m^H m
  double2 *aslot = reinterpret_cast<double2 *>(tile);  // [LOADS][256]
#pragma unroll
  for (int l = 0; l < LOADS; ++l) aslot[l * 256 + tid] = a_acc[l];
  double *mmslot = reinterpret_cast<double *>(&msum[0][0]);  // [128] (msum is free now)
  if (tid < kGramChunk) mmslot[tid] = mm_acc;
  __syncthreads();
  if (tid < D) {
    // frame f lives in slot l = f / 4 of threads 64 (f % 4) ... 64 (f % 4) + 63
    const int l = tid / 4, t0 = 64 * (tid % 4);
    double ar = 0.0, ai = 0.0;
    for (int k = 0; k < 64; ++k) {
      const double2 v = aslot[l * 256 + t0 + k];
      ar += v.x;
      ai += v.y;
    }
    out[2 * D * D + tid] = ar;
    out[2 * D * D + D + tid] = ai;
  }
  if (tid == 0) {
    double s = 0.0;
    for (int k = 0; k < kGramChunk; ++k) s += mmslot[k];
    out[2 * D * D + 2 * D] = s;
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
  for (int g = g0; g < g1; ++g) s += in[(size_t)g * L + l];
  out[(size_t)g2 * L + l] = s;
}

// Assemble the Hermitian C = (m^H m) 1 1^T + 1 a^T + conj(a) 1^T + R^H R from the
// summed partials (S = Re R^H R upper blocks, Q = A^T B of R = A + iB).
__global__ __launch_bounds__(256) void gram_finalize(const double *__restrict__ in2, int G2, int D, int nt,
                                                     double2 *__restrict__ cov) {
  const size_t L = partial_len(D);
  for (int e = threadIdx.x; e < nt * nt; e += 256) {
    const int s = e / nt, t = e % nt;
    const int lo = s < t ? s : t, hi = s < t ? t : s;
    double re = 0.0, qst = 0.0, qts = 0.0, mm = 0.0, alo = 0.0, ahi = 0.0, ais = 0.0, ait = 0.0;
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
}

}  // namespace

GramLayout gram_layout(int nt, long long npix) {
  GramLayout L;
  L.nb = nt <= 32 ? 1 : 2;
  L.D = 32 * L.nb;
  L.chunks = (npix + kGramChunk - 1) / kGramChunk;
  L.groups = (int)((L.chunks + kGramChunksPerWG - 1) / kGramChunksPerWG);
  L.groups2 = L.groups < 16 ? L.groups : 16;
  L.partial_bytes = (size_t)L.groups * partial_len(L.D) * sizeof(double);
  L.partial2_bytes = (size_t)L.groups2 * partial_len(L.D) * sizeof(double);
  return L;
}

hipError_t launch_gram(const GramLayout &L, const float2 *holo, int nt, long long npix, double *partial,
                       double *partial2, double *cov, hipStream_t s) {
  {
    ProfScope ps("gram_partial", s);
    if (L.nb == 1)
      hipLaunchKernelGGL(gram_partial<1>, dim3(L.groups), dim3(256), 0, s, holo, nt, npix, L.chunks, partial);
    else
      hipLaunchKernelGGL(gram_partial<2>, dim3(L.groups), dim3(256), 0, s, holo, nt, npix, L.chunks, partial);
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
    hipLaunchKernelGGL(gram_finalize, dim3(1), dim3(256), 0, s, partial2, L.groups2, L.D, nt,
                       reinterpret_cast<double2 *>(cov));
  }
  return hipGetLastError();
}

}  // namespace hh
