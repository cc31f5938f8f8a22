// Step (b), Eq. (4): C = H^{t*} H as a tall-skinny split-K Gram on FP32 MFMA.
//
// With H = A + iB (A, B real, one column per frame):
//   Re C = A^T A + B^T B,   Im C[s][t] = (A^T B)[s][t] - (A^T B)[t][s].
// Each workgroup stages 128-pixel x n_t tiles of H in LDS (coalesced loads) and
// feeds v_mfma_f32_32x32x2f32 with one frame per lane (32 lanes) and two pixels
// per instruction (the two half-waves).  FP32 sums cover at most 512 pixels;
// they are then converted to FP64 and combined in a fixed order (waves, then
// workgroups in two levels), so the result is deterministic.
#include "hh_internal.h"

namespace hh {
namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kLD = kGramChunk + 1;  // padded LDS row (complex): bank spread across frames

// Output of accumulator register r on lane l of a 32x32 MFMA block.
__device__ __forceinline__ int acc_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

template <int NB>
__global__ __launch_bounds__(256) void gram_partial(const float2 *__restrict__ H, int nt, long long npix,
                                                    long long nchunks, double *__restrict__ partial) {
  constexpr int D = 32 * NB;
  constexpr int NS = NB == 1 ? 1 : 3;  // S blocks: 00 | 00, 01, 11
  constexpr int NQ = NB * NB;          // Q blocks: all
  __shared__ float2 tile[D * kLD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int fr = lane & 31, half = lane >> 5;

  v16f S[NS], Q[NQ];
#pragma unroll
  for (int b = 0; b < NS; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) S[b][r] = 0.f;
#pragma unroll
  for (int b = 0; b < NQ; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) Q[b][r] = 0.f;

  const long long c0 = (long long)blockIdx.x * kGramChunksPerWG;
  const long long c1 = c0 + kGramChunksPerWG < nchunks ? c0 + kGramChunksPerWG : nchunks;
  constexpr int PAIRS = kGramChunk / 2;           // float4 (2 pixels) per tile row
  constexpr int LOADS = D * PAIRS / 256;          // float4 per thread per tile
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
  double *out = partial + (size_t)blockIdx.x * 2 * D * D;
  for (int i = tid; i < 2 * D * D; i += 256) out[i] = acc[i];
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

// Assemble the Hermitian C from the summed S (= A^T A + B^T B, upper blocks) and Q (= A^T B).
__global__ __launch_bounds__(256) void gram_finalize(const double *__restrict__ in2, int G2, int D, int nt,
                                                     double2 *__restrict__ cov) {
  const size_t L = 2 * (size_t)D * D;
  for (int e = threadIdx.x; e < nt * nt; e += 256) {
    const int s = e / nt, t = e % nt;
    const int lo = s < t ? s : t, hi = s < t ? t : s;
    double re = 0.0, qst = 0.0, qts = 0.0;
    for (int g = 0; g < G2; ++g) {
      const double *p = in2 + g * L;
      re += p[lo * D + hi];
      qst += p[(size_t)D * D + s * D + t];
      qts += p[(size_t)D * D + t * D + s];
    }
    cov[e] = make_double2(re, qst - qts);
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
  L.partial_bytes = (size_t)L.groups * 2 * L.D * L.D * sizeof(double);
  L.partial2_bytes = (size_t)L.groups2 * 2 * L.D * L.D * sizeof(double);
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
  const int Lw = 2 * L.D * L.D;
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
