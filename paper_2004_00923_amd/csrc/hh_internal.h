// Internal declarations shared by the HIP translation units of libhh.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/hh.h"

namespace hh {

// Device tables for one optical/shape configuration (owned by the plan cache).
struct Plan {
  int device = -1;
  int nx = 0, ny = 0;
  float2 *chirp_x = nullptr;  // [nx]  exp(-i alpha (m - nx/2)^2)
  float2 *chirp_y = nullptr;  // [ny]  exp(-i alpha (n - ny/2)^2)
  float2 *tw_x = nullptr;     // [nx]  exp(-2 pi i j / nx)
  float2 *tw_y = nullptr;     // [ny]  exp(-2 pi i j / ny)
  int cus = 256;              // compute units of the device (sizes persistent grids)
};

// Returns nullptr and sets the error text on failure.
const Plan *get_plan(const hh_params &p);
// Unitary DFT basis W[t][f] (complex128, nt x nt) on the current device, cached.
const double *get_dft_basis(int nt);

void set_error(const char *fmt, ...);

// Kernel launch bracket used by the optional profiler.
struct ProfScope {
  const char *name;
  hipStream_t stream;
  void *ev0 = nullptr;
  ProfScope(const char *n, hipStream_t s);
  ~ProfScope();
};

// ---- launchers (each returns hipSuccess or the launch error) ----

struct Tune;
// Step (a): row pass (uint16 -> chirp -> row FFT) then in-place column FFT.
hipError_t launch_fresnel(const Plan &pl, const Tune &tu, const uint16_t *frames, int nframes, float2 *holo,
                          hipStream_t s);
// FP16 storage form of step (a): mean[p] = temporal mean of the frames (float),
// m = Fresnel(mean) (complex64), r16[t] = FP16(scale * Fresnel(frame_t - mean)).
// group_buf holds fresnel_group_frames(nx, ny, nframes, tu.group) FP32 frames.
typedef _Float16 h2 __attribute__((ext_vector_type(2)));
int fresnel_group_frames(int nx, int ny, int nframes, int tuned);
hipError_t launch_fresnel_r16(const Plan &pl, const Tune &tu, const uint16_t *frames, int nframes, float *mean,
                              float2 *m, float2 *group_buf, h2 *r16, float scale, hipStream_t s);

// Step (b): split-K Gram partials, fixed-order reduction, Hermitian assembly.
// Length (doubles) of one covariance partial: S, Q (D x D each), a (re, im), m^H m, pad.
// C[s][t] = S[min][max] + m^H m + a[s] + a[t] + i (Q[s][t] - Q[t][s] + a'[t] - a'[s]),
// a = re part, a' = im part of the rank-one vector.
__host__ __device__ constexpr int partial_len(int D) { return 2 * D * D + 2 * D + 2; }

struct GramLayout {
  int nb = 1;              // 32-frame blocks (1 or 2)
  int D = 32;              // 32 * nb
  int pxw = 256;           // pixels per wave (split-K chunk); FP32 sums of <= 2 pxw products
  int ref = 0;             // FP32 form, n_t <= 32: reference of the split, 0 = temporal mean, 1 = frame 0
  long long chunks = 0;    // pixel chunks of pxw pixels (one per wave)
  int groups = 0;          // workgroups of the partial kernel
  int groups2 = 0;         // second-level partial count
  size_t partial_bytes = 0, partial2_bytes = 0;
};
// Tuned launch choices for one problem shape (see the autotuner in hh_api.hip).
struct Tune {
  int rows = 0;      // row-FFT launch shape (0..3)
  int cols = 0;      // column-FFT launch shape (0..2)
  int pxw = 256;     // Gram pixels per wave: 256, 512 or 1024
  int group = 0;     // frames per Fresnel group, 0 = about 64 MiB of holograms
  int gram_ref = 0;  // reference of the covariance's mean split (FP32 form): 0 temporal mean, 1 frame 0
  int fused = 0;     // FP32 pipeline: 1 = the three-pass form (fresnel_pca.hip) where the shape allows it
};
constexpr int kGramPxwMin = 256;  // the workspace is sized for the smallest split-K chunk
GramLayout gram_layout(int nt, long long npix, int pxw = kGramPxwMin);
// precision: HH_FP32, or a low-precision form of the R^H R contraction (n_t <= 32;
// larger stacks use the FP32 form).
// finalize = false: stop after the second-level partials (the eigensolver assembles C).
hipError_t launch_gram(const GramLayout &L, const float2 *holo, int nt, long long npix,
                       double *partial, double *partial2, double *cov, hipStream_t s, int precision = HH_FP32,
                       bool finalize = true);
// Second half of launch_gram: fixed-order reduction of L.groups partials into
// L.groups2, then (finalize) the Hermitian assembly into cov.
hipError_t launch_gram_tail(const GramLayout &L, int nt, double *partial, double *partial2, double *cov,
                            hipStream_t s, bool finalize);
// Exact covariance from the frames, C = N_pix I^T I (n_t <= 64; frames 16-byte aligned).
hipError_t launch_gram_u16(const GramLayout &L, const uint16_t *frames, int nt, long long npix, double *partial,
                           double *partial2, double *cov, hipStream_t s, bool finalize = true);
// FP16 storage form: H = m 1^T + r16 / s with inv_s = 1 / s (n_t <= 32).
hipError_t launch_gram_r16(const GramLayout &L, const h2 *r16, const float2 *m, int nt, long long npix, float inv_s,
                           double *partial, double *partial2, double *cov, hipStream_t s, bool finalize = true);

// Steps (a)-(e) of the FP32 form in three passes (fresnel_pca.hip): the column
// transform with a radix-4 split of the rows into tbuf (complex64, the size of
// the holograms), then the quarter-row transforms with the covariance partials
// (*groups partials, at most max_groups); after the eigensolver, the same
// transforms with the projection and |.|^2.  Shapes: fused_supported.
bool fused_supported(int nx, int ny, int nt);
hipError_t launch_fused_front(const Plan &pl, const uint16_t *frames, int nt, float2 *tbuf, int max_groups,
                              double *partial, int *groups, hipStream_t s);
hipError_t launch_fused_back(const Plan &pl, const float2 *tbuf, int nt, const double *V, int k_lo, int k_hi,
                             int mode, float *image, hipStream_t s);

// Step (c): one workgroup per problem; problems are passed by value (kernel argument).
// One eigenproblem.  Either cov holds C (complex128 [n][n]), or part2 holds the
// covariance's second-level partial sums (g2 partials of the D-wide layout), in
// which case the solver assembles C itself and also stores it to cov.
struct EighProblem {
  int n;
  const double *cov;
  double *evals;
  double *evecs;
  int *info;
  const double *part2 = nullptr;
  int g2 = 0, D = 0;
  int method = HH_EIGH_JACOBI;  // HH_EIGH_JACOBI or HH_EIGH_TRIDIAG
};
constexpr int kMaxEighBatch = 64;
struct EighBatch {
  EighProblem prob[kMaxEighBatch];
};
hipError_t launch_eigh(int nt, const double *cov, double *evals, double *evecs, int *info,
                       int max_sweeps, hipStream_t s);
// max_iter: Jacobi sweeps, or QL iterations per eigenvalue
hipError_t launch_eigh_batch(const EighProblem *probs, int count, int max_iter, hipStream_t s);

// Steps (d)+(e)
// precision: HH_FP32 (and the forms that store H differently) project in FP32/FP64;
// the forms HH_BF16 .. HH_FP8E4M3 (nt <= 32) project the kept components on MFMA in
// their operand format unless mode is HH_PROJ_COMPLEMENT.
hipError_t launch_project(const float2 *holo, int nt, long long npix, const double *V, int k_lo,
                          int k_hi, int mode, float *image, hipStream_t s, int precision = HH_FP32);
// FP16 storage form of steps (d)+(e): H = m + r16 * inv_s
hipError_t launch_project_r16(const h2 *r16, const float2 *m, float inv_s, int nt, long long npix, const double *V,
                              int k_lo, int k_hi, int mode, float *image, hipStream_t s);
// Projection-first image from the frames (needs the plan's tables): inter holds
// K = k_hi - k_lo + 1 row-transformed components (complex64 [K][ny][nx]), eparts
// kMaxEnergyChunks partial images (float [chunks][ny][nx]).  real_v: read Re V only.
constexpr int kMaxEnergyChunks = 8;
int project_frames_chunks(int nx, int ny, int K, int cus);
hipError_t launch_project_frames(const Plan &pl, const uint16_t *frames, int nt, const double *V, int k_lo, int k_hi,
                                 bool real_v, float2 *inter, float *eparts, float *image, hipStream_t s);
// SVD-filtered stack, Eq. (3)
hipError_t launch_svd_filter(const float2 *holo, int nt, long long npix, const double *V, int k_lo, int k_hi,
                             int mode, float2 *out, hipStream_t s);

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

}  // namespace hh
