// Fourier demodulation, Eqs. (8)-(9), for a power-of-two n_t <= 64: the discrete Fourier
// transform of each pixel's n_t hologram samples along time, in registers, for one window or
// for several windows of a stream (window w takes frames w hop .. w hop + n_t - 1).
//
// One pixel per thread.  Its samples H[t][p] are frame-major, and consecutive threads
// take consecutive pixels, so every load of a wave reads 512 contiguous bytes and the
// n_t loads of a thread are all in flight at once.  A forward DFT along t (radix-2, in
// registers, no exchange between lanes) gives every bin X_f = sum_t H[t][p] W_nt^{t f};
// the image is (1/n_t) sum_{f=k_lo..k_hi} |X_f|^2, summed in FP64 — the projection onto
// the basis columns W[.][f] = exp(-2 i pi t f / n_t) / sqrt(n_t) of Eq. (8), at
// (n_t / 2) log2(n_t) butterflies per pixel instead of n_t multiply-adds per kept bin.
// A thread goes through the windows of a launch in turn, so the frames that consecutive
// windows share are read again while its pixels' lines are still in the L2 cache.
#include "fourier.h"

#include "fft_common.h"
#include "hh_internal.h"

namespace hh {
namespace {

template <int NT>
__global__ __launch_bounds__(256) void fourier_band(const float2 *__restrict__ H, long long npix, int nwin, int hop,
                                                    int k_lo, int k_hi, float *__restrict__ image) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= npix) return;
  for (int w = 0; w < nwin; ++w) {
    const float2 *Hw = H + (long long)w * hop * npix;
    float2 v[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) v[t] = Hw[(long long)t * npix + p];
    dft_reg<NT>(v);
    double s = 0.0;
#pragma unroll
    for (int f = 0; f < NT; ++f) {
      const float e = v[f].x * v[f].x + v[f].y * v[f].y;
      s += (f >= k_lo && f <= k_hi) ? (double)e : 0.0;
    }
    image[(long long)w * npix + p] = (float)(s * (1.0 / NT));
  }
}

template <int NT>
hipError_t launch_nt(const float2 *H, long long npix, int nwin, int hop, int k_lo, int k_hi, float *image,
                     hipStream_t s) {
  ProfScope ps("fourier_band", s);
  const long long blocks = (npix + 255) / 256;
  hipLaunchKernelGGL((fourier_band<NT>), dim3((unsigned)blocks), dim3(256), 0, s, H, npix, nwin, hop, k_lo, k_hi,
                     image);
  return hipGetLastError();
}

}  // namespace

bool fourier_band_supported(int nt) { return nt >= 2 && nt <= 64 && (nt & (nt - 1)) == 0; }

hipError_t launch_fourier_band(const float2 *holo, int nt, long long npix, int nwin, int hop, int k_lo, int k_hi,
                               float *image, hipStream_t s) {
  if (npix <= 0 || nwin < 1 || hop < 1 || k_lo < 0 || k_hi < k_lo || k_hi >= nt) return hipErrorInvalidValue;
  switch (nt) {
    case 2: return launch_nt<2>(holo, npix, nwin, hop, k_lo, k_hi, image, s);
    case 4: return launch_nt<4>(holo, npix, nwin, hop, k_lo, k_hi, image, s);
    case 8: return launch_nt<8>(holo, npix, nwin, hop, k_lo, k_hi, image, s);
    case 16: return launch_nt<16>(holo, npix, nwin, hop, k_lo, k_hi, image, s);
    case 32: return launch_nt<32>(holo, npix, nwin, hop, k_lo, k_hi, image, s);
    case 64: return launch_nt<64>(holo, npix, nwin, hop, k_lo, k_hi, image, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace hh
