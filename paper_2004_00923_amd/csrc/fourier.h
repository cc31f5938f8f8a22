// Fourier demodulation by a per-pixel FFT along time (Eqs. (8)-(9)).
#pragma once

#include <hip/hip_runtime.h>

namespace hh {

// True for the n_t that launch_fourier_band takes: powers of two from 2 to 64.
bool fourier_band_supported(int nt);

// For the windows w = 0 .. nwin-1 of frames H[w hop + t], t < nt:
// image[w][p] = sum_{f=k_lo..k_hi} |sum_t H[w hop + t][p] W[t][f]|^2,
// W[t][f] = exp(-2 i pi t f / nt) / sqrt(nt); H complex64 [(nwin - 1) hop + nt][npix]
// (16-byte aligned), image float32 [nwin][npix]; 0 <= k_lo <= k_hi < nt, nwin, hop >= 1.
// hipErrorInvalidValue for an nt it does not take.
hipError_t launch_fourier_band(const float2 *holo, int nt, long long npix, int nwin, int hop, int k_lo, int k_hi,
                               float *image, hipStream_t s);

}  // namespace hh
