// Internal declarations of the selection kernels (peaks, cascade).
#pragma once

#include "fredec_internal.h"

namespace fredec {

struct Peak {
  int64_t j;  // grid index
  double z;
};

struct CascadeParams {
  double zc[FREDEC_MAX_POOL + 1];  // zc[d]: threshold of a test between models differing by d frequencies
};

hipError_t launch_peaks(hipStream_t st, const double* z, const uint8_t* flags, int64_t F, double zmin, Peak* out,
                        unsigned long long* count, int64_t cap);
// Highest interior local maximum of z[0..F) by the peak rule of launch_peaks
// (largest z, then lowest index) into *out (j = -1 if there is none); part:
// peak_max_parts(F) partial results.
int64_t peak_max_parts(int64_t F);
hipError_t launch_peak_max(hipStream_t st, const double* z, const uint8_t* flags, int64_t F, Peak* part, Peak* out);
hipError_t launch_cascade(hipStream_t st, const double* ltab, int n, int64_t N, const CascadeParams& p, uint8_t* surv,
                          uint8_t* sup, uint8_t* maximal, double* G);

}  // namespace fredec
