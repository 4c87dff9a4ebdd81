// Internal declarations shared by the translation units of libfredec.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fredec.h"

namespace fredec {

constexpr int BLOCK = 256;               // threads per workgroup of every kernel
constexpr int MAXM = FREDEC_MAX_BASE;    // largest base model of a scan
constexpr int MAXK = 2 * MAXM + 1;       // base columns 1, cos, sin, ...
constexpr int MAXKP = MAXK + 1;          // base columns plus the data column
constexpr double MASK_WIDTH = 0.05;      // |f - f'| T_eff below this is masked
constexpr double PIVOT_TOL = 1e-13;      // relative Cholesky pivot threshold

// Per-series description built on the host and uploaded with each call.
struct SeriesIn {
  int64_t soff;     // first sample in the caller's arrays
  int64_t N;        // number of samples
  int64_t goff;     // first output element of this series
  int64_t F;        // grid size
  int64_t rec_off;  // first double of this series in the record array
  int64_t phi_off;  // first double of this series in the basis array
  double df;        // grid step: f_j = (j+1) df
  double rot_step;  // frequency step of the trig recurrence (tile stride * df)
  int32_t m;        // base frequencies
  int32_t KP;       // 2m + 2 columns: 1, cos f'_1, sin f'_1, ..., data
  double base_f[MAXM];
};

// Per-series quantities computed on the device by the preparation kernel.
struct SeriesHdr {
  double l_m;       // chi^2 minimum of the base model (normalised data)
  double NH;        // N - 3m - 4
  double T_eff;     // sqrt(4 pi Var(t))
  double D;         // <x~^2> (= 1 up to rounding)
  double stats[6];  // <t>, <x>, s_x, Var(t), T_eff, sum(w)
  int32_t status;   // 0 or a negative FREDEC_E* code
  int32_t pad;
  double inv_diag[MAXK];
  double a_b[MAXK];                 // L_A^{-1} g_b
  double L[MAXK * (MAXK + 1) / 2];  // Cholesky factor of the base normal matrix, packed rows
};

struct ScanWork {
  int32_t series;
  int32_t pad;
  int64_t j0;  // first grid index of the tile
};

__host__ __device__ constexpr int rec_stride(int KP) { return ((KP + 3) + 1) & ~1; }

// ------------------------------------------------------------ device math
// sin(2 pi y) and cos(2 pi y) for |y| <= 1/8 by their Taylor series in y:
// coefficients (-1)^k (2 pi)^(2k+1) / (2k+1)! and (-1)^k (2 pi)^(2k) / (2k)!,
// rounded to float64.  The first omitted terms are below 1e-19 (sin) and
// 3e-18 (cos) on |y| <= 1/8.
__device__ __forceinline__ void sincos_rev(double p, double& s, double& c) {
  // p is a phase in revolutions; reduce to p = n + q/4 + y, |y| <= 1/8.
  const double r = p - __builtin_rint(p);        // exact, |r| <= 1/2
  const double q = __builtin_rint(4.0 * r);      // -2..2
  const double y = __builtin_fma(-0.25, q, r);   // exact, |y| <= 1/8
  const double y2 = y * y;
  double sp = 0.10422916220813984;
  sp = __builtin_fma(sp, y2, -0.7181223017785006);
  sp = __builtin_fma(sp, y2, 3.819952584848282);
  sp = __builtin_fma(sp, y2, -15.09464257682299);
  sp = __builtin_fma(sp, y2, 42.058693944897655);
  sp = __builtin_fma(sp, y2, -76.70585975306139);
  sp = __builtin_fma(sp, y2, 81.60524927607506);
  sp = __builtin_fma(sp, y2, -41.34170224039976);
  sp = __builtin_fma(sp, y2, 6.283185307179586);
  sp = sp * y;
  double cp = 0.28200596845579123;
  cp = __builtin_fma(cp, y2, -1.714390711088672);
  cp = __builtin_fma(cp, y2, 7.903536371318469);
  cp = __builtin_fma(cp, y2, -26.4262567833744);
  cp = __builtin_fma(cp, y2, 60.24464137187666);
  cp = __builtin_fma(cp, y2, -85.45681720669373);
  cp = __builtin_fma(cp, y2, 64.9393940226683);
  cp = __builtin_fma(cp, y2, -19.739208802178716);
  cp = __builtin_fma(cp, y2, 1.0);
  // angle = q * pi/2 + 2 pi y: rotate by the quadrant
  const int iq = static_cast<int>(q) & 3;
  const double ss = (iq & 1) ? cp : sp;
  const double cc = (iq & 1) ? sp : cp;
  s = (iq & 2) ? -ss : ss;
  c = (iq == 1 || iq == 2) ? -cc : cc;
}

// Deterministic block-wide sum of NV values (fixed tree order).
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh) {
  const int tid = threadIdx.x;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) sh[k * BLOCK + tid] = v[k];
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if (tid < s) {
#pragma unroll
      for (int k = 0; k < NV; ++k) sh[k * BLOCK + tid] += sh[k * BLOCK + tid + s];
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = sh[k * BLOCK];
  __syncthreads();
}

// ------------------------------------------------------------ launchers
hipError_t launch_prep(hipStream_t st, int n_series, const SeriesIn* sin, SeriesHdr* hdr,
                       const double* t, const double* x, const double* w,
                       double* tau, double* xt, double* wt, double* rec, double* phi, int with_base);
hipError_t launch_scan_f64(hipStream_t st, int KP, int n_work, const ScanWork* work,
                           const SeriesIn* sin, const SeriesHdr* hdr, const double* rec,
                           double* z, uint8_t* flags);
hipError_t launch_scan_at_f64(hipStream_t st, int KP, const SeriesIn* sin, const SeriesHdr* hdr,
                              const double* rec, const int64_t* idx, int64_t n_idx,
                              double* z, uint8_t* flags);
hipError_t launch_copy_stats(hipStream_t st, int n_series, const SeriesHdr* hdr, const SeriesIn* sin,
                             double* l_base, int32_t* status, double* stats);
int scan_freqs_per_thread(int KP);  // R of the float64 scan kernel

}  // namespace fredec
