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
constexpr double RHO_MIN = 0.6;          // reduced-precision scan: re-score in float64 below this
                                         // relative Schur pivot (trial columns nearly in the base span)
constexpr double LRATIO_MIN = 0.5;       // ... and where l_{m+1} / l_m falls below this (strong peaks,
                                         // where l_{m+1} = l_m - |a_psi|^2 cancels)

// Per-series description built on the host and uploaded with each call.
struct SeriesIn {
  int64_t soff;     // first sample in the caller's arrays
  int64_t N;        // number of samples
  int64_t goff;     // first output element of this series
  int64_t F;        // grid size
  int64_t rec_off;  // first double of this series in the float64 record array
  int64_t phi_off;  // first double of this series in the basis scratch array
  int64_t g32_off;  // first float of this series in the float32 operand array
  int64_t aux_off;  // first double of this series in the float32 kernel's aux array
  int64_t b16_off;  // first 8-half vector of this series in the split float16 operand array
  int64_t pt_off;   // first float2 of this series' phasor rows e^{2 pi i b df tau} (split float16 scan)
  double df;        // grid step: f_j = (j+1) df
  double rot_step;  // frequency step of the float64 kernel's recurrence (BLOCK * df)
  double rot_tile;  // frequency step of the MFMA kernel's recurrence (16 * df)
  int32_t m;        // base frequencies
  int32_t KP;       // 2m + 2 columns: orthonormal base columns q_0..q_{2m}, residual r_b
  int32_t NT;       // 16-column tiles of the MFMA operand (K = KP - 1 base columns)
  int32_t outputs;  // PREP_* operand sets the scan kernel of this series reads
  int64_t ptile0;   // first sample tile of this series in the preparation launch
  int64_t ppart_off;  // first double of its per-tile Gram partials (pntiles KP(KP+1)/2)
  int64_t pm_off;   // first double of its basis-change matrix (KP(KP+1)/2)
  int32_t prows;    // samples per preparation tile (prep_rows(KP))
  int32_t pntiles;  // preparation tiles, ceil(N / prows)
  double base_f[MAXM];
};

// Per-series quantities computed on the device by the preparation kernel.
struct SeriesHdr {
  double l_m;       // chi^2 minimum of the base model (normalised data)
  double NH;        // N - 3m - 4
  double T_eff;     // sqrt(4 pi Var(t))
  double D;         // <x~^2> (= 1 up to rounding)
  double W1;        // <1> = sum of the normalised weights (= 1 up to rounding)
  double stats[6];  // <t>, <x>, s_x, Var(t), T_eff, sum(w)
  double b16_inv;   // 1 / S, S the power-of-two scale of the split float16 operand
  double wmax;      // largest normalised weight
  int32_t status;   // 0 or a negative FREDEC_E* code
  int32_t pad;
};

struct ScanWork {
  int32_t series;
  int32_t pad;  // sample chunk of a split scan (0 otherwise)
  int64_t j0;  // first grid index of the tile
};

// A grid point of the reduced-precision scan to be re-scored in float64.
struct Rescore {
  int32_t series;
  int32_t pad;
  int64_t j;
};

// Outputs requested from the preparation kernel.
enum PrepFlags {
  PREP_BASE = 1,   // base-model precomputation (otherwise only the normalised series)
  PREP_REC64 = 2,  // float64 records (float64 scan, float32 VALU scan, re-scoring)
  PREP_G32 = 4,    // float32 column copy g32 (float32 VALU and MFMA scans)
  PREP_AUX = 8,    // aux records (float32 MFMA and split-float16 scans)
  PREP_F16 = 16    // split float16 operand b16
};

// float64 scan record per sample: tau, cos/sin(2 pi 256 df tau), the KP
// weighted columns, cos/sin(2 pi df tau); padded to an even count
__host__ __device__ constexpr int rec_stride(int KP) { return ((KP + 5) + 1) & ~1; }
constexpr int AUX_STRIDE = 8;  // doubles per sample of the MFMA kernel's aux record
__host__ __device__ constexpr int col_tiles(int KP) { return (KP - 1 + 15) / 16; }

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

// Table of e^{2 pi i k / 256}, k = 0..255 (cos, sin), for sincos_tab; filled
// by the threads of a block (one sincos_rev of an exact phase each).
constexpr int TRIG_TAB = 256;
__device__ __forceinline__ void trig_table_fill(double2* tab) {
  for (int k = threadIdx.x; k < TRIG_TAB; k += blockDim.x) {
    double s, c;
    sincos_rev(static_cast<double>(k) / TRIG_TAB, s, c);
    tab[k] = double2{c, s};
  }
}

// sin(2 pi p) and cos(2 pi p) from the table: p = n + k/256 + y with
// |y| <= 1/512 (both reductions exact), e^{2 pi i p} = T[k] e^{2 pi i y},
// e^{2 pi i y} by its Taylor series in y (coefficients (2 pi)^j / j!; the
// first omitted terms are below 2e-23 (sin) and 2e-20 (cos)).  About two
// thirds of the instructions of sincos_rev, and within a few float64 ulps.
__device__ __forceinline__ void sincos_tab(double p, const double2* __restrict__ tab, double& s, double& c) {
  const double r = p - __builtin_rint(p);                    // exact, |r| <= 1/2
  const double kf = __builtin_rint(static_cast<double>(TRIG_TAB) * r);  // -128..128
  const double y = __builtin_fma(-1.0 / TRIG_TAB, kf, r);    // exact, |y| <= 1/512
  const double y2 = y * y;
  double sp = __builtin_fma(y2, -76.70585975306139, 81.60524927607506);
  sp = __builtin_fma(sp, y2, -41.34170224039976);
  sp = __builtin_fma(sp, y2, 6.283185307179586);
  sp = sp * y;
  double cp = __builtin_fma(y2, -85.45681720669373, 64.9393940226683);
  cp = __builtin_fma(cp, y2, -19.739208802178716);
  cp = __builtin_fma(cp, y2, 1.0);
  const double2 t = tab[static_cast<int>(kf) & (TRIG_TAB - 1)];
  c = __builtin_fma(t.x, cp, -t.y * sp);
  s = __builtin_fma(t.y, cp, t.x * sp);
}

// Sum of v over aligned groups of L lanes (L = 4, 8, 16, 32 or 64), left in
// every lane of the group; a fixed sequence of exchanges, so the result is
// deterministic and identical in all lanes: DPP quad permutations (lane ^ 1,
// lane ^ 2), half-row and row mirrors (the other quad of an 8-lane half row,
// the other half of a 16-lane row), then swaps of 16 and 32 lanes.
template <int CTRL>
__device__ __forceinline__ double dpp_plus(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return v + __hiloint2double(__builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false),
                              __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false));
}

template <int L>
__device__ __forceinline__ double group_sum(double v) {
  static_assert(L == 4 || L == 8 || L == 16 || L == 32 || L == 64, "lane group of 4..64");
  v = dpp_plus<0xB1>(v);   // quad_perm [1,0,3,2]
  v = dpp_plus<0x4E>(v);   // quad_perm [2,3,0,1]
  if (L >= 8) v = dpp_plus<0x141>(v);  // row_half_mirror
  if (L >= 16) v = dpp_plus<0x140>(v);  // row_mirror
  if (L >= 32) v += __shfl_xor(v, 16);
  if (L >= 64) v += __shfl_xor(v, 32);
  return v;
}

// Final step of one scan frequency: 2x2 Cholesky of the Schur block
// S = [[Scc, Scs], [Scs, Sss]] (the extension of the base factor by the trial
// columns cos, sin - Sect. 3), a_psi = L_S^{-1} h, l_{m+1} = l_m - |a_psi|^2,
// z = (N - 3m - 4)/2 ln(l_m / l_{m+1}) (eq. zpowrel).  Flags as in fredec.h.
__device__ __forceinline__ void schur_finish(double Scc, double Scs, double Sss, double cc, double ss, double hc,
                                             double hs, double f, const SeriesIn& si, const SeriesHdr& h,
                                             double& z, uint8_t& flag, double* lratio = nullptr) {
  if (lratio) *lratio = 1.0;
  bool masked = false;
  for (int k = 0; k < si.m; ++k) masked |= fabs(f - si.base_f[k]) * h.T_eff < MASK_WIDTH;
  flag = 0;
  z = 0.0;
  if (masked) {
    flag = FREDEC_FLAG_MASKED;
    return;
  }
  bool ok = Scc > PIVOT_TOL * cc;
  const double l11 = sqrt(ok ? Scc : 1.0);
  const double l21 = Scs / l11;
  const double d2 = Sss - l21 * l21;
  ok = ok && (d2 > PIVOT_TOL * ss);
  if (!ok) {
    flag = FREDEC_FLAG_SINGULAR;
    return;
  }
  const double l22 = sqrt(d2);
  const double a1 = hc / l11;
  const double a2 = (hs - l21 * a1) / l22;
  const double l1 = h.l_m - (a1 * a1 + a2 * a2);
  if (lratio) *lratio = l1 / h.l_m;
  if (!(l1 > 0.0)) {
    flag = FREDEC_FLAG_PERFECT;
    z = __builtin_inf();
    return;
  }
  z = 0.5 * h.NH * log(h.l_m / l1);
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
// Samples per preparation tile of a series with KP columns: up to 256 rows
// of prep_rs(KP) + PREP_PSS doubles within PREP_TILE doubles of LDS, a
// multiple of 32.
constexpr int PREP_TILE = 5120;
constexpr int PREP_PSS = 9;
__host__ __device__ constexpr int prep_rs(int KP) { return KP | 1; }
__host__ __device__ constexpr int prep_rows(int KP) {
  return ((PREP_TILE / (prep_rs(KP) + PREP_PSS)) & ~31) < BLOCK ? ((PREP_TILE / (prep_rs(KP) + PREP_PSS)) & ~31)
                                                                  : BLOCK;
}
// Tile fields of a series for the preparation launch (host); advances the
// running tile, Gram-partial and matrix offsets.
inline void prep_assign(SeriesIn& d, int64_t& ptile, int64_t& ppart, int64_t& pm) {
  const int64_t kpp = static_cast<int64_t>(d.KP) * (d.KP + 1) / 2;
  d.prows = prep_rows(d.KP);
  d.pntiles = static_cast<int32_t>((d.N + d.prows - 1) / d.prows);
  d.ptile0 = ptile;
  d.ppart_off = ppart;
  d.pm_off = pm;
  ptile += d.pntiles;
  ppart += d.pntiles * kpp;
  pm += kpp;
}
// Normalisation and (flags & PREP_BASE) base-model precomputation of
// n_series series.  With PREP_BASE the series' SeriesIn carry the tile fields
// (ptile0, ppart_off, pm_off, prows, pntiles; n_tiles tiles in all) and the
// workspace arrays ppart (per-tile Gram partials) and pm (per-series basis
// change) are used; kp_max is the largest KP.
hipError_t launch_prep(hipStream_t st, int n_series, int kp_max, int64_t n_tiles, const SeriesIn* sin,
                       SeriesHdr* hdr, const double* t, const double* x, const double* w, double* tau, double* xt,
                       double* wt, double* rec, double* phi, float* g32, double* aux, void* b16, void* pt16,
                       double* ppart, double* pm, int flags);
// float64 re-scoring of the listed points (per-series lists at list[goff_s ..],
// count[s] entries each; off: 2 n_series + 3 int64 of workspace for the plan)
hipError_t launch_rescore(hipStream_t st, int NT, int grid, int n_series, const SeriesIn* sin, const SeriesHdr* hdr,
                          const double* rec, const Rescore* list, const unsigned long long* count, int64_t* off,
                          double* z, uint8_t* flags);
hipError_t launch_zero_u64(hipStream_t st, unsigned long long* p, int n);
// nsplit > 1: the work items cover sample chunks (ScanWork::pad = chunk) of
// one series of F_split grid points, whose sums go to part (nsplit (2 KP + 3)
// F_split doubles) and are then added in chunk order and finished.
hipError_t launch_scan_f64(hipStream_t st, int KP, int n_work, const ScanWork* work,
                           const SeriesIn* sin, const SeriesHdr* hdr, const double* rec,
                           double* z, uint8_t* flags, double* part = nullptr, int nsplit = 1,
                           int64_t F_split = 0);
// Sample chunks of a float64 scan of one series: fewer than 128 frequency
// tiles (wide fits on the chip) are split over up to 16 chunks of at least 256
// samples; 1 = no split.
int scan_f64_nsplit(int64_t N, int KP, int64_t F);
hipError_t launch_scan_at_f64(hipStream_t st, int KP, const SeriesIn* sin, const SeriesHdr* hdr,
                              const double* rec, const int64_t* idx, int64_t n_idx,
                              double* z, uint8_t* flags);
hipError_t launch_copy_stats(hipStream_t st, int n_series, const SeriesHdr* hdr, const SeriesIn* sin,
                             double* l_base, int32_t* status, double* stats);
int scan_freqs_per_thread(int KP);  // R of the float64 scan kernel
// Reduced-precision VALU scan (float32 sums, float64 phasors and data column);
// records as the float64 scan plus the float32 column copy g32.
hipError_t launch_scan_f32(hipStream_t st, int KP, int n_work, const ScanWork* work, const SeriesIn* sin,
                           const SeriesHdr* hdr, const double* rec, const float* g32, double* z, uint8_t* flags,
                           Rescore* list, unsigned long long* count);
int scan_f32_freqs_per_thread(int KP);  // R of the float32 VALU scan kernel
constexpr int F32_VALU_MAX_KP = 26;     // larger base models use the split-float16 MFMA form
constexpr int F32_AUTO_VALU_MAX_KP = 6;  // automatic form: VALU kernel for m <= 2, split float16 MFMA above
// Reduced-precision MFMA scan on split float16 operands (aux records and the
// preparation kernel's float16 operand array b16, 8-half vectors).
constexpr int f16x3_freq_tiles(int NT) { return NT <= 1 ? 4 : NT <= 2 ? 2 : 1; }  // default 16-frequency tiles per wave
// supported (column tiles, frequency tiles per wave): FT in {1, 2, 4} with NT FT <= 4
constexpr bool f16x3_tile_supported(int NT, int FT) {
  return NT >= 1 && NT <= 4 && (FT == 1 || FT == 2 || FT == 4) && NT * FT <= 4;
}
// nsplit > 1 (one series): the work items cover sample chunks (ScanWork::pad)
// and write raw sums to `part`; a reduction kernel over the F_split grid
// points adds them in chunk order and finishes the points.
hipError_t launch_scan_f16x3(hipStream_t st, int NT, int FT, int n_work, const ScanWork* work, const SeriesIn* sin,
                             const SeriesHdr* hdr, const double* aux, const void* b16, const void* pt16, double* z,
                             uint8_t* flags, Rescore* list, unsigned long long* count, double* part = nullptr,
                             int nsplit = 1, int64_t F_split = 0);
// Sample chunks of a split-float16 scan of one series: grids that give fewer
// than two workgroups per CU (512) at the default tile are split over up to 16
// chunks of at least 1024 samples; 1 = no split.  Partial sums per chunk and
// grid point: 4 doubles and 2 x 16 NT floats.
int scan_f16x3_nsplit(int64_t N, int NT, int64_t F);
__host__ __device__ constexpr int64_t f16x3_part_bytes(int nsplit, int NT, int64_t F) {
  return static_cast<int64_t>(nsplit) * F * (4 * 8 + 2 * 16 * NT * 4);
}
// 8-half vectors of the float16 operand of a series of N samples and NT column tiles:
// per step of 32 samples and column tile, a high and a low part of 64 lanes.
__host__ __device__ constexpr int64_t b16_vectors(int64_t N, int NT) { return (N + 31) / 32 * NT * 2 * 64; }
// Phasor rows of the split-float16 scan, written by the preparation: per tile
// of PT_TS samples, the 16 rows e^{2 pi i b df tau_s} (b < 16, float64 rounded
// to float32), each PT_TS consecutive float2, zero beyond N.  They depend on
// the series and the grid step only, so every workgroup of the scan copies
// them instead of computing them.
constexpr int PT_TS = 128;
__host__ __device__ constexpr int64_t pt16_float2(int64_t N) { return (N + PT_TS - 1) / PT_TS * 16 * PT_TS; }

}  // namespace fredec
