// Residual periodogram scan, reduced-precision VALU form (eq. zpowrel with
// n = 1, Sects. 3, 5).
//
// Same layout as the float64 scan: one lane owns R grid frequencies
// f_{j0+t+256r}, the per-sample records are uniform across the block and read
// as scalars.  The inner loop runs in float32 except for the data column:
//   phasor      the float32 complex product eat[s][a][r] * bt[s][b] of two
//               unit phasors computed in float64 by the block and rounded
//               once (the tables of build_phasor_tables32), so no rotation
//               chain accumulates rounding;
//   U_c[k], U_s[k] = <q_k cos>, <q_k sin>
//               float32 multiply-adds against a float32 copy of the weighted
//               columns w~ q_k, summed per tile of TS samples and the tile
//               sums added in float32 (they enter z only through U^T U in the
//               Schur block, where a relative error e moves z by about
//               2 e |U|^2 / S: small wherever the trial columns are not close
//               to the base span, and those points are re-scored);
//   <cos^2>, <cos sin>
//               float32 per tile, tile sums added in float64;
//   h = <r_b cos>, <r_b sin>
//               float64 multiply-adds of the float32 phasor (the data column
//               enters z linearly, and float32 accumulation of it costs
//               several 1e-7 in z at N = 10^4);
//   <sin^2> = <1> - <cos^2>.
// Non-packed float32 VALU instructions issue at twice the float64 rate when
// at least two waves per SIMD issue them, so R is chosen to keep the
// accumulators within about 128 VGPRs (four waves per SIMD).  Grid points
// where float32 loses accuracy - relative Schur pivot of the trial columns
// below RHO_MIN, or l_{m+1} / l_m below LRATIO_MIN - are listed and re-scored
// in float64 by rescore_kernel, as for the MFMA form.
#include "fredec_internal.h"
#include "scan_phasor.h"

namespace fredec {

namespace {

// Frequencies per lane: R (4 K + 10) accumulator registers (float32 tile and
// running sums of U, float32 tile sums of C, float64 C and h) within about
// 96 VGPRs, leaving room for the operands below 128.
constexpr int R32_of(int KP) {
  int r = 96 / (4 * KP + 6);
  return r < 1 ? 1 : (r > 8 ? 8 : r);
}

// Samples per phasor-table tile: 64 for R <= 2, else 32 (LDS of a block
// TS 16 (R + 1) 8 bytes <= 29 KB, four blocks per CU).
constexpr int TS32_of(int R) { return R <= 2 ? 64 : 32; }

template <int KP, int R>
__global__ __launch_bounds__(BLOCK) void scan_f32_kernel(const ScanWork* __restrict__ work,
                                                         const SeriesIn* __restrict__ sin_,
                                                         const SeriesHdr* __restrict__ hdr,
                                                         const double* __restrict__ rec,
                                                         const float* __restrict__ g32,
                                                         double* __restrict__ z_out, uint8_t* __restrict__ flags_out,
                                                         Rescore* __restrict__ list,
                                                         unsigned long long* __restrict__ count) {
  constexpr int K = KP - 1;
  constexpr int P = rec_stride(KP);
  constexpr int TS = TS32_of(R);
  const ScanWork wk = work[blockIdx.x];
  const SeriesIn& si = sin_[wk.series];
  const SeriesHdr& h = hdr[wk.series];
  const int64_t N = si.N;
  const int64_t F = si.F;
  const double df = si.df;
  const int GW = 16 * si.NT;  // floats per sample of the float32 column copy
  const int64_t jb = wk.j0 + threadIdx.x;
  double* zs = z_out + si.goff;
  uint8_t* fs = flags_out ? flags_out + si.goff : nullptr;
  if (h.status != 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t j = jb + (int64_t)BLOCK * r;
      if (j < F) {
        zs[j] = __builtin_nan("");
        if (fs) fs[j] = FREDEC_FLAG_BADSERIES;
      }
    }
    return;
  }
  float uc[R][K], us[R][K];  // tile sums of U
  float Uc[R][K], Us[R][K];  // running sums of the tile sums
  float cc32[R], cs32[R];    // tile sums of <cos^2>, <cos sin>
  double cc[R], cs[R], hc[R], hs[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int k = 0; k < K; ++k) uc[r][k] = us[r][k] = Uc[r][k] = Us[r][k] = 0.0f;
    cc32[r] = cs32[r] = 0.0f;
    cc[r] = cs[r] = hc[r] = hs[r] = 0.0;
  }

  __shared__ float2 eat[TS * 16 * R];
  __shared__ float2 bt[TS * 16];
  const int ta = threadIdx.x >> 4, tb = threadIdx.x & 15;
  // a zero in a VGPR that the compiler cannot fold: g[k] + zv is a copy of
  // the scalar g[k] into a vector register
  float zv;
  asm volatile("v_mov_b32 %0, 0" : "=v"(zv));
  const double fb = static_cast<double>(wk.j0 + 1) * df;
  const double* __restrict__ q0 = rec + si.rec_off;
  const float* __restrict__ g0 = g32 + si.g32_off;
  for (int64_t i0 = 0; i0 < N; i0 += TS) {
    const int nts = N - i0 < TS ? static_cast<int>(N - i0) : TS;
    __syncthreads();
    build_phasor_tables32<KP, R, TS>(q0 + i0 * P, P, nts, fb, eat, bt);
    __syncthreads();
    const double* __restrict__ q = q0 + i0 * P;
    const float* __restrict__ g = g0 + i0 * GW;
    // four samples per iteration: their scalar and LDS loads are issued
    // together, so one wait covers them
#pragma unroll 4
    for (int sl = 0; sl < nts; ++sl, q += P, g += GW) {
      const float2 bv = bt[sl * 16 + tb];
      const double gr = q[3 + K];  // w~ r_b
      // the sample's float32 columns (w~ q_k, then w~) copied into VGPRs:
      // one scalar-operand read per value instead of 2R
      float gv[K + 1];
#pragma unroll
      for (int k = 0; k <= K; ++k) gv[k] = g[k] + zv;
      const float wf = gv[K];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float2 e = eat[(sl * 16 + ta) * R + r];
        const float c = __builtin_fmaf(e.x, bv.x, -e.y * bv.y);
        const float s = __builtin_fmaf(e.y, bv.x, e.x * bv.y);
#pragma unroll
        for (int k = 0; k < K; ++k) {
          uc[r][k] = __builtin_fmaf(gv[k], c, uc[r][k]);
          us[r][k] = __builtin_fmaf(gv[k], s, us[r][k]);
        }
        const float wc = wf * c;
        cc32[r] = __builtin_fmaf(wc, c, cc32[r]);
        cs32[r] = __builtin_fmaf(wc, s, cs32[r]);
        hc[r] = __builtin_fma(gr, static_cast<double>(c), hc[r]);
        hs[r] = __builtin_fma(gr, static_cast<double>(s), hs[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        Uc[r][k] += uc[r][k];
        Us[r][k] += us[r][k];
        uc[r][k] = us[r][k] = 0.0f;
      }
      cc[r] += static_cast<double>(cc32[r]);
      cs[r] += static_cast<double>(cs32[r]);
      cc32[r] = cs32[r] = 0.0f;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t j = jb + (int64_t)BLOCK * r;
    if (j >= F) continue;
    const double ss = h.W1 - cc[r];
    double Scc = cc[r], Scs = cs[r], Sss = ss;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double u = static_cast<double>(Uc[r][k]), v = static_cast<double>(Us[r][k]);
      Scc = __builtin_fma(-u, u, Scc);
      Scs = __builtin_fma(-u, v, Scs);
      Sss = __builtin_fma(-v, v, Sss);
    }
    double z;
    uint8_t fl;
    double lratio;
    schur_finish(Scc, Scs, Sss, cc[r], ss, hc[r], hs[r], static_cast<double>(j + 1) * df, si, h, z, fl, &lratio);
    // relative pivots of the trial columns and the depth of the peak decide
    // whether the float32 sums are accurate enough (see the MFMA form)
    const double l21 = Scs / sqrt(fmax(Scc, 1e-300));
    const double rho = fmin(Scc / cc[r], (Sss - l21 * l21) / ss);
    if (!(fl & FREDEC_FLAG_MASKED) && (!(rho >= RHO_MIN) || !(lratio >= LRATIO_MIN))) {
      const unsigned long long slot = atomicAdd(count + wk.series, 1ull);
      list[si.goff + slot] = Rescore{wk.series, 0, j};
    }
    zs[j] = z;
    if (fs) fs[j] = fl;
  }
}

template <int KP>
hipError_t launch_kp32(hipStream_t st, int n_work, const ScanWork* work, const SeriesIn* sin, const SeriesHdr* hdr,
                       const double* rec, const float* g32, double* z, uint8_t* flags, Rescore* list,
                       unsigned long long* count) {
  scan_f32_kernel<KP, R32_of(KP)><<<n_work, BLOCK, 0, st>>>(work, sin, hdr, rec, g32, z, flags, list, count);
  return hipGetLastError();
}

}  // namespace

int scan_f32_freqs_per_thread(int KP) { return R32_of(KP); }

hipError_t launch_scan_f32(hipStream_t st, int KP, int n_work, const ScanWork* work, const SeriesIn* sin,
                           const SeriesHdr* hdr, const double* rec, const float* g32, double* z, uint8_t* flags,
                           Rescore* list, unsigned long long* count) {
  if (n_work <= 0) return hipSuccess;
  switch (KP) {
#define X(kp) \
  case kp: return launch_kp32<kp>(st, n_work, work, sin, hdr, rec, g32, z, flags, list, count);
    X(2) X(4) X(6) X(8) X(10) X(12) X(14) X(16) X(18) X(20) X(22) X(24) X(26)
#undef X
    default: return hipErrorInvalidValue;
  }
}

}  // namespace fredec
