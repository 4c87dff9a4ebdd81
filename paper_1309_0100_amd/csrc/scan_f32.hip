// Residual periodogram scan, reduced-precision VALU form (eq. zpowrel with
// n = 1, Sects. 3, 5).
//
// Same layout as the float64 scan: one lane owns R grid frequencies
// f_{j0+t+256r}, the per-sample records are uniform across the block and read
// as scalars, and the phasor of the lane's first frequency is E0 A_a B_b from
// the block's LDS tables (float64), rotated in float64 to the other R-1.
// The arithmetic per (frequency, sample) pair differs:
//   cos, sin                 rounded to float32 after the float64 phasor;
//   U_c[k], U_s[k] = <q_k cos>, <q_k sin>, and <cos^2>, <cos sin>
//                            float32 multiply-adds against float32 copies of
//                            the weighted columns (w~ q_k, w~), added into
//                            float64 totals at the end of every 64-sample tile;
//   h = <r_b cos>, <r_b sin> float64 (the data column enters z linearly);
//   <sin^2> = <1> - <cos^2>.
// On this GPU a float32 VALU multiply-add costs half a float64 one and runs
// at the float32 matrix-core rate (which it does not overlap), so the 2K + 2
// float32 sums cost what K + 1 float64 ones do.  Grid points where float32
// loses accuracy - relative Schur pivot of the trial columns below RHO_MIN,
// or l_{m+1} / l_m below LRATIO_MIN - are listed and re-scored in float64 by
// rescore_kernel, exactly as for the MFMA form.
#include "fredec_internal.h"
#include "scan_phasor.h"

namespace fredec {

namespace {

// Frequencies per lane: R (6 KP + 4) accumulator registers (float32 sums,
// their float64 totals, the float64 data column) within about 128 VGPRs.
constexpr int R32_of(int KP) {
  int r = 128 / (6 * KP + 4);
  return r < 1 ? 1 : (r > 8 ? 8 : r);
}

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
  // float32 tile sums: U_c[k], U_s[k] (k < K), <cos^2>, <cos sin>
  float uc[R][K], us[R][K], cc32[R], cs32[R];
  // float64 totals and the float64 data column
  double Uc[R][K], Us[R][K], cc[R], cs[R], hc[R], hs[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      uc[r][k] = us[r][k] = 0.0f;
      Uc[r][k] = Us[r][k] = 0.0;
    }
    cc32[r] = cs32[r] = 0.0f;
    cc[r] = cs[r] = hc[r] = hs[r] = 0.0;
  }

  constexpr int TS = 64;  // samples per table tile (and per float32 partial sum)
  __shared__ double2 eash[TS][16];
  __shared__ double2 bsh[TS][16];
  const int ta_ = threadIdx.x >> 4, tb_ = threadIdx.x & 15;
  const double fb = static_cast<double>(wk.j0 + 1) * df;
  const double* __restrict__ q0 = rec + si.rec_off;
  const float* __restrict__ g0 = g32 + si.g32_off;
  for (int64_t i0 = 0; i0 < N; i0 += TS) {
    const int nts = N - i0 < TS ? static_cast<int>(N - i0) : TS;
    __syncthreads();
    build_phasor_tables<KP>(q0 + i0 * P, P, nts, fb, eash, bsh);
    __syncthreads();
    const double* __restrict__ q = q0 + i0 * P;
    const float* __restrict__ g = g0 + i0 * GW;
    // four samples per iteration: their scalar and LDS loads are issued
    // together, so one wait covers them
#pragma unroll 4
    for (int sl = 0; sl < nts; ++sl, q += P, g += GW) {
      const double2 ea = eash[sl][ta_];
      const double2 bb = bsh[sl][tb_];
      double c = __builtin_fma(ea.x, bb.x, -ea.y * bb.y);
      double s = __builtin_fma(ea.y, bb.x, ea.x * bb.y);
      const double rc = q[1], rs = q[2];
      const double gr = q[3 + K];  // w~ r_b
      const float wf = g[K];       // w~
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r) {
          const double cn = __builtin_fma(c, rc, -s * rs);
          s = __builtin_fma(s, rc, c * rs);
          c = cn;
        }
        const float cf = static_cast<float>(c), sf = static_cast<float>(s);
#pragma unroll
        for (int k = 0; k < K; ++k) {
          uc[r][k] = __builtin_fmaf(g[k], cf, uc[r][k]);
          us[r][k] = __builtin_fmaf(g[k], sf, us[r][k]);
        }
        const float wc = wf * cf;
        cc32[r] = __builtin_fmaf(wc, cf, cc32[r]);
        cs32[r] = __builtin_fmaf(wc, sf, cs32[r]);
        hc[r] = __builtin_fma(gr, c, hc[r]);
        hs[r] = __builtin_fma(gr, s, hs[r]);
      }
    }
    // float32 tile sums into the float64 totals
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        Uc[r][k] += static_cast<double>(uc[r][k]);
        Us[r][k] += static_cast<double>(us[r][k]);
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
      Scc = __builtin_fma(-Uc[r][k], Uc[r][k], Scc);
      Scs = __builtin_fma(-Uc[r][k], Us[r][k], Scs);
      Sss = __builtin_fma(-Us[r][k], Us[r][k], Sss);
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
      const unsigned long long slot = atomicAdd(count, 1ull);
      list[slot] = Rescore{wk.series, 0, j};
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
