// Residual periodogram scan in float64 (eq. zpowrel with n = 1, Sects. 3, 5).
//
// Layout: one lane owns R grid frequencies f_{j0+t+256r}, r = 0..R-1, and
// walks over all samples of its series.  The per-sample record
// [tau, cos(2 pi s tau), sin(2 pi s tau), w~ q_0 .. w~ q_{K-1}, w~ r_b,
//  cos(2 pi df tau), sin(2 pi df tau)]
// (s = 256 df; q the orthonormal base columns, r_b the base residual, both
// from the preparation kernel) is the same for every lane, so it is read with
// scalar loads and used as a scalar operand.  The phasor of the lane's first
// frequency at a sample is a product of three factors,
//   e^{2 pi i (j0 + 1 + 16a + b) df tau} = E0 * A_a * B_b   (t = 16a + b),
// with E0 (the block's first frequency) from the float64 phase reduction and
// A_a = e^{2 pi i 16 a df tau}, B_b = e^{2 pi i b df tau} from powers of
// e^{2 pi i df tau}; the block builds E0 A_a and B_b for a tile of 64 samples
// in LDS, so each lane spends one complex multiplication per sample instead
// of a sin/cos.  The other R-1 frequencies follow by rotation with the
// record's (cos, sin)(2 pi s tau).  Per frequency the lane accumulates
//   U_c[k] = <q_k cos>, U_s[k] = <q_k sin>, h = <r_b cos>, <r_b sin>,
//   <cos^2>, <cos sin>   (<sin^2> = <1> - <cos^2>, eq. idn)
// and the epilogue extends the base Cholesky factor by the 2x2 Schur block of
// the trial column pair (the incremental extension of Sect. 3):
//   S = C - U^T U, a_psi = L_S^{-1} h, l_{m+1} = l_m - |a_psi|^2,
//   z = (N - 3m - 4)/2 ln(l_m / l_{m+1}).
#include "fredec_internal.h"
#include "scan_phasor.h"

namespace fredec {

namespace {

// Frequencies per lane: as many as keep the R (2 KP + 3) float64 sums within
// about 190 VGPRs (two waves per SIMD).
constexpr int R_of(int KP) {
  int r = 92 / (2 * KP + 3);
  return r < 1 ? 1 : (r > 8 ? 8 : r);
}

// Epilogue of one frequency from its sums (orthonormal base columns q_k,
// base residual r_b; see the preparation kernel), all weighted by w~ q_0:
//   acc[0], acc[1]          <q_0 cos>, <q_0 sin>
//   acc[2], acc[3]          <cos^2>, <cos sin>  (acc[4] is not used)
//   acc[3+2k], acc[4+2k]    <q_k cos>, <q_k sin> (k = 1..K-1), then <r_b cos>, <r_b sin> (k = K)
// q_0 = <1>^{-1/2} is the constant column, so <sin^2> = <1> - <cos^2> (eq.
// idn) is sqrt(<1>) - acc[2] in these units.
template <int KP>
__device__ __forceinline__ void scan_epilogue(const double (&acc)[2 * KP + 3], double f, const SeriesIn& si,
                                              const SeriesHdr& h, double& z, uint8_t& flag) {
  constexpr int K = KP - 1;
  const double cc = acc[2], ss = sqrt(h.W1) - acc[2];
  double Scc = cc, Scs = acc[3], Sss = ss;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double uc = (k == 0) ? acc[0] : acc[3 + 2 * k];
    const double us = (k == 0) ? acc[1] : acc[4 + 2 * k];
    Scc = __builtin_fma(-uc, uc, Scc);
    Scs = __builtin_fma(-uc, us, Scs);
    Sss = __builtin_fma(-us, us, Sss);
  }
  const double hc = acc[3 + 2 * K], hs = acc[4 + 2 * K];
  schur_finish(Scc, Scs, Sss, cc, ss, hc, hs, f, si, h, z, flag);
}

constexpr int F64_TS = 64;  // samples per table tile of the float64 scan

// Samples per chunk when a scan is split over nsplit sample chunks (whole tiles).
__host__ __device__ inline int64_t f64_chunk(int64_t N, int nsplit) {
  return ((N + nsplit - 1) / nsplit + F64_TS - 1) / F64_TS * F64_TS;
}

// SPLIT: the work item covers the samples of chunk wk.pad (of nsplit) and
// writes its raw sums to part[(chunk NS + k) F + j] for the reduction kernel
// instead of finishing the frequencies.
template <int KP, int R, bool SPLIT>
__global__ __launch_bounds__(BLOCK) void scan_f64_kernel(const ScanWork* __restrict__ work,
                                                         const SeriesIn* __restrict__ sin_,
                                                         const SeriesHdr* __restrict__ hdr,
                                                         const double* __restrict__ rec,
                                                         double* __restrict__ z_out, uint8_t* __restrict__ flags_out,
                                                         double* __restrict__ part, int nsplit) {
  constexpr int NS = 2 * KP + 3;
  constexpr int P = rec_stride(KP);
  const ScanWork wk = work[blockIdx.x];
  const SeriesIn& si = sin_[wk.series];
  const SeriesHdr& h = hdr[wk.series];
  const int64_t N = si.N;
  const int64_t F = si.F;
  const double df = si.df;
  const int64_t jb = wk.j0 + threadIdx.x;
  double* zs = z_out + si.goff;
  uint8_t* fs = flags_out ? flags_out + si.goff : nullptr;
  int64_t i_lo = 0, i_hi = N;
  if constexpr (SPLIT) {
    const int64_t nc = f64_chunk(N, nsplit);
    i_lo = static_cast<int64_t>(wk.pad) * nc;
    i_hi = i_lo + nc < N ? i_lo + nc : N;
    if (h.status != 0) return;  // the reduction writes NaN
  }
  if (!SPLIT && h.status != 0) {
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
  double acc[R][NS];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[r][k] = 0.0;

  constexpr int TS = F64_TS;  // samples per table tile
  __shared__ double2 eash[TS][16];  // E0 A_a per sample, a = t / 16
  __shared__ double2 bsh[TS][16];   // B_b per sample, b = t % 16
  const int ta_ = threadIdx.x >> 4, tb_ = threadIdx.x & 15;
  const double fb = static_cast<double>(wk.j0 + 1) * df;  // the block's first frequency
  const double* __restrict__ q0 = rec + si.rec_off;
  for (int64_t i0 = i_lo; i0 < i_hi; i0 += TS) {
    const int nts = i_hi - i0 < TS ? static_cast<int>(i_hi - i0) : TS;
    __syncthreads();
    build_phasor_tables<KP>(q0 + i0 * P, P, nts, fb, eash, bsh);
    __syncthreads();
    // two samples per iteration: their scalar and LDS loads are issued
    // together, so one wait covers both
    const double* __restrict__ q = q0 + i0 * P;
#pragma unroll 2
    for (int sl = 0; sl < nts; ++sl, q += P) {
      const double2 ea = eash[sl][ta_];
      const double2 bb = bsh[sl][tb_];
      double c = __builtin_fma(ea.x, bb.x, -ea.y * bb.y);
      double s = __builtin_fma(ea.y, bb.x, ea.x * bb.y);
      const double rc = q[1], rs = q[2];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (r) {
          const double cn = __builtin_fma(c, rc, -s * rs);
          s = __builtin_fma(s, rc, c * rs);
          c = cn;
        }
        const double g0 = q[3];
        const double tc = g0 * c, tsn = g0 * s;
        acc[r][0] += tc;
        acc[r][1] += tsn;
        acc[r][2] = __builtin_fma(tc, c, acc[r][2]);
        acc[r][3] = __builtin_fma(tc, s, acc[r][3]);
#pragma unroll
        for (int k = 1; k < KP; ++k) {
          const double g = q[3 + k];
          acc[r][3 + 2 * k] = __builtin_fma(g, c, acc[r][3 + 2 * k]);
          acc[r][4 + 2 * k] = __builtin_fma(g, s, acc[r][4 + 2 * k]);
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t j = jb + (int64_t)BLOCK * r;
    if (j < F) {
      if constexpr (SPLIT) {
        double* pc = part + static_cast<int64_t>(wk.pad) * NS * F + j;
#pragma unroll
        for (int k = 0; k < NS; ++k) pc[k * F] = acc[r][k];
      } else {
        double z;
        uint8_t fl;
        scan_epilogue<KP>(acc[r], static_cast<double>(j + 1) * df, si, h, z, fl);
        zs[j] = z;
        if (fs) fs[j] = fl;
      }
    }
  }
}

// The chunks' sums of a split scan (one series) added in chunk order, then
// the epilogue: one thread per grid frequency.
template <int KP>
__global__ __launch_bounds__(BLOCK) void scan_f64_reduce_kernel(const SeriesIn* __restrict__ sin_,
                                                                const SeriesHdr* __restrict__ hdr,
                                                                const double* __restrict__ part, int nsplit,
                                                                double* __restrict__ z_out,
                                                                uint8_t* __restrict__ flags_out) {
  constexpr int NS = 2 * KP + 3;
  const SeriesIn& si = sin_[0];
  const SeriesHdr& h = hdr[0];
  const int64_t F = si.F;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  if (j >= F) return;
  double* zs = z_out + si.goff;
  uint8_t* fs = flags_out ? flags_out + si.goff : nullptr;
  if (h.status != 0) {
    zs[j] = __builtin_nan("");
    if (fs) fs[j] = FREDEC_FLAG_BADSERIES;
    return;
  }
  double acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    double v = 0.0;
    for (int c = 0; c < nsplit; ++c) v += part[(static_cast<int64_t>(c) * NS + k) * F + j];
    acc[k] = v;
  }
  double z;
  uint8_t fl;
  scan_epilogue<KP>(acc, static_cast<double>(j + 1) * si.df, si, h, z, fl);
  zs[j] = z;
  if (fs) fs[j] = fl;
}

// Same statistic at an explicit list of grid indices of one series: one
// workgroup per index, its samples spread over the four waves (float64 phase
// reduction and sin/cos per sample), the 2 KP + 3 partial sums reduced across
// each wave with DPP and shuffles and then across the waves in wave order
// (fixed order: deterministic).  A wave per index left each wave one long
// dependent chain of record loads (about 300 us for N = 10^4).
template <int KP>
__global__ __launch_bounds__(BLOCK) void scan_at_f64_kernel(const SeriesIn* __restrict__ sin_,
                                                            const SeriesHdr* __restrict__ hdr,
                                                            const double* __restrict__ rec,
                                                            const int64_t* __restrict__ idx, int64_t n_idx,
                                                            double* __restrict__ z_out, uint8_t* __restrict__ flags_out) {
  constexpr int NS = 2 * KP + 3;
  constexpr int P = rec_stride(KP);
  constexpr int NW = BLOCK / 64;
  __shared__ double part[NW][NS];
  const SeriesIn& si = sin_[0];
  const SeriesHdr& h = hdr[0];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t g = blockIdx.x;
  if (g >= n_idx) return;  // uniform over the block
  if (h.status != 0) {
    if (threadIdx.x == 0) {
      z_out[g] = __builtin_nan("");
      if (flags_out) flags_out[g] = FREDEC_FLAG_BADSERIES;
    }
    return;
  }
  const int64_t j = idx[g];
  const double f = static_cast<double>(j + 1) * si.df;
  double acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0.0;
  const double* __restrict__ q0 = rec + si.rec_off;
  for (int64_t i = threadIdx.x; i < si.N; i += BLOCK) {
    const double* q = q0 + i * P;
    double s, c;
    sincos_rev(f * q[0], s, c);
    const double g0 = q[3];
    const double tc = g0 * c, tsn = g0 * s;
    acc[0] += tc;
    acc[1] += tsn;
    acc[2] = __builtin_fma(tc, c, acc[2]);
    acc[3] = __builtin_fma(tc, s, acc[3]);
#pragma unroll
    for (int k = 1; k < KP; ++k) {
      const double gk = q[3 + k];
      acc[3 + 2 * k] = __builtin_fma(gk, c, acc[3 + 2 * k]);
      acc[4 + 2 * k] = __builtin_fma(gk, s, acc[4 + 2 * k]);
    }
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    acc[k] = group_sum<64>(acc[k]);
    if (lane == 0) part[wave][k] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      double v = part[0][k];
#pragma unroll
      for (int w2 = 1; w2 < NW; ++w2) v += part[w2][k];
      acc[k] = v;
    }
    double z;
    uint8_t fl;
    scan_epilogue<KP>(acc, f, si, h, z, fl);
    z_out[g] = z;
    if (flags_out) flags_out[g] = fl;
  }
}

template <int KP>
hipError_t launch_kp(hipStream_t st, int n_work, const ScanWork* work, const SeriesIn* sin, const SeriesHdr* hdr,
                     const double* rec, double* z, uint8_t* flags, double* part, int nsplit, int64_t F_split) {
  if (nsplit > 1) {
    scan_f64_kernel<KP, R_of(KP), true><<<n_work, BLOCK, 0, st>>>(work, sin, hdr, rec, z, flags, part, nsplit);
    scan_f64_reduce_kernel<KP><<<static_cast<unsigned>((F_split + BLOCK - 1) / BLOCK), BLOCK, 0, st>>>(
        sin, hdr, part, nsplit, z, flags);
  } else {
    scan_f64_kernel<KP, R_of(KP), false><<<n_work, BLOCK, 0, st>>>(work, sin, hdr, rec, z, flags, nullptr, 1);
  }
  return hipGetLastError();
}

template <int KP>
hipError_t launch_at_kp(hipStream_t st, const SeriesIn* sin, const SeriesHdr* hdr, const double* rec,
                        const int64_t* idx, int64_t n_idx, double* z, uint8_t* flags) {
  // one workgroup per index
  scan_at_f64_kernel<KP><<<static_cast<unsigned>(n_idx), BLOCK, 0, st>>>(sin, hdr, rec, idx, n_idx, z, flags);
  return hipGetLastError();
}

}  // namespace

int scan_freqs_per_thread(int KP) { return R_of(KP); }

int scan_f64_nsplit(int64_t N, int KP, int64_t F) {
  const int64_t tile = static_cast<int64_t>(BLOCK) * R_of(KP);
  const int64_t tiles = (F + tile - 1) / tile;
  if (tiles >= 128) return 1;
  int64_t ns = 256 / tiles;
  if (ns > 16) ns = 16;
  if (ns > N / 256) ns = N / 256;
  return ns < 2 ? 1 : static_cast<int>(ns);
}

#define FREDEC_KP_CASES(X) \
  X(2) X(4) X(6) X(8) X(10) X(12) X(14) X(16) X(18) X(20) X(22) X(24) X(26) \
  X(28) X(30) X(32) X(34) X(36) X(38) X(40) X(42) X(44) X(46) X(48) X(50)

hipError_t launch_scan_f64(hipStream_t st, int KP, int n_work, const ScanWork* work, const SeriesIn* sin,
                           const SeriesHdr* hdr, const double* rec, double* z, uint8_t* flags, double* part,
                           int nsplit, int64_t F_split) {
  if (n_work <= 0) return hipSuccess;
  switch (KP) {
#define X(kp) \
  case kp:    \
    return launch_kp<kp>(st, n_work, work, sin, hdr, rec, z, flags, part, nsplit, F_split);
    FREDEC_KP_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_scan_at_f64(hipStream_t st, int KP, const SeriesIn* sin, const SeriesHdr* hdr, const double* rec,
                              const int64_t* idx, int64_t n_idx, double* z, uint8_t* flags) {
  if (n_idx <= 0) return hipSuccess;
  if (n_idx > 0x7fffffff) return hipErrorInvalidValue;  // one workgroup per index
  switch (KP) {
#define X(kp) \
  case kp:    \
    return launch_at_kp<kp>(st, sin, hdr, rec, idx, n_idx, z, flags);
    FREDEC_KP_CASES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace fredec
