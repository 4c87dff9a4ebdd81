// float64 re-scoring of the grid points that the reduced-precision scan
// kernels listed (eq. zpowrel with n = 1): points where the trial columns lie
// nearly in the span of the base model (relative Schur pivot below RHO_MIN:
// next to a base frequency, or f T_eff of order 1) and the tops of strong
// peaks (l_{m+1} / l_m below LRATIO_MIN), where reduced-precision sums lose
// accuracy.  Every sum is recomputed in float64 from the float64 records, with
// the table-based float64 sin/cos, and the Schur epilogue of the float64 scan
// finishes the point.
#include "fredec_internal.h"

namespace fredec {

namespace {

// Plan of the float64 re-scoring (one workgroup).  off[0 .. n] = exclusive
// prefix over series of ceil(count[s] / 64) (chunks of 64 points),
// off[n + 1 .. 2n + 1] = exclusive prefix of count[s] (points), off[2n + 2] =
// the mode: 1 (one lane per point, chunks of a series) when there are at
// least `lane_min` chunks, else 0 (one workgroup per point, samples over its
// lanes), which keeps a few points of long series from running on a handful
// of waves.  Each thread sums a contiguous range of series; the thread totals
// are scanned in a fixed order.
__global__ __launch_bounds__(BLOCK) void rescore_plan_kernel(int n_series, const unsigned long long* __restrict__ count,
                                                             int64_t lane_min, int64_t* __restrict__ off) {
  __shared__ int64_t tot[2][BLOCK];
  const int tid = threadIdx.x;
  const int per = (n_series + BLOCK - 1) / BLOCK;
  const int s0 = tid * per, s1 = min(n_series, s0 + per);
  int64_t tc = 0, tp = 0;
  for (int s = s0; s < s1; ++s) {
    tc += static_cast<int64_t>((count[s] + 63) / 64);
    tp += static_cast<int64_t>(count[s]);
  }
  tot[0][tid] = tc;
  tot[1][tid] = tp;
  __syncthreads();
  if (tid < 2) {
    int64_t acc = 0;
    for (int k = 0; k < BLOCK; ++k) {
      const int64_t v = tot[tid][k];
      tot[tid][k] = acc;
      acc += v;
    }
    off[tid * (n_series + 1) + n_series] = acc;
    if (tid == 0) off[2 * n_series + 2] = acc >= lane_min ? 1 : 0;
  }
  __syncthreads();
  int64_t oc = tot[0][tid], op = tot[1][tid];
  for (int s = s0; s < s1; ++s) {
    off[s] = oc;
    off[n_series + 1 + s] = op;
    oc += static_cast<int64_t>((count[s] + 63) / 64);
    op += static_cast<int64_t>(count[s]);
  }
}

// Series of item c of a prefix array o[0 .. n] (o[0] = 0 <= c < o[n]): the
// last s with o[s] <= c (uniform in the wave).
__device__ __forceinline__ int series_of(const int64_t* __restrict__ o, int n, int64_t c) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (o[mid] <= c) lo = mid; else hi = mid;
  }
  return lo;
}

// Schur epilogue of one re-scored point from its 2 KP + 3 sums (the data
// column is the sum pair of column KP - 1).
template <int KP>
__device__ __forceinline__ void rescore_finish(const double (&acc)[2 * KP + 3], double f, const SeriesIn& si,
                                               const SeriesHdr& h, double& z, uint8_t& fl) {
  constexpr int K = KP - 1;
  const double cc = acc[2], ss = acc[4];
  double Scc = cc, Scs = acc[3], Sss = ss;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const double uc = (q == 0) ? acc[0] : acc[3 + 2 * q];
    const double us = (q == 0) ? acc[1] : acc[4 + 2 * q];
    Scc = __builtin_fma(-uc, uc, Scc);
    Scs = __builtin_fma(-uc, us, Scs);
    Sss = __builtin_fma(-us, us, Sss);
  }
  const double hc = (K == 0) ? acc[0] : acc[3 + 2 * K];
  const double hs = (K == 0) ? acc[1] : acc[4 + 2 * K];
  schur_finish(Scc, Scs, Sss, cc, ss, hc, hs, f, si, h, z, fl);
}

// Sums of one sample for one frequency (phase reduction and sin/cos in
// float64): the 2 KP + 3 entries of acc.  KP is the exact column count of
// the series, so the record's columns are loads at constant offsets (wide
// scalar loads where the record is uniform across the wave).
template <int KP>
__device__ __forceinline__ void rescore_sample(const double* __restrict__ q, double f,
                                               const double2* __restrict__ tab, double (&acc)[2 * KP + 3]) {
  double g[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) g[k] = q[3 + k];
  double sv, cv;
  sincos_tab(f * q[0], tab, sv, cv);
  const double tc = g[0] * cv, tsn = g[0] * sv;
  acc[0] += tc;
  acc[1] += tsn;
  acc[2] = __builtin_fma(tc, cv, acc[2]);
  acc[3] = __builtin_fma(tc, sv, acc[3]);
  acc[4] = __builtin_fma(tsn, sv, acc[4]);
#pragma unroll
  for (int k = 1; k < KP; ++k) {
    acc[3 + 2 * k] = __builtin_fma(g[k], cv, acc[3 + 2 * k]);
    acc[4 + 2 * k] = __builtin_fma(g[k], sv, acc[4 + 2 * k]);
  }
}

// One wavefront's chunk of up to 64 points of one series (one lane per
// point; `live` lanes past the series' count compute but store nothing).
template <int KP>
__device__ __forceinline__ void rescore_chunk(const SeriesIn& si, const SeriesHdr& h, const double* __restrict__ rec,
                                              const double2* __restrict__ tab, int64_t j, bool live,
                                              double* __restrict__ z_out, uint8_t* __restrict__ flags_out) {
  constexpr int P = rec_stride(KP);
  const double f = static_cast<double>(j + 1) * si.df;
  double acc[2 * KP + 3];
#pragma unroll
  for (int q = 0; q < 2 * KP + 3; ++q) acc[q] = 0.0;
  const double* __restrict__ qr = rec + si.rec_off;
#pragma unroll 2
  for (int64_t i = 0; i < si.N; ++i) rescore_sample<KP>(qr + i * P, f, tab, acc);
  if (live) {
    double z;
    uint8_t fl;
    rescore_finish<KP>(acc, f, si, h, z, fl);
    z_out[si.goff + j] = z;
    if (flags_out) flags_out[si.goff + j] = fl | FREDEC_FLAG_RESCORED;
  }
}

// One point over a workgroup (samples over its lanes; the waves' sums added
// in wave order through `part`, which holds at least 2 KP + 3 doubles per wave).
template <int KP>
__device__ __forceinline__ void rescore_point_block(const SeriesIn& si, const SeriesHdr& h,
                                                    const double* __restrict__ rec, const double2* __restrict__ tab,
                                                    int64_t j, double* part, int part_stride,
                                                    double* __restrict__ z_out, uint8_t* __restrict__ flags_out) {
  constexpr int P = rec_stride(KP);
  constexpr int NS = 2 * KP + 3;
  constexpr int NW = BLOCK / 64;
  const int lane = threadIdx.x & 63;
  const int wb = threadIdx.x >> 6;
  const double f = static_cast<double>(j + 1) * si.df;
  double acc[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) acc[q] = 0.0;
  const double* q0 = rec + si.rec_off;
#pragma unroll 1
  for (int64_t i = threadIdx.x; i < si.N; i += BLOCK) rescore_sample<KP>(q0 + i * P, f, tab, acc);
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    acc[q] = group_sum<64>(acc[q]);
    asm volatile("" : "+v"(acc[q]));  // one sum at a time: keeps the register count down
    if (lane == 0) part[wb * part_stride + q] = acc[q];
  }
  __syncthreads();
  // the waves' sums added in wave order, one thread per sum, into wave 0's slots
  for (int q = threadIdx.x; q < NS; q += BLOCK) {
    double v = part[q];
#pragma unroll
    for (int w = 1; w < NW; ++w) v += part[w * part_stride + q];
    part[q] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NS; ++q) acc[q] = part[q];
    double z;
    uint8_t fl;
    rescore_finish<KP>(acc, f, si, h, z, fl);
    z_out[si.goff + j] = z;
    if (flags_out) flags_out[si.goff + j] = fl | FREDEC_FLAG_RESCORED;
  }
  __syncthreads();  // part is reused by the next point
}

// Dispatch on the series' column count KP = 2 m + 2 (uniform over the
// workgroup's current item) to the body compiled for it; KP <= KPMAX.
#define FREDEC_RESCORE_KP_CASES(X) \
  X(2) X(4) X(6) X(8) X(10) X(12) X(14) X(16) X(18) X(20) X(22) X(24) X(26) X(28) X(30) X(32) X(34) X(36) \
  X(38) X(40) X(42) X(44) X(46) X(48) X(50)
static_assert(MAXKP == 50, "the KP cases cover 2 .. MAXKP");

// float64 re-scoring, many points: series s's points sit at list[goff_s ..
// goff_s + count[s]) and are taken in chunks of 64, one wavefront per chunk
// and one lane per point, so that the sample records of the series are
// uniform across the wave (scalar loads) and every lane accumulates the sums
// of its own frequency, with no cross-lane reduction.
template <int KPMAX>
__global__ __launch_bounds__(BLOCK) void rescore_lanes_kernel(int n_series, const SeriesIn* __restrict__ sin_,
                                                              const SeriesHdr* __restrict__ hdr,
                                                              const double* __restrict__ rec,
                                                              const Rescore* __restrict__ list,
                                                              const unsigned long long* __restrict__ count,
                                                              const int64_t* __restrict__ off,
                                                              double* __restrict__ z_out,
                                                              uint8_t* __restrict__ flags_out) {
  __shared__ double2 tab[TRIG_TAB];
  if (off[2 * n_series + 2] != 1) return;  // uniform over the grid
  trig_table_fill(tab);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t n_chunks = off[n_series];
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (BLOCK / 64);
  const int64_t w0 = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x * (BLOCK / 64) + (threadIdx.x >> 6)));
  for (int64_t c = w0; c < n_chunks; c += waves) {
    const int s = series_of(off, n_series, c);
    const SeriesIn& si = sin_[s];
    const SeriesHdr& h = hdr[s];
    const int64_t k = (c - off[s]) * 64 + lane;
    const bool live = k < static_cast<int64_t>(count[s]);
    const int64_t j = live ? list[si.goff + k].j : 0;
    switch (si.KP) {
#define X(kp)                                                                   \
  case kp:                                                                      \
    if constexpr (kp <= KPMAX) rescore_chunk<kp>(si, h, rec, tab, j, live, z_out, flags_out); \
    break;
      FREDEC_RESCORE_KP_CASES(X)
#undef X
      default: break;
    }
  }
}

// float64 re-scoring, few points: one workgroup per point, the samples
// spread over its 256 lanes, the 2 KP + 3 partial sums reduced across each
// wave with DPP and shuffles, then over the waves in wave order.
template <int KPMAX>
__global__ __launch_bounds__(BLOCK) void rescore_wave_kernel(int n_series, const SeriesIn* __restrict__ sin_,
                                                             const SeriesHdr* __restrict__ hdr,
                                                             const double* __restrict__ rec,
                                                             const Rescore* __restrict__ list,
                                                             const int64_t* __restrict__ off,
                                                             double* __restrict__ z_out,
                                                             uint8_t* __restrict__ flags_out) {
  constexpr int NS = 2 * KPMAX + 3;
  constexpr int NW = BLOCK / 64;
  __shared__ double2 tab[TRIG_TAB];
  __shared__ double part[NW * NS];  // the waves' sums of the current point
  if (off[2 * n_series + 2] != 0) return;  // uniform over the grid
  trig_table_fill(tab);
  __syncthreads();
  const int64_t* poff = off + n_series + 1;
  const int64_t n_pts = poff[n_series];
  // one workgroup per point (few points: the samples over all 256 lanes keep
  // the record loads of each lane short), the waves' sums added in wave order
  for (int64_t e = blockIdx.x; e < n_pts; e += gridDim.x) {
    const int s = series_of(poff, n_series, e);
    const SeriesIn& si = sin_[s];
    const SeriesHdr& h = hdr[s];
    const int64_t j = list[si.goff + (e - poff[s])].j;
    switch (si.KP) {
#define X(kp)                                                                                 \
  case kp:                                                                                    \
    if constexpr (kp <= KPMAX) rescore_point_block<kp>(si, h, rec, tab, j, part, NS, z_out, flags_out); \
    break;
      FREDEC_RESCORE_KP_CASES(X)
#undef X
      default: break;
    }
  }
}

__global__ void zero_u64_kernel(unsigned long long* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

}  // namespace

hipError_t launch_rescore(hipStream_t st, int NT, int grid, int n_series, const SeriesIn* sin, const SeriesHdr* hdr,
                          const double* rec, const Rescore* list, const unsigned long long* count, int64_t* off,
                          double* z, uint8_t* flags) {
  // one lane per point once the chunks give every SIMD two waves
  rescore_plan_kernel<<<1, BLOCK, 0, st>>>(n_series, count, 2LL * grid * (BLOCK / 64), off);
  switch (NT) {
#define X(nt, kp)                                                                                                \
  case nt:                                                                                                       \
    rescore_lanes_kernel<kp><<<grid, BLOCK, 0, st>>>(n_series, sin, hdr, rec, list, count, off, z, flags); \
    rescore_wave_kernel<kp><<<grid, BLOCK, 0, st>>>(n_series, sin, hdr, rec, list, off, z, flags);          \
    break;
    X(1, 17) X(2, 33) X(3, 49) X(4, MAXKP)
#undef X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zero_u64(hipStream_t st, unsigned long long* p, int n) {
  zero_u64_kernel<<<(n + 63) / 64, 64, 0, st>>>(p, n);
  return hipGetLastError();
}

}  // namespace fredec

