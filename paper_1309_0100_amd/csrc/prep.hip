// Normalisation (Sect. 4.1, eq. idn) and base-model precomputation for the
// residual scan (eq. zpowrel).
//
// The base model's columns phi = (1, cos 2 pi f'_k t, sin 2 pi f'_k t) are
// replaced by an orthonormal basis q = L_A^{-1} phi (L_A the Cholesky factor
// of A = <phi phi^T>, Sect. 3) and the data by the base-model residual
// r_b = x~ - q . a_b with a_b = L_A^{-1} <x~ phi>.  The statistic is unchanged
// (the same column space and the same residual), but the scan then needs no
// triangular solve per frequency and its sums are better conditioned:
//   U = <q psi>, S = <psi psi^T> - U^T U, h = <r_b psi>,
//   l_{m+1} = l_m - h^T S^{-1} h,  l_m = D - |a_b|^2,  psi = (cos, sin)(2 pi f t).
//
// Three launches, so that the per-sample work of a series is spread over one
// workgroup per tile of up to 256 samples rather than walked by one
// workgroup:
//   prep_stats_kernel  one workgroup per series: weighted moments, T_eff,
//                      input checks (and, without a base model, the
//                      normalised series);
//   prep_rows_kernel   one per tile: normalised samples, the rows
//                      phi_i = (1, cos, sin .., x~_i) and their Gram matrix on
//                      float64 MFMA;
//   prep_factor_kernel one per series: the tiles' Gram matrices added, A
//                      factored, the basis change M formed;
//   prep_basis_kernel  one per tile: [w~ q; w~ r_b] = w~ M phi on float64
//                      MFMA and the operand records of the scan kernels.
#include "fredec_internal.h"

namespace fredec {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr int MAXNB = (MAXKP + 15) / 16;        // 16-column blocks of the Gram matrix
constexpr int MAXTL = MAXNB * (MAXNB + 1) / 2;  // its lower block triangle
constexpr int MAXKPP = MAXKP * (MAXKP + 1) / 2;
static_assert(prep_rows(MAXKP) >= 32, "sample tile below one 32-sample group");
static_assert(PREP_TILE >= 4 * BLOCK, "Gram reduction scratch");

// Workgroup barrier that waits for the LDS accesses only (no thread reads
// global memory written by another thread of its workgroup before the
// kernel's end).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// floor(e / d) for 0 <= e < 2^21 from a float reciprocal inv ~ 1/d: e + 1/2
// lies at least 1/2 away from a multiple of d, far beyond the float rounding
// of (e + 1/2) inv.
__device__ __forceinline__ int div_small(int e, float inv) {
  return static_cast<int>((static_cast<float>(e) + 0.5f) * inv);
}

// Series owning preparation tile b (uniform across the workgroup).
__device__ __forceinline__ int tile_series(const SeriesIn* __restrict__ sin, int n, int64_t b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (sin[mid].ptile0 <= b) lo = mid; else hi = mid;
  }
  return lo;
}

// Deterministic block sums (fixed order): wavefront sums by DPP, then the four
// wavefront totals in wave order.  red: 4 NV doubles of LDS.
template <int NV>
__device__ __forceinline__ void block_sum4(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = group_sum<64>(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = ((red[k] + red[NV + k]) + red[2 * NV + k]) + red[3 * NV + k];
}

__device__ __forceinline__ double block_max4(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// ---------------------------------------------------------------- statistics
__global__ __launch_bounds__(BLOCK) void prep_stats_kernel(const SeriesIn* __restrict__ sin_,
                                                           SeriesHdr* __restrict__ hdr, const double* __restrict__ t,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ w, double* __restrict__ tau,
                                                           double* __restrict__ xt, double* __restrict__ wt,
                                                           int flags) {
  __shared__ double red[4 * 8];
  const int tid = threadIdx.x;
  const SeriesIn& si = sin_[blockIdx.x];
  SeriesHdr& h = hdr[blockIdx.x];
  const int64_t N = si.N;
  const double* ts = t + si.soff;
  const double* xs = x + si.soff;
  const double* ws = w + si.soff;
  const bool with_base = (flags & PREP_BASE) != 0;

  // pass 1: weight sum, weighted first and raw second moments, input validity
  // (Sect. 2: w_i > 0) and the largest weight
  double v1[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double wmax = 0.0;
#pragma unroll 4
  for (int64_t i = tid; i < N; i += BLOCK) {
    const double wi = ws[i], ti = ts[i], xi = xs[i];
    const bool ok = (wi > 0.0) && isfinite(wi) && isfinite(ti) && isfinite(xi);
    v1[0] += wi;
    v1[1] += wi * ti;
    v1[2] += wi * xi;
    v1[3] += wi * ti * ti;
    v1[4] += wi * xi * xi;
    v1[5] += ok ? 0.0 : 1.0;
    wmax = fmax(wmax, wi);
  }
  block_sum4(v1, red);
  wmax = block_max4(wmax, red);
  int status = 0;
  if (v1[5] != 0.0 || !(v1[0] > 0.0) || !isfinite(v1[0])) status = FREDEC_EWEIGHT;
  const double W = v1[0];
  const double tbar = v1[1] / W, xbar = v1[2] / W;

  // pass 2: central second moments
  double v2[2] = {0.0, 0.0};
#pragma unroll 4
  for (int64_t i = tid; i < N; i += BLOCK) {
    const double wi = ws[i] / W;
    const double ta = ts[i] - tbar, d = xs[i] - xbar;
    v2[0] += wi * ta * ta;
    v2[1] += wi * d * d;
  }
  block_sum4(v2, red);
  const double var_t = v2[0], sx2 = v2[1];
  if (status == 0 && (sx2 <= 1e-28 * (v1[4] / W) || var_t <= 1e-28 * (v1[3] / W))) status = FREDEC_EDEGEN;
  if (status == 0 && with_base && N - 3 * static_cast<int64_t>(si.m) - 4 <= 0) status = FREDEC_EDOF;
  const double sx = sqrt(sx2);
  const double T_eff = sqrt(4.0 * M_PI * var_t);
  if (tid == 0) {
    h.T_eff = T_eff;
    h.stats[0] = tbar;
    h.stats[1] = xbar;
    h.stats[2] = sx;
    h.stats[3] = var_t;
    h.stats[4] = T_eff;
    h.stats[5] = W;
    h.wmax = wmax / W;
    h.status = status;
    if (with_base) {
      h.l_m = 0.0;
      h.NH = static_cast<double>(N - 3 * static_cast<int64_t>(si.m) - 4);
    }
  }
  if (!with_base) {
    double* taus = tau + si.soff;
    double* xts = xt + si.soff;
    double* wts = wt + si.soff;
#pragma unroll 4
    for (int64_t i = tid; i < N; i += BLOCK) {
      taus[i] = ts[i] - tbar;
      xts[i] = (xs[i] - xbar) / sx;
      wts[i] = ws[i] / W;
    }
  }
}

// ------------------------------------------------------- rows and factorisation
__global__ __launch_bounds__(BLOCK) void prep_rows_kernel(int n_series, const SeriesIn* __restrict__ sin_,
                                                          const SeriesHdr* __restrict__ hdr, const double* __restrict__ t,
                                                          const double* __restrict__ x,
                                                          const double* __restrict__ w, double* __restrict__ tau,
                                                          double* __restrict__ xt, double* __restrict__ wt,
                                                          double* __restrict__ phi, double* __restrict__ ppart) {
  extern __shared__ double tile[];  // staged rows (stride KP | 1); Gram reduction scratch
  __shared__ double wsh[BLOCK];
  const int tid = threadIdx.x;
  const int s = tile_series(sin_, n_series, blockIdx.x);
  const SeriesIn& si = sin_[s];
  const SeriesHdr& h = hdr[s];
  if (h.status != 0) return;
  const int64_t N = si.N;
  const int KP = si.KP;
  const int m = si.m;
  const int RS = prep_rs(KP);
  const int T = si.prows;
  const int KPP = KP * (KP + 1) / 2;
  const int64_t tl = blockIdx.x - si.ptile0;
  const int64_t i0 = tl * T;
  const int nts = N - i0 < T ? static_cast<int>(N - i0) : T;
  const double tbar = h.stats[0], xbar = h.stats[1], sx = h.stats[2], W = h.stats[5];
  const int nbk = (KP + 15) / 16;
  const int lane = tid & 63, wave = tid >> 6;
  const int c16 = lane & 15, kq = lane >> 4;

  // normalised samples and the rows phi_i of the tile, in LDS and in the phi
  // array (zero rows beyond N)
  if (tid < T) {
    double* row = tile + tid * RS;
    if (tid < nts) {
      const int64_t i = si.soff + i0 + tid;
      const double wi = w[i] / W;
      const double ta = t[i] - tbar;
      const double xi = (x[i] - xbar) / sx;
      tau[i] = ta;
      xt[i] = xi;
      wt[i] = wi;
      wsh[tid] = wi;
      row[0] = 1.0;
      for (int k = 0; k < m; ++k) {
        double sn, cs;
        sincos_rev(si.base_f[k] * ta, sn, cs);
        row[1 + 2 * k] = cs;
        row[2 + 2 * k] = sn;
      }
      row[KP - 1] = xi;
    } else {
      wsh[tid] = 0.0;
      for (int c = 0; c < KP; ++c) row[c] = 0.0;
    }
  }
  lds_barrier();
  {
    double* dst = phi + si.phi_off + i0 * KP;
    const int nel = nts * KP;
    const float invKP = 1.0f / static_cast<float>(KP);
    for (int e = tid; e < nel; e += BLOCK) {
      const int sl = div_small(e, invKP);
      dst[e] = tile[sl * RS + (e - sl * KP)];
    }
  }
  // Gram of the tile's rows on float64 MFMA: each wavefront takes every
  // fourth step of four samples and accumulates all lower 16x16 tiles of the
  // KP x KP Gram (lane (c16, kq): column c16 of the tile's row / column block
  // at the step's sample kq; D[r][c] in lane c + 16 (r % 4), register r / 4)
  v4d acc[MAXTL];
#pragma unroll
  for (int b = 0; b < MAXTL; ++b) acc[b] = v4d{0.0, 0.0, 0.0, 0.0};
  const int nsteps = (nts + 3) >> 2;
  for (int st = wave; st < nsteps; st += BLOCK / 64) {
    const int sl = 4 * st + kq;
    const double* row = tile + sl * RS;
    const double wv = wsh[sl];
    double col[MAXNB];
#pragma unroll
    for (int b = 0; b < MAXNB; ++b) col[b] = row[(b < nbk && 16 * b + c16 < KP) ? 16 * b + c16 : 0];
#pragma unroll
    for (int b = 0; b < MAXNB; ++b) col[b] = (b < nbk && 16 * b + c16 < KP) ? col[b] : 0.0;
#pragma unroll
    for (int b1 = 0; b1 < MAXNB; ++b1) {
      if (b1 < nbk) {
#pragma unroll
        for (int b2 = 0; b2 <= b1; ++b2)
          acc[b1 * (b1 + 1) / 2 + b2] =
              __builtin_amdgcn_mfma_f64_16x16x4f64(col[b1], wv * col[b2], acc[b1 * (b1 + 1) / 2 + b2], 0, 0, 0);
      }
    }
  }
  lds_barrier();
  // the four wavefronts' partial tiles, summed in wave order, to this tile's
  // Gram partial (packed lower triangle)
  double* part = ppart + si.ppart_off + tl * KPP;
#pragma unroll
  for (int b1 = 0; b1 < MAXNB; ++b1) {
    if (b1 < nbk) {
#pragma unroll
      for (int b2 = 0; b2 <= b1; ++b2) {
        const v4d a = acc[b1 * (b1 + 1) / 2 + b2];
#pragma unroll
        for (int v = 0; v < 4; ++v) tile[(wave * 4 + v) * 64 + lane] = a[v];
        lds_barrier();
        {
          const int v = tid >> 6;
          const double sum = ((tile[v * 64 + lane] + tile[(4 + v) * 64 + lane]) + tile[(8 + v) * 64 + lane]) +
                             tile[(12 + v) * 64 + lane];
          const int r = 16 * b1 + kq + 4 * v;
          const int c = 16 * b2 + c16;
          if (r < KP && c <= r) part[r * (r + 1) / 2 + c] = sum;
        }
        lds_barrier();
      }
    }
  }
}

// ------------------------------------------------------------ factorisation
__global__ __launch_bounds__(BLOCK) void prep_factor_kernel(const SeriesIn* __restrict__ sin_,
                                                            SeriesHdr* __restrict__ hdr,
                                                            const double* __restrict__ ppart,
                                                            double* __restrict__ pm) {
  __shared__ double gram[MAXKPP];
  __shared__ double Lsh[MAXK * (MAXK + 1) / 2];
  __shared__ double invd[MAXK];
  __shared__ double ab[MAXK];
  __shared__ double diag0[MAXK];
  __shared__ int bad_sh, status_sh;
  const int tid = threadIdx.x;
  const SeriesIn& si = sin_[blockIdx.x];
  SeriesHdr& h = hdr[blockIdx.x];
  if (h.status != 0) return;
  const int KP = si.KP;
  const int K = KP - 1;
  const int KPP = KP * (KP + 1) / 2;

  // Gram matrix: base normal matrix A, right-hand side g_b in the last row,
  // D = <x~^2> its last entry; the tile partials added in tile order
  {
    const double* p0 = ppart + si.ppart_off;
    for (int e = tid; e < KPP; e += BLOCK) {
      double v = 0.0;
#pragma unroll 8
      for (int k = 0; k < si.pntiles; ++k) v += p0[static_cast<int64_t>(k) * KPP + e];
      gram[e] = v;
    }
  }
  __syncthreads();  // the pivots below read entries summed by other threads
  // Cholesky A = L L^T (Sect. 3), right-looking: per column j the pivot and
  // the column below it, then the rank-one update of the trailing block, each
  // entry by its own thread (gram's rows 0..K-1 are overwritten; the original
  // diagonal is kept for the relative pivot test).
  for (int j = tid; j < K; j += BLOCK) diag0[j] = gram[j * (j + 1) / 2 + j];
  if (tid == 0) bad_sh = 0;
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    const double d = gram[j * (j + 1) / 2 + j];
    if (!(d > PIVOT_TOL * diag0[j])) {  // uniform: every thread reads the same pivot
      if (tid == 0) bad_sh = 1;
      break;
    }
    const double ljj = sqrt(d), inv = 1.0 / ljj;
    if (tid == 0) {
      Lsh[j * (j + 1) / 2 + j] = ljj;
      invd[j] = inv;
    }
    for (int i = j + 1 + tid; i < K; i += BLOCK) Lsh[i * (i + 1) / 2 + j] = gram[i * (i + 1) / 2 + j] * inv;
    __syncthreads();
    const int nr = K - 1 - j;  // trailing rows j+1 .. K-1
    for (int e = tid; e < nr * nr; e += BLOCK) {
      const int a = e / nr, b = e - a * nr;
      if (b <= a) {
        const int i = j + 1 + a, k = j + 1 + b;
        gram[i * (i + 1) / 2 + k] -= Lsh[i * (i + 1) / 2 + j] * Lsh[k * (k + 1) / 2 + j];
      }
    }
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0) {
    const int status = bad_sh ? FREDEC_ESINGULAR : 0;
    // a_b = L^{-1} g_b, l_m = D - a_b.a_b
    if (status == 0) {
      const double* gb = gram + K * (K + 1) / 2;  // row K: <x~ phi_k>, then D
      double aa = 0.0;
      for (int i = 0; i < K; ++i) {
        double v = gb[i];
        for (int k = 0; k < i; ++k) v -= Lsh[i * (i + 1) / 2 + k] * ab[k];
        ab[i] = v * invd[i];
        aa += ab[i] * ab[i];
      }
      h.D = gb[K];
      h.l_m = gb[K] - aa;
      // Split float16 operand of the MFMA scan, B = S sqrt(w~) q_k: since
      // sum_i w~_i q_k(i)^2 = 1, every |sqrt(w~_i) q_k(i)| <= 1; S = 2^12
      // puts twice that bound at 2^13, so |B| <= 2^12 (the float16 range
      // ends near 2^16) and the low parts of the typical entries clear the
      // float16 subnormals.
      h.b16_inv = 1.0 / 4096.0;
    }
    h.W1 = gram[0];
    h.status = status;
    status_sh = status;
  }
  __syncthreads();
  if (status_sh != 0) return;

  // The basis change as one matrix: [q; r_b] = M phi with
  //   M = [[X, 0], [-a_b^T X, 1]],  X = L^{-1},
  // packed (lower triangle, KP rows).  X by right-looking forward substitution
  // of L X = I: row j is final once scaled by 1 / L_jj, then it updates the
  // rows below it (one entry per thread).
  for (int e = tid; e < K * (K + 1) / 2; e += BLOCK) gram[e] = 0.0;
  __syncthreads();
  for (int j = tid; j < K; j += BLOCK) gram[j * (j + 1) / 2 + j] = 1.0;
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    const int rj = j * (j + 1) / 2;
    for (int c = tid; c <= j; c += BLOCK) gram[rj + c] *= invd[j];
    __syncthreads();
    const int nr = K - 1 - j, nc = j + 1;
    for (int e = tid; e < nr * nc; e += BLOCK) {
      const int a = e / nc, c = e - a * nc;
      const int k = j + 1 + a;
      gram[k * (k + 1) / 2 + c] -= Lsh[k * (k + 1) / 2 + j] * gram[rj + c];
    }
    __syncthreads();
  }
  double* M = pm + si.pm_off;
  for (int c = tid; c <= K; c += BLOCK) {
    double v = 1.0;
    if (c < K) {
      v = 0.0;
      for (int k = c; k < K; ++k) v = __builtin_fma(-ab[k], gram[k * (k + 1) / 2 + c], v);
    }
    M[K * (K + 1) / 2 + c] = v;
  }
  for (int e = tid; e < K * (K + 1) / 2; e += BLOCK) M[e] = gram[e];
}

// ------------------------------------------------------------ basis change
__global__ __launch_bounds__(BLOCK) void prep_basis_kernel(int n_series, const SeriesIn* __restrict__ sin_,
                                                           const SeriesHdr* __restrict__ hdr,
                                                           const double* __restrict__ tau,
                                                           const double* __restrict__ wt,
                                                           const double* __restrict__ phi,
                                                           const double* __restrict__ pm, double* __restrict__ rec,
                                                           float* __restrict__ g32, double* __restrict__ aux,
                                                           _Float16* __restrict__ b16, float2* __restrict__ pt16,
                                                           int flags) {
  extern __shared__ double tile[];  // rows (stride KP | 1), then PREP_PSS scalars per sample
  __shared__ double Msh[MAXKPP];
  __shared__ double wsh[BLOCK];
  const int tid = threadIdx.x;
  const int s = tile_series(sin_, n_series, blockIdx.x);
  const SeriesIn& si = sin_[s];
  const SeriesHdr& h = hdr[s];
  if (h.status != 0) return;
  const int64_t N = si.N;
  const int KP = si.KP;
  const int K = KP - 1;
  const int RS = prep_rs(KP);
  const int T = si.prows;
  const int KPP = KP * (KP + 1) / 2;
  const int64_t tl = blockIdx.x - si.ptile0;
  const int64_t i0 = tl * T;
  const int nts = N - i0 < T ? static_cast<int>(N - i0) : T;
  const int nbk = (KP + 15) / 16;
  const int lane = tid & 63, wave = tid >> 6;
  const int c16 = lane & 15, kq = lane >> 4;
  const int P = rec_stride(KP);
  const int NT = si.NT;
  const int G32W = 16 * NT;
  const bool w_rec = (flags & PREP_REC64) != 0;
  const bool w_g32 = (flags & si.outputs & PREP_G32) != 0;
  const bool w_aux = (flags & si.outputs & PREP_AUX) != 0;
  const bool w_f16 = (flags & si.outputs & PREP_F16) != 0;

  // M, the tile's rows, w~ and tau of the thread's sample
  for (int e = tid; e < KPP; e += BLOCK) Msh[e] = pm[si.pm_off + e];
  {
    const double* src = phi + si.phi_off + i0 * KP;
    const int nel = nts * KP;
    const float invKP = 1.0f / static_cast<float>(KP);
    constexpr int PER = (PREP_TILE + BLOCK - 1) / BLOCK;
    double v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = u * BLOCK + tid;
      v[u] = src[e < nel ? e : 0];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = u * BLOCK + tid;
      if (e < nel) {
        const int sl = div_small(e, invKP);
        tile[sl * RS + (e - sl * KP)] = v[u];
      }
    }
  }
  double ta = 0.0;
  if (tid < nts) {
    wsh[tid] = wt[si.soff + i0 + tid];
    ta = tau[si.soff + i0 + tid];
  }
  lds_barrier();

  // w~ q = w~ X phi and w~ r_b on float64 MFMA: each wavefront takes every
  // fourth block of 16 samples (lane (c16, kq) feeds phi at sample c16,
  // column j0 + kq and M at row 16 b + c16, column j0 + kq; the result for
  // sample kq + 4 v, column 16 b + c16 is in register v), written back over
  // the rows, weighted
  for (int sb = wave; 16 * sb < nts; sb += BLOCK / 64) {
    v4d o[MAXNB];
#pragma unroll
    for (int b = 0; b < MAXNB; ++b) o[b] = v4d{0.0, 0.0, 0.0, 0.0};
    const double* arow = tile + (16 * sb + c16) * RS;
    for (int j0 = 0; j0 < KP; j0 += 4) {
      const int jj = j0 + kq;
      // operands read unconditionally (clamped indices, zeroed by select)
      const double ar = arow[jj < KP ? jj : 0];
      double br[MAXNB];
#pragma unroll
      for (int b = 0; b < MAXNB; ++b) {
        const int c = 16 * b + c16;
        br[b] = Msh[c < KP && jj <= c ? c * (c + 1) / 2 + jj : 0];
      }
      const double av = jj < KP ? ar : 0.0;
#pragma unroll
      for (int b = 0; b < MAXNB; ++b) {
        if (b < nbk) {
          const int c = 16 * b + c16;
          o[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, c < KP && jj <= c ? br[b] : 0.0, o[b], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int b = 0; b < MAXNB; ++b) {
      if (b < nbk) {
        const int c = 16 * b + c16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int sl = 16 * sb + kq + 4 * v;
          if (c < KP) tile[sl * RS + c] = wsh[sl] * o[b][v];
        }
      }
    }
  }
  // per-sample scalars: tau, e^{2 pi i 256 df tau}, e^{2 pi i 16 df tau},
  // e^{2 pi i df tau} (cos, sin each), w~
  double* psc = tile + T * RS;
  if (tid < nts) {
    double* ps = psc + tid * PREP_PSS;
    ps[0] = ta;
    if (w_rec) sincos_rev(si.rot_step * ta, ps[2], ps[1]);
    if (w_aux) sincos_rev(si.rot_tile * ta, ps[4], ps[3]);
    sincos_rev(si.df * ta, ps[6], ps[5]);
    ps[7] = wsh[tid];
  }
  lds_barrier();

  // records of the tile's samples: contiguous blocks, written with
  // consecutive lanes on consecutive elements, one LDS read per element
  if (w_rec) {
    // tau, e^{2 pi i 256 df tau}, w~ q_0 .. w~ q_{K-1}, w~ r_b, e^{2 pi i df tau}, pad
    double* dst = rec + si.rec_off + i0 * P;
    const int n = nts * P;
    const float invP = 1.0f / static_cast<float>(P);
#pragma unroll 4
    for (int e = tid; e < n; e += BLOCK) {
      const int sl = div_small(e, invP), f = e - sl * P;
      const bool in_row = f >= 3 && f < KP + 3;
      const int pf = f < 3 ? f : f - KP + 2;  // cos, sin of e^{2 pi i df tau} at 5, 6
      const double v = tile[in_row ? sl * RS + f - 3 : T * RS + sl * PREP_PSS + (f < KP + 5 ? pf : 0)];
      dst[e] = f < KP + 5 ? v : 0.0;
    }
  }
  if (w_g32) {
    // w~ q_0 .. w~ q_{K-1}, then w~ (column K, never read by the MFMA kernel,
    // whose padding columns only produce unused sums, carries w~ for the VALU
    // kernel's <cos^2>, <cos sin>), then zeros
    float* dst = g32 + si.g32_off + i0 * G32W;
    const int n = nts * G32W;
    const float invG = 1.0f / static_cast<float>(G32W);
#pragma unroll 4
    for (int e = tid; e < n; e += BLOCK) {
      const int sl = div_small(e, invG), f = e - sl * G32W;
      const double v = tile[f < K ? sl * RS + f : T * RS + sl * PREP_PSS + 7];
      dst[e] = f <= K ? static_cast<float>(v) : 0.0f;
    }
  }
  if (w_aux) {
    // tau, e^{2 pi i 16 df tau}, sqrt(w~), sqrt(w~) r_b, 0, e^{2 pi i df tau}
    // (the split-float16 scan folds sqrt(w~) into its trial phasors)
    double* dst = aux + si.aux_off + i0 * AUX_STRIDE;
    const int n = nts * AUX_STRIDE;
#pragma unroll 4
    for (int e = tid; e < n; e += BLOCK) {
      const int sl = e >> 3, f = e & 7;
      const int pf = f == 0 ? 0 : f == 1 ? 3 : f == 2 ? 4 : f == 3 ? 7 : f == 6 ? 5 : 6;
      const double v = tile[f == 4 ? sl * RS + KP - 1 : T * RS + sl * PREP_PSS + pf];
      const double sw = sqrt(tile[T * RS + sl * PREP_PSS + 7]);
      dst[e] = f == 5 ? 0.0 : f == 3 ? sw : f == 4 ? v / sw : v;
    }
  }
  if (w_f16) {
    // phasor rows e^{2 pi i b df tau} (b < 16) of the tile's samples, by
    // rotation from b = 0 in float64, into their PT_TS-sample tiles; the
    // series' last tile is zero-filled to its end
    float2* pts = pt16 + si.pt_off;
    const int64_t iend = i0 + nts == N ? (N + PT_TS - 1) / PT_TS * PT_TS : i0 + nts;
    for (int64_t i = i0 + tid; i < iend; i += BLOCK) {
      const int sl = static_cast<int>(i - i0);
      float2* dst = pts + (i / PT_TS) * (16 * PT_TS) + (i % PT_TS);
      if (sl < nts) {
        const double wc = psc[sl * PREP_PSS + 5], ws = psc[sl * PREP_PSS + 6];
        double pc = 1.0, ps = 0.0;
        for (int b = 0; b < 16; ++b) {
          dst[b * PT_TS] = float2{static_cast<float>(pc), static_cast<float>(ps)};
          const double nc = __builtin_fma(pc, wc, -ps * ws);
          ps = __builtin_fma(ps, wc, pc * ws);
          pc = nc;
        }
      } else {
        for (int b = 0; b < 16; ++b) dst[b * PT_TS] = float2{0.0f, 0.0f};
      }
    }
  }
  if (w_f16) {
    // B = S sqrt(w~) q_k = hi + lo.  Layout: per step g of 32 samples and column
    // tile nt, the high part then the low part, each 64 lanes x 8 halves;
    // lane L holds column 16 nt + L % 16 at samples 32 g + 8 (L / 16) + e,
    // e < 8 (zero beyond N and beyond column K).
    const double S = 1.0 / h.b16_inv;
    _Float16* bser = b16 + si.b16_off * 8;
    const int64_t g0 = i0 / 32;  // T is a multiple of 32
    const int n_ent = ((nts + 31) / 32) * NT * 64;
    for (int e = tid; e < n_ent; e += BLOCK) {
      const int L = e & 63;
      const int gtl = e >> 6;  // local step * NT + nt
      const int nt = gtl % NT;
      const int col = 16 * nt + (L & 15);
      const int s0 = 32 * (gtl / NT) + 8 * (L >> 4);
      const int64_t gt = g0 * NT + gtl;
      h8 vhi, vlo;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int sl = s0 + k;
        const bool in = sl < nts && col < K;
        // tile holds w~ q_k; B takes sqrt(w~) q_k
        double v = in ? S * tile[in ? sl * RS + col : 0] / sqrt(tile[T * RS + (in ? sl : 0) * PREP_PSS + 7]) : 0.0;
        v = fmin(fmax(v, -65504.0), 65504.0);
        // hi: rounded to float32, then to float16 (the opaque copy keeps the
        // compiler from fusing the two roundings into a float64-to-float16
        // conversion, which has no instruction); lo: the remainder, exact in
        // float64, rounded the same way
        float vf = static_cast<float>(v);
        asm volatile("" : "+v"(vf));
        const _Float16 vh = static_cast<_Float16>(vf);
        float rf = static_cast<float>(v - static_cast<double>(vh));
        asm volatile("" : "+v"(rf));
        vhi[k] = vh;
        vlo[k] = static_cast<_Float16>(rf);
      }
      h8* dsth = reinterpret_cast<h8*>(bser) + (gt * 2) * 64 + L;
      dsth[0] = vhi;
      dsth[64] = vlo;
    }
  }
}

__global__ void copy_stats_kernel(int n_series, const SeriesHdr* __restrict__ hdr, double* __restrict__ l_base,
                                  int32_t* __restrict__ status, double* __restrict__ stats) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_series) return;
  const SeriesHdr& h = hdr[s];
  if (l_base) l_base[s] = h.status == 0 ? h.l_m : __builtin_nan("");
  if (status) status[s] = h.status;
  if (stats) {
    for (int k = 0; k < 6; ++k) stats[6 * s + k] = h.stats[k];
  }
}

}  // namespace

hipError_t launch_prep(hipStream_t st, int n_series, int kp_max, int64_t n_tiles, const SeriesIn* sin,
                       SeriesHdr* hdr, const double* t, const double* x, const double* w, double* tau, double* xt,
                       double* wt, double* rec, double* phi, float* g32, double* aux, void* b16, void* pt16,
                       double* ppart, double* pm, int flags) {
  if (n_series <= 0) return hipSuccess;
  if ((flags & PREP_BASE) &&
      (kp_max < 2 || kp_max > MAXKP || n_tiles <= 0 || n_tiles > 0x7fffffff || !ppart || !pm))
    return hipErrorInvalidValue;
  prep_stats_kernel<<<n_series, BLOCK, 0, st>>>(sin, hdr, t, x, w, tau, xt, wt, flags);
  if (!(flags & PREP_BASE)) return hipGetLastError();
  // Every series' tile (prep_rows(KP) rows of prep_rs(KP) doubles, plus
  // PREP_PSS per row for the basis kernel, KP <= kp_max) fits
  // min(PREP_TILE, BLOCK (prep_rs(kp_max) [+ PREP_PSS])); the rows kernel
  // also needs the Gram reduction scratch.
  int d_basis = BLOCK * (prep_rs(kp_max) + PREP_PSS);
  if (d_basis > PREP_TILE) d_basis = PREP_TILE;
  int d_rows = BLOCK * prep_rs(kp_max);
  if (d_rows > PREP_TILE) d_rows = PREP_TILE;
  if (d_rows < 4 * BLOCK) d_rows = 4 * BLOCK;
  const int nb = static_cast<int>(n_tiles);
  prep_rows_kernel<<<nb, BLOCK, sizeof(double) * static_cast<size_t>(d_rows), st>>>(n_series, sin, hdr, t, x, w, tau,
                                                                                    xt, wt, phi, ppart);
  prep_factor_kernel<<<n_series, BLOCK, 0, st>>>(sin, hdr, ppart, pm);
  prep_basis_kernel<<<nb, BLOCK, sizeof(double) * static_cast<size_t>(d_basis), st>>>(
      n_series, sin, hdr, tau, wt, phi, pm, rec, g32, aux, static_cast<_Float16*>(b16), static_cast<float2*>(pt16),
      flags);
  return hipGetLastError();
}

hipError_t launch_copy_stats(hipStream_t st, int n_series, const SeriesHdr* hdr, const SeriesIn* sin,
                             double* l_base, int32_t* status, double* stats) {
  (void)sin;
  if (n_series <= 0 || (!l_base && !status && !stats)) return hipSuccess;
  copy_stats_kernel<<<(n_series + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(n_series, hdr, l_base, status, stats);
  return hipGetLastError();
}

}  // namespace fredec
