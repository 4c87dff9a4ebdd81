// Normalisation (Sect. 4.1, eq. idn) and base-model precomputation for the
// residual scan (eq. zpowrel): one workgroup per series.
//
// The base model's columns phi = (1, cos 2 pi f'_k t, sin 2 pi f'_k t) are
// replaced by an orthonormal basis q = L_A^{-1} phi (L_A the Cholesky factor
// of A = <phi phi^T>, Sect. 3) and the data by the base-model residual
// r_b = x~ - q . a_b with a_b = L_A^{-1} <x~ phi>.  The statistic is unchanged
// (the same column space and the same residual), but the scan then needs no
// triangular solve per frequency and its sums are better conditioned:
//   U = <q psi>, S = <psi psi^T> - U^T U, h = <r_b psi>,
//   l_{m+1} = l_m - h^T S^{-1} h,  l_m = D - |a_b|^2,  psi = (cos, sin)(2 pi f t).
#include "fredec_internal.h"

namespace fredec {

namespace {

constexpr int SUMS = 4;  // most values of one block reduction

__global__ __launch_bounds__(BLOCK) void prep_kernel(const SeriesIn* __restrict__ sin_, SeriesHdr* __restrict__ hdr,
                                                     const double* __restrict__ t, const double* __restrict__ x,
                                                     const double* __restrict__ w, double* __restrict__ tau,
                                                     double* __restrict__ xt, double* __restrict__ wt,
                                                     double* __restrict__ rec, double* __restrict__ phi,
                                                     float* __restrict__ g32, double* __restrict__ aux,
                                                     _Float16* __restrict__ b16, int flags) {
  __shared__ double sh[SUMS * BLOCK];
  __shared__ double gram[MAXKP * (MAXKP + 1) / 2];
  __shared__ double Lsh[MAXK * (MAXK + 1) / 2];
  __shared__ double invd[MAXK];
  __shared__ double ab[MAXK];
  __shared__ int status_sh;
  const int tid = threadIdx.x;
  const SeriesIn& si = sin_[blockIdx.x];
  SeriesHdr& h = hdr[blockIdx.x];
  const int64_t N = si.N;
  const double* ts = t + si.soff;
  const double* xs = x + si.soff;
  const double* ws = w + si.soff;
  double* taus = tau + si.soff;
  double* xts = xt + si.soff;
  double* wts = wt + si.soff;
  const bool with_base = (flags & PREP_BASE) != 0;

  // pass 1: sum of weights and input validity (Sect. 2: w_i > 0)
  double v1[2] = {0.0, 0.0};
  for (int64_t i = tid; i < N; i += BLOCK) {
    const double wi = ws[i], ti = ts[i], xi = xs[i];
    v1[0] += wi;
    const bool ok = (wi > 0.0) && isfinite(wi) && isfinite(ti) && isfinite(xi);
    v1[1] += ok ? 0.0 : 1.0;
  }
  block_sum(v1, sh);
  int status = 0;
  if (v1[1] != 0.0 || !(v1[0] > 0.0) || !isfinite(v1[0])) status = FREDEC_EWEIGHT;
  const double W = v1[0];

  // pass 2: weighted means of t and x
  double v2[2] = {0.0, 0.0};
  for (int64_t i = tid; i < N; i += BLOCK) {
    const double wi = ws[i] / W;
    v2[0] += wi * ts[i];
    v2[1] += wi * xs[i];
  }
  block_sum(v2, sh);
  const double tbar = v2[0], xbar = v2[1];

  // pass 3: second moments
  double v3[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = tid; i < N; i += BLOCK) {
    const double wi = ws[i] / W;
    const double ta = ts[i] - tbar, d = xs[i] - xbar;
    v3[0] += wi * ta * ta;
    v3[1] += wi * d * d;
    v3[2] += wi * xs[i] * xs[i];
    v3[3] += wi * ts[i] * ts[i];
  }
  block_sum(v3, sh);
  const double var_t = v3[0], sx2 = v3[1];
  if (status == 0 && (sx2 <= 1e-28 * v3[2] || var_t <= 1e-28 * v3[3])) status = FREDEC_EDEGEN;
  const double sx = sqrt(sx2);
  const double T_eff = sqrt(4.0 * M_PI * var_t);

  // pass 4: normalised series and, for scans, the base columns phi
  const int KP = si.KP;
  const int K = KP - 1;
  const int m = si.m;
  for (int64_t i = tid; i < N; i += BLOCK) {
    const double wi = ws[i] / W;
    const double ta = ts[i] - tbar;
    const double xi = (xs[i] - xbar) / sx;
    taus[i] = ta;
    xts[i] = xi;
    wts[i] = wi;
    if (with_base) {
      double* ph = phi + si.phi_off + i * KP;
      ph[0] = 1.0;
      for (int k = 0; k < m; ++k) {
        double s, c;
        sincos_rev(si.base_f[k] * ta, s, c);
        ph[1 + 2 * k] = c;
        ph[2 + 2 * k] = s;
      }
      ph[KP - 1] = xi;
    }
  }
  if (!with_base) {
    if (tid == 0) {
      h.T_eff = T_eff;
      h.stats[0] = tbar;
      h.stats[1] = xbar;
      h.stats[2] = sx;
      h.stats[3] = var_t;
      h.stats[4] = T_eff;
      h.stats[5] = W;
      h.status = status;
    }
    return;
  }
  __syncthreads();

  // Gram of the columns (1, cos f'_k, sin f'_k, x~): base normal matrix A,
  // right-hand side g_b (last row) and D = <x~^2> (last diagonal entry), on
  // float64 MFMA: the lower 16x16 tiles of the KP x KP Gram are dealt to the
  // four waves, each tile accumulated over all samples four at a time
  // (lane (c16, kq): column c16 of the tile's row / column block at sample
  // i0 + kq; D[r][c] in lane c + 16 (r % 4), register r / 4).
  {
    typedef double v4d __attribute__((ext_vector_type(4)));
    const int lane = tid & 63, wave = tid >> 6;
    const int c16 = lane & 15, kq = lane >> 4;
    const int nbk = (KP + 15) / 16;
    const int ntiles = nbk * (nbk + 1) / 2;
    const double* phs = phi + si.phi_off;
    for (int tl = wave; tl < ntiles; tl += BLOCK / 64) {
      int b1 = 0;
      while ((b1 + 1) * (b1 + 2) / 2 <= tl) ++b1;
      const int b2 = tl - b1 * (b1 + 1) / 2;
      const int ca = 16 * b1 + c16, cb = 16 * b2 + c16;
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
      for (int64_t i0 = 0; i0 < N; i0 += 4) {
        const int64_t i = i0 + kq;
        const bool in = i < N;
        const double av = (in && ca < KP) ? phs[i * KP + ca] : 0.0;
        const double bv = (in && cb < KP) ? wts[i] * phs[i * KP + cb] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * b1 + kq + 4 * v;
        const int c = 16 * b2 + c16;
        if (r < KP && c <= r) gram[r * (r + 1) / 2 + c] = acc[v];
      }
    }
  }
  __syncthreads();

  // Cholesky A = L L^T (Sect. 3), column by column: the pivot by thread 0,
  // the entries below it by one thread each.
  __shared__ int bad_sh;
  if (tid == 0) bad_sh = 0;
  __syncthreads();
  for (int j = 0; j < K; ++j) {
    if (tid == 0) {
      double d = gram[j * (j + 1) / 2 + j];
      for (int k = 0; k < j; ++k) d -= Lsh[j * (j + 1) / 2 + k] * Lsh[j * (j + 1) / 2 + k];
      if (!(d > PIVOT_TOL * gram[j * (j + 1) / 2 + j])) {
        bad_sh = 1;
      } else {
        const double ljj = sqrt(d);
        Lsh[j * (j + 1) / 2 + j] = ljj;
        invd[j] = 1.0 / ljj;
      }
    }
    __syncthreads();
    if (bad_sh) break;
    for (int i = j + 1 + tid; i < K; i += BLOCK) {
      double v = gram[i * (i + 1) / 2 + j];
      for (int k = 0; k < j; ++k) v -= Lsh[i * (i + 1) / 2 + k] * Lsh[j * (j + 1) / 2 + k];
      Lsh[i * (i + 1) / 2 + j] = v * invd[j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (status == 0 && bad_sh) status = FREDEC_ESINGULAR;
    // a_b = L^{-1} g_b, l_m = D - a_b.a_b
    double lm = 0.0;
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
      h.W1 = gram[0];
      lm = gb[K] - aa;
    }
    if (status == 0 && N - 3 * m - 4 <= 0) status = FREDEC_EDOF;
    h.l_m = lm;
    h.NH = static_cast<double>(N - 3 * m - 4);
    h.T_eff = T_eff;
    h.stats[0] = tbar;
    h.stats[1] = xbar;
    h.stats[2] = sx;
    h.stats[3] = var_t;
    h.stats[4] = T_eff;
    h.stats[5] = W;
    h.status = status;
    status_sh = status;
  }
  __syncthreads();
  if (status_sh != 0) return;

  // pass 5: orthonormal columns q = L^{-1} phi (in place) and residual r_b;
  // operand records for the scan kernels
  const int P = rec_stride(KP);
  const int G32W = 16 * si.NT;
  double gmax = 0.0;  // max |w~ q_k| (scale of the float16 operand)
  for (int64_t i = tid; i < N; i += BLOCK) {
    double* ph = phi + si.phi_off + i * KP;
    const double wi = wts[i];
    double r = ph[KP - 1];
    for (int k = 0; k < K; ++k) {
      double v = ph[k];
      for (int j = 0; j < k; ++j) v -= Lsh[k * (k + 1) / 2 + j] * ph[j];
      v *= invd[k];
      ph[k] = v;
      r -= v * ab[k];
      gmax = fmax(gmax, fabs(wi * v));
    }
    ph[KP - 1] = r;
    const double ta = taus[i];
    if (flags & PREP_REC64) {
      double* q = rec + si.rec_off + i * P;
      double rs, rc;
      sincos_rev(si.rot_step * ta, rs, rc);
      q[0] = ta;
      q[1] = rc;
      q[2] = rs;
      for (int k = 0; k < KP; ++k) q[3 + k] = wi * ph[k];
      double s1, c1;
      sincos_rev(si.df * ta, s1, c1);
      q[KP + 3] = c1;
      q[KP + 4] = s1;
    }
    if (flags & si.outputs & PREP_G32) {
      float* g = g32 + si.g32_off + i * G32W;
      for (int k = 0; k < K; ++k) g[k] = static_cast<float>(wi * ph[k]);
      // column K (never read by the MFMA kernel, whose padding columns only
      // produce unused sums) carries w~ for the VALU kernel's <cos^2>, <cos sin>
      g[K] = static_cast<float>(wi);
      for (int k = K + 1; k < G32W; ++k) g[k] = 0.0f;
    }
    if (flags & si.outputs & PREP_AUX) {
      double* a = aux + si.aux_off + i * AUX_STRIDE;
      double rs, rc, s1, c1;
      sincos_rev(si.rot_tile * ta, rs, rc);
      sincos_rev(si.df * ta, s1, c1);
      a[0] = ta;
      a[1] = rc;
      a[2] = rs;
      a[3] = wi;
      a[4] = wi * r;
      a[5] = 0.0;
      a[6] = c1;
      a[7] = s1;
    }
  }
  if (!(flags & si.outputs & PREP_F16)) return;

  // pass 6: split float16 operand of the MFMA scan, B = S w~ q_k = hi + lo
  // (both float16, lo = the float32 remainder), S = 2^e with max |B| in
  // (2^13, 2^14] so that low parts stay clear of the float16 subnormals.
  // Layout: per step g of 32 samples and column tile nt, the high part then
  // the low part, each 64 lanes x 8 halves; lane L holds column
  // 16 nt + L % 16 at samples 32 g + 8 (L / 16) + e, e < 8 (zero beyond N
  // and beyond column K).
  {
    double mx[1] = {gmax};
    __syncthreads();
    sh[tid] = mx[0];
    __syncthreads();
    for (int o = BLOCK / 2; o > 0; o >>= 1) {
      if (tid < o) sh[tid] = fmax(sh[tid], sh[tid + o]);
      __syncthreads();
    }
    gmax = sh[0];
    __syncthreads();
  }
  int ex = 0;
  if (gmax > 0.0) (void)frexp(gmax, &ex);  // gmax in [2^(ex-1), 2^ex)
  const double S = gmax > 0.0 ? ldexp(1.0, 14 - ex) : 1.0;
  if (tid == 0) h.b16_inv = 1.0 / S;
  const int NT = si.NT;
  const int64_t n_vec = b16_vectors(N, NT) / 2;  // (step, tile, lane) entries
  const double* phs5 = phi + si.phi_off;
  _Float16* bser = b16 + si.b16_off * 8;
  for (int64_t e = tid; e < n_vec; e += BLOCK) {
    const int L = static_cast<int>(e & 63);
    const int64_t gt = e >> 6;  // g * NT + nt
    const int nt = static_cast<int>(gt % NT);
    const int col = 16 * nt + (L & 15);
    const int64_t i0 = (gt / NT) * 32 + 8 * (L >> 4);
    _Float16* hi = bser + ((gt * 2) * 64 + L) * 8;
    _Float16* lo = hi + 64 * 8;
    for (int k = 0; k < 8; ++k) {
      const int64_t i = i0 + k;
      const double v = (i < N && col < K) ? S * wts[i] * phs5[i * KP + col] : 0.0;
      const _Float16 vh = static_cast<_Float16>(v);
      hi[k] = vh;
      lo[k] = static_cast<_Float16>(v - static_cast<double>(vh));
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

hipError_t launch_prep(hipStream_t st, int n_series, const SeriesIn* sin, SeriesHdr* hdr, const double* t,
                       const double* x, const double* w, double* tau, double* xt, double* wt, double* rec,
                       double* phi, float* g32, double* aux, void* b16, int flags) {
  if (n_series <= 0) return hipSuccess;
  prep_kernel<<<n_series, BLOCK, 0, st>>>(sin, hdr, t, x, w, tau, xt, wt, rec, phi, g32, aux,
                                          static_cast<_Float16*>(b16), flags);
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
