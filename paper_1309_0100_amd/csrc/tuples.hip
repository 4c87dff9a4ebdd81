// Tuple statistics z_n(f_1..f_n) (eq. zpow), their local refinement by
// Gauss-Newton steps (Sect. 3, eq. lsqf) and the adjoint gradient.
//
// tuple_gram_kernel: one workgroup per tuple builds the weighted Gram matrix
//   G = sum_i w~_i phi(t_i) phi(t_i)^T
// of on-the-fly generated columns on float64 MFMA (v_mfma_f64_16x16x4_f64):
//   forward columns  1, cos 2 pi f_k t, sin 2 pi f_k t (k = 1..n), x~
//   GN columns       the forward ones, then t' cos 2 pi f_k t, t' sin 2 pi f_k t
//                    (t' = t / sigma_t): the t-weighted averages from which the
//                    Fisher matrix Q_f of the frequencies follows (eqs. avrg1, avrg2).
// Each lane of an MFMA step owns one (column, sample) pair; A = B = sqrt(w~)
// * column values, so D accumulates the Gram block by block (lower triangle
// of 16x16 blocks only).  The sin/cos of each (frequency, sample) is
// evaluated once per step by one lane and shared through LDS.
// tuple_solve_kernel: one thread per tuple, float64: Cholesky of the model
// block, l, theta*, z, and the Gauss-Newton step with the step control shared
// with the oracle (clamp, accept/halve, tolerance).
// tuple_gram_lanes_kernel<n, L>: the forward Gram of tuples of exactly
// n <= 6 frequencies on the VALU, L lanes per tuple (each 1/L of the
// samples): every sin/cos is evaluated once, only the lower triangle
// (C(C+1)/2 multiply-adds per sample, C = 2n + 2) is accumulated, and the L
// partial Gram matrices are added with cross-lane permutations.  For these
// sizes this does less work than the MFMA kernel, whose 16-column blocks are
// mostly padding (float64 MFMA and float64 VALU have the same peak rate on
// this chip).  L is
// chosen per launch so that a group of tuples fills the GPU.
// tuple_adjoint_kernel (any n, one wavefront per tuple, samples over lanes)
// and tuple_adjoint_lanes_kernel<n, L> (n <= 6, L lanes per tuple): recompute
// the trig terms, the residual r = x~ - Phi theta* and <r J_k>, <J_k^2>
// (J_k = d mu / d f_k), reduced across lanes.
#include <algorithm>

#include "fredec_internal.h"
#include "fredec_tuples_internal.h"

namespace fredec {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// One workgroup per tuple; its four wavefronts take every fourth step of eight
// samples and add their partial Gram matrices in wave order at the end (short
// workgroups, so that the last round of a launch leaves little of the GPU
// idle).  Per step of eight samples, lane (c8, s8) first evaluates cos and
// sin of the frequencies c8, c8 + 8, ... at sample s8 (one float64 sin/cos
// pair per frequency and sample) and writes the columns they make (cos, sin,
// and in the Gauss-Newton mode t' cos, t' sin), each times sqrt(w~) of the
// sample, into a wave-private LDS table of the eight samples' column values
// (the columns 1 and x~ by lane c8 = 0, the padding columns zero), so that no
// operand needs a weight multiply; then, for each half of four samples, lane
// (c16, kq) reads the value of its column 16 b + c16 at sample kq for every
// 16-column block b, and the wave accumulates the lower-triangle blocks of
// the Gram on float64 MFMA.
//
// Column layout.  TV = 0: the blocks hold the Gram's own column order
// (1, cos/sin pairs, x~, t' cos/sin pairs), padded to 16 NB.  TV > 0: the
// blocks hold only the trigonometric columns (the cos/sin pairs, then the
// t' pairs) and TV extra columns, 1, x~ and the trigonometric columns past
// 16 NB, are accumulated against every column on the VALU (TV multiply-adds
// per block and sample, summed over the sample lanes and the waves at the
// end).  The host picks TV > 0 where it saves issue time: a 16x16x4 float64
// MFMA costs that of 16 float64 multiply-adds.
template <int NB, int TV>
__global__ __launch_bounds__(BLOCK) void tuple_gram_kernel(const TupleDesc* __restrict__ desc,
                                                           const int32_t* __restrict__ order,
                                                           int /* n_order: one block per tuple */,
                                                           const TupleCommon* __restrict__ com,
                                                           const double* __restrict__ tau, const double* __restrict__ xt,
                                                           const double* __restrict__ wt,
                                                           const double* __restrict__ ftry,
                                                           const TupleState* __restrict__ state,
                                                           double* __restrict__ gram, int mode) {
  // frequencies per lane (eight per pass): n <= 8 NB - 1 (TV = 0) or
  // 2 n <= 16 NB + 4
  constexpr int NRMAX = TV == 0 ? NB : NB + 1;
  constexpr int XO = 16 * NB;             // first extra slot (TV > 0)
  constexpr int CW = XO + (TV > 0 ? 16 : 0);
  constexpr int TSZ = 512;                // samples per block-wide staging tile
  constexpr int NW = BLOCK / 64;
  constexpr int SP = 8;                   // samples per step
  __shared__ double colv[NW][SP][CW];     // per wave: the column values of the step's samples
  __shared__ double stage[3][TSZ];        // tau, x~, w~ of the tile
  __shared__ double2 tab[TRIG_TAB];
  // one tuple per block (the launch has n_order blocks)
  const int ti = order[blockIdx.x];
  if (state[ti].done) return;  // uniform over the block
  trig_table_fill(tab);
  const int wb = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const TupleDesc& d = desc[ti];
  const int n = d.n;
  const bool gn = mode == TUPLE_GN;
  const int C = gn ? 4 * n + 2 : 2 * n + 2;
  const int T = C - 2;       // trigonometric columns
  const int K = 2 * n + 1;   // the x~ column; the t' columns follow it
  const double* f = ftry + d.foff;
  const int c16 = lane & 15;  // MFMA operands: column within the block
  const int kq = lane >> 4;   // and sample within the four of an MFMA
  const int c8 = lane & 7;    // trigonometry: frequency c8 + 8 r
  const int s8 = lane >> 3;   // at sample s8 of the step
  const int nr = (n + 7) >> 3;
  // Gram column of trigonometric column q (cos/sin pairs, then t' pairs)
  auto gcol = [&](int q) { return q < 2 * n ? q + 1 : q + 2; };
  // table slot of trigonometric column q
  auto tslot = [&](int q) { return TV == 0 ? gcol(q) : (q < XO ? q : q + 2); };
  // frequency, and the slots of its cos/sin and t' cos/sin pairs (a pair
  // never straddles 16 NB: both are even)
  double fk[NRMAX];
  int sl[NRMAX], st[NRMAX];
#pragma unroll
  for (int r = 0; r < NRMAX; ++r) {
    const int kk = c8 + 8 * r;
    fk[r] = kk < n ? f[kk] : 0.0;
    sl[r] = kk < n ? tslot(2 * kk) : 0;
    st[r] = kk < n ? tslot(2 * n + 2 * kk) : 0;
  }
  const int slot1 = TV == 0 ? 0 : XO;
  const int slotx = TV == 0 ? K : XO + 1;
  double(*cw)[CW] = colv[wb];
  for (int e = lane; e < SP * CW; e += 64) cw[e / CW][e % CW] = 0.0;  // padding stays zero
  __builtin_amdgcn_wave_barrier();
  const double inv_sig = com->inv_sigma_t;
  constexpr int NTILE = NB * (NB + 1) / 2;
  v4d acc[NTILE];
#pragma unroll
  for (int q = 0; q < NTILE; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
  constexpr int TVA = TV > 0 ? TV : 1;
  double xacc[TVA][NB + 1];
#pragma unroll
  for (int j = 0; j < TVA; ++j)
#pragma unroll
    for (int b = 0; b <= NB; ++b) xacc[j][b] = 0.0;
  const int64_t N = com->N;
  for (int64_t t0 = 0; t0 < N; t0 += TSZ) {
    const int ns = N - t0 < TSZ ? static_cast<int>(N - t0) : TSZ;
    __syncthreads();
    for (int k = threadIdx.x; k < TSZ; k += BLOCK) {
      const bool in = k < ns;
      stage[0][k] = in ? tau[t0 + k] : 0.0;
      stage[1][k] = in ? xt[t0 + k] : 0.0;
      stage[2][k] = in ? sqrt(wt[t0 + k]) : 0.0;  // sqrt(w~): folded into every column value
    }
    __syncthreads();
    // the block's waves take every fourth step of eight samples: one sin/cos
    // pass over eight frequencies x eight samples, then two MFMA steps of four
    for (int s0 = SP * wb; s0 < ns; s0 += SP * NW) {
      {
        const int il = s0 + s8;  // beyond ns the staged values are 0
        const double ta = stage[0][il];
        const double sw = stage[2][il];
        const double tt = ta * inv_sig;
#pragma unroll
        for (int r = 0; r < NRMAX; ++r) {
          if (r < nr) {
            const int kk = c8 + 8 * r;
            double sv, cv;
            sincos_tab(fk[r] * ta, tab, sv, cv);
            cv *= sw;
            sv *= sw;
            if (kk < n) {
              cw[s8][sl[r]] = cv;
              cw[s8][sl[r] + 1] = sv;
              if (gn) {
                cw[s8][st[r]] = cv * tt;
                cw[s8][st[r] + 1] = sv * tt;
              }
            }
          }
        }
        if (c8 == 0) {
          cw[s8][slot1] = sw;
          cw[s8][slotx] = stage[1][il] * sw;
        }
      }
      __builtin_amdgcn_wave_barrier();
      double a[2][NB], ax[2], ex[2][TVA];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int row = 4 * u + kq;
#pragma unroll
        for (int b = 0; b < NB; ++b) a[u][b] = cw[row][16 * b + c16];
        if constexpr (TV > 0) {
          ax[u] = cw[row][XO + c16];
#pragma unroll
          for (int j = 0; j < TV; ++j) ex[u][j] = cw[row][XO + j];
        }
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        double bw[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) bw[b] = a[u][b];
        if constexpr (TV > 0) {
#pragma unroll
          for (int j = 0; j < TV; ++j) {
            const double ej = ex[u][j];
#pragma unroll
            for (int b = 0; b < NB; ++b) xacc[j][b] = __builtin_fma(ej, a[u][b], xacc[j][b]);
            xacc[j][NB] = __builtin_fma(ej, ax[u], xacc[j][NB]);
          }
        }
        int q = 0;
#pragma unroll
        for (int b1 = 0; b1 < NB; ++b1)
#pragma unroll
          for (int b2 = 0; b2 <= b1; ++b2) {
            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][b1], bw[b2], acc[q], 0, 0, 0);
            ++q;
          }
      }
    }
  }
  // The waves' partial sums, added in wave order through LDS one 16x16 block
  // at a time (the accumulators are only stored, which keeps them in the
  // registers the MFMA writes): thread (rk, rl) sums register rk of lane rl
  // over the waves and writes that Gram entry.
  // D[i][j] of block (b1, b2) sits in lane j + 16 (i % 4), register i / 4.
  double* red = &stage[0][0];  // [NW][4][64]
  static_assert(3 * TSZ >= NW * 4 * 64, "reduction scratch");
  double* G = gram + d.goff;
  const int64_t gs = d.gs;
  const int rk = threadIdx.x >> 6, rl = threadIdx.x & 63;
  const int rc16 = rl & 15, rkq = rl >> 4;
  auto sum_waves = [&]() {
    double v = red[rk * 64 + rl];
#pragma unroll
    for (int w = 1; w < NW; ++w) v += red[(w * 4 + rk) * 64 + rl];
    return v;
  };
  int q = 0;
#pragma unroll
  for (int b1 = 0; b1 < NB; ++b1)
#pragma unroll
    for (int b2 = 0; b2 <= b1; ++b2) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 4; ++k) red[(wb * 4 + k) * 64 + lane] = acc[q][k];
      __syncthreads();
      const double v = sum_waves();
      const int r = 16 * b1 + rkq + 4 * rk;
      const int c = 16 * b2 + rc16;
      if (TV == 0) {
        if (r < C && c <= r) G[(r * (r + 1) / 2 + c) * gs] = v;
      } else if (r < T && c <= r) {
        const int gr = gcol(r), gc = gcol(c);
        G[(gr * (gr + 1) / 2 + gc) * gs] = v;
      }
      ++q;
    }
  if constexpr (TV > 0) {
    // <w~ e_j col> for extra column j against the block column 16 b + c16
    // (b < NB) or extra column c16 (b = NB): summed over the waves and the
    // four sample lanes, four (j, b) pairs at a time
    auto xcol = [&](int j) { return j == 0 ? 0 : j == 1 ? K : gcol(XO + j - 2); };
    constexpr int NX = TV * (NB + 1);
#pragma unroll
    for (int e = 0; e < NX; e += 4) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 4; ++k)
        red[(wb * 4 + k) * 64 + lane] = e + k < NX ? xacc[(e + k) / (NB + 1)][(e + k) % (NB + 1)] : 0.0;
      __syncthreads();
      const int ex = e + rk;
      if (ex < NX && rl < 16) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll
          for (int g = 0; g < 4; ++g) v += red[(w * 4 + rk) * 64 + 16 * g + rl];
        const int j = ex / (NB + 1), b = ex % (NB + 1);
        const int gj = xcol(j);
        int gc = -1;
        if (b < NB) {
          if (16 * b + rl < T) gc = gcol(16 * b + rl);
        } else if (rl < TV) {
          gc = xcol(rl);
          if (gc > gj) gc = -1;  // each extra pair once
        }
        if (gc >= 0) {
          const int r = gj > gc ? gj : gc, c = gj > gc ? gc : gj;
          G[(r * (r + 1) / 2 + c) * gs] = v;
        }
      }
    }
  }
}


constexpr int pidx(int r, int c) { return r * (r + 1) / 2 + c; }

// The forward solve of the tuples of a block from their Gram matrices in LDS
// (gsh[q TPB + j] = packed lower element q, column order 1, cos/sin pairs,
// x~, of the block's tuple j): the steps of tuple_solve_kernel's forward mode
// (merged-frequency test, l_0, Cholesky with the relative pivot test,
// a = L^{-1} g, l = D - a.a, the acceptance test, theta* = L^{-T} a), then
// the tuple is done.  Sixteen lanes (one DPP row) take one tuple: lane i
// holds row i of the augmented matrix [[G, g], [g^T, D]] (C = 2 NF + 2 rows),
// whose Cholesky factor has a = L^{-1} g as its last row.  Column j: lane j
// forms the pivot, its row is broadcast to the other lanes, each lane below
// finishes its own element; theta* = L^{-T} a runs from the last column back,
// each step one 16-lane sum of L_kj theta_k.  Every lane of the block runs
// the same instruction stream (no divergence around the cross-lane steps);
// only the stores are predicated.
template <int NF, int TPB>
__device__ __forceinline__ void fwd_solve_block(const double* gsh, const TupleDesc* __restrict__ desc,
                                                const int32_t* __restrict__ order, int n_order,
                                                const TupleCommon* __restrict__ com,
                                                const double* __restrict__ ftry, double* __restrict__ facc,
                                                double* __restrict__ theta, TupleState* __restrict__ state) {
  constexpr int C = 2 * NF + 2;  // rows of the augmented matrix
  constexpr int K = C - 1;       // the data row
  static_assert(C <= 16, "one DPP row per tuple");
  const int i = threadIdx.x & 15;
  const int lane = threadIdx.x & 63;
  for (int p = 0; p < (TPB + 15) / 16; ++p) {
    const int tb = p * 16 + (threadIdx.x >> 4);
    const int g2 = blockIdx.x * TPB + tb;
    const bool valid = tb < TPB && g2 < n_order;
    const int t2 = valid ? order[g2] : 0;
    const bool live = valid && !state[t2].done;
    const int tbc = tb < TPB ? tb : 0;
    // row i (zero beyond the matrix)
    double r[C];
#pragma unroll
    for (int k = 0; k < C; ++k) r[k] = (i < C && k <= i) ? gsh[((i * (i + 1)) / 2 + k) * TPB + tbc] : 0.0;
    const double g00 = __shfl(r[0], 0, 16);
    const double l0 = r[K] - r[0] * r[0] / g00;  // on lane K
    bool own_ok = true;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      double piv = r[j];
#pragma unroll
      for (int k = 0; k < j; ++k) piv -= r[k] * r[k];
      if (i == j) {
        own_ok = piv > PIVOT_TOL * r[j];
        r[j] = sqrt(own_ok ? piv : 1.0);
      }
      double q[C];
#pragma unroll
      for (int k = 0; k <= j; ++k) q[k] = __shfl(r[k], j, 16);
      const double inv = 1.0 / q[j];
      if (i > j) {
        double v = r[j];
#pragma unroll
        for (int k = 0; k < j; ++k) v -= r[k] * q[k];
        r[j] = v * inv;
      }
    }
    // l = D - a.a on lane K
    double aa = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) aa += r[k] * r[k];
    const double l = r[K] - aa;
    const uint64_t bal = __ballot(own_ok);
    const bool chol_ok = ((bal >> (lane & 48)) & 0xFFFFull) == 0xFFFFull;
    // theta* = L^{-T} a: lane i keeps theta_i
    double th = 0.0;
#pragma unroll
    for (int j = K - 1; j >= 0; --j) {
      const double c = (i > j && i < K) ? r[j] * th : 0.0;
      const double sum = group_sum<16>(c);
      const double aj = __shfl(r[j], K, 16);
      if (i == j) th = (aj - sum) / r[j];
    }
    // decision on lane K, broadcast to the tuple's lanes
    int accept = 0;
    if (i == K && live) {
      const TupleDesc& d = desc[t2];
      TupleState& S = state[t2];
      const double* ft = ftry + d.foff;
      double f[NF];
#pragma unroll
      for (int k = 0; k < NF; ++k) f[k] = ft[k];
      const double T = com->T_eff;
      bool degen = false;
#pragma unroll
      for (int k = 0; k < NF; ++k)
#pragma unroll
        for (int m = k + 1; m < NF; ++m) degen |= fabs(f[k] - f[m]) * T < MASK_WIDTH;
      const bool ok = chol_ok && !degen;
      S.done = 1;
      if (ok && l <= S.l_acc * (1.0 + ACCEPT_RTOL)) {
        accept = 1;
        double* fa = facc + d.foff;
#pragma unroll
        for (int k = 0; k < NF; ++k) fa[k] = f[k];
        S.has_acc = 1;
        S.l_acc = l;
        S.l0 = l0;
        S.halvings = 0;
      } else if (!S.has_acc) {
        S.flags = FREDEC_FLAG_DEGENERATE;  // the start point itself is degenerate
      }
    }
    accept = __shfl(accept, K, 16);
    if (accept && i < K) theta[desc[t2].thoff + i] = th;
  }
}

// sin/cos(2 pi p) for the lane-group kernels: float64 (sincos_tab with the
// block's table) or, in the reduced-precision form, the float64 phase
// reduction p - rint(p) followed by the hardware float32 sin/cos of the
// reduced phase (v_sin_f32 and v_cos_f32 take their argument in
// revolutions), widened to float64.
template <bool F32>
__device__ __forceinline__ void tuple_sincos(double p, const double2* __restrict__ tab, double& s, double& c) {
  if constexpr (F32) {
    const float r = static_cast<float>(p - __builtin_rint(p));
    s = static_cast<double>(__builtin_amdgcn_sinf(r));
    c = static_cast<double>(__builtin_amdgcn_cosf(r));
  } else {
    sincos_tab(p, tab, s, c);
  }
}

// Whether Gram element (a, b) of the lane-group kernels is the <w sin_k^2> of
// a member, which the float64 form derives as <w> - <w cos_k^2> (eq. idn)
// instead of summing it.  The float32-trig form sums it: its hardware sin
// and cos satisfy cos^2 + sin^2 = 1 only to float32 accuracy, and the
// matrix must stay the Gram of the columns it was built from.
template <int NF, bool F32>
__device__ constexpr bool derived_sin2(int a, int b) {
  return !F32 && a == b && a >= 2 && a <= 2 * NF && a % 2 == 0;
}

// Whether a lane-group Gram kernel is held to 256 registers, two waves per
// SIMD: the float64 form at NF = 6, whose 99 summed Gram elements (eq. idn
// saves six) then fit with the sample loop unspilled (measured 19% faster
// than one wave per SIMD).  The float32-trig form sums all 105: held to 256
// registers it spills inside the sample loop.
template <int NF, bool F32>
__host__ __device__ constexpr bool lanes_two_waves() {
  return NF >= 6 && !F32;
}

// Whether packed element q = pidx(a, b) is such a derived <w sin_k^2>.
template <int NF, bool F32>
__device__ constexpr bool derived_sin2_at(int q) {
  for (int k = 0; k < NF; ++k)
    if (derived_sin2<NF, F32>(2 + 2 * k, 2 + 2 * k) && q == pidx(2 + 2 * k, 2 + 2 * k)) return true;
  return false;
}

// L lanes per tuple; the tuples of one launch all have NF frequencies.
template <int NF, int L, bool F32>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(lanes_two_waves<NF, F32>() ? 2 : 1)))
void tuple_gram_lanes_kernel(const TupleDesc* __restrict__ desc,
                                                                 const int32_t* __restrict__ order, int n_order,
                                                                 const TupleCommon* __restrict__ com,
                                                                 const double* __restrict__ tau,
                                                                 const double* __restrict__ xt,
                                                                 const double* __restrict__ wt,
                                                                 const double* __restrict__ ftry,
                                                                 TupleState* __restrict__ state,
                                                                 double* __restrict__ gram,
                                                                 double* __restrict__ facc,
                                                                 double* __restrict__ theta, int fuse) {
  constexpr int C = 2 * NF + 2;
  constexpr int NACC = C * (C + 1) / 2;
  __shared__ double2 tab[F32 ? 1 : TRIG_TAB];
  if constexpr (!F32) {
    trig_table_fill(tab);
    __syncthreads();
  }
  const int64_t gt = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  const int grp = static_cast<int>(gt / L);
  const int r = static_cast<int>(gt % L);
  const bool in_range = grp < n_order;
  const int ti = in_range ? order[grp] : 0;
  const bool live = in_range && !state[ti].done;
  double f[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) f[k] = live ? ftry[desc[ti].foff + k] : 0.0;
  double acc[NACC];
#pragma unroll
  for (int q = 0; q < NACC; ++q) acc[q] = 0.0;
  if (live) {
    const int64_t N = com->N;
    // the next sample's tau, w~, x~ are loaded while this one is processed,
    // except in the kernels held to 256 registers for two waves per SIMD
    // (there the three values would be spilled to scratch)
    constexpr bool PREFETCH = !lanes_two_waves<NF, F32>();
    double nta = 0.0, nwi = 0.0, nxi = 0.0;
    if (PREFETCH && r < N) {
      nta = tau[r];
      nwi = wt[r];
      nxi = xt[r];
    }
#pragma unroll 1
    for (int64_t i = r; i < N; i += L) {
      double ta, wi, xi;
      if constexpr (PREFETCH) {
        ta = nta;
        wi = nwi;
        xi = nxi;
        if (i + L < N) {
          nta = tau[i + L];
          nwi = wt[i + L];
          nxi = xt[i + L];
        }
      } else {
        ta = tau[i];
        wi = wt[i];
        xi = xt[i];
      }
      double phi[C];
      phi[0] = 1.0;
#pragma unroll
      for (int k = 0; k < NF; ++k) tuple_sincos<F32>(f[k] * ta, tab, phi[2 + 2 * k], phi[1 + 2 * k]);
      phi[C - 1] = xi;
#pragma unroll
      for (int a = 0; a < C; ++a) {
        const double wa = wi * phi[a];
        acc[pidx(a, 0)] += wa;
#pragma unroll
        for (int b = 1; b <= a; ++b)
          if (!derived_sin2<NF, F32>(a, b)) acc[pidx(a, b)] = __builtin_fma(wa, phi[b], acc[pidx(a, b)]);
      }
    }
  }
  // The L partial sums of the group are added (fixed order: deterministic)
  // and the block's Gram matrices go to LDS ([element][tuple of the block])
  // one element at a time, so that each accumulator is free once stored.
  constexpr int TPB = BLOCK / L;
  __shared__ double gsh[NACC * TPB];
  const int tb = threadIdx.x / L;
#pragma unroll
  for (int q = 0; q < NACC; ++q) {
    if (derived_sin2_at<NF, F32>(q)) continue;
    acc[q] = group_sum<L>(acc[q]);
    asm volatile("" : "+v"(acc[q]));  // complete each sum here: keeps the register count of the loop
    if (r == 0) gsh[q * TPB + tb] = acc[q];
  }
  // <w sin^2> = <w> - <w cos^2> (eq. idn) where it was not summed
  if (r == 0) {
#pragma unroll
    for (int k = 0; k < NF; ++k)
      if (derived_sin2<NF, F32>(2 + 2 * k, 2 + 2 * k))
        gsh[pidx(2 + 2 * k, 2 + 2 * k) * TPB + tb] = acc[0] - acc[pidx(1 + 2 * k, 1 + 2 * k)];
  }
  __syncthreads();
  if (!fuse) {
    // the Gram matrices to memory, element-major across the block's tuples
    for (int e = threadIdx.x; e < NACC * TPB; e += BLOCK) {
      const int q = e / TPB, j = e % TPB;
      const int g2 = blockIdx.x * TPB + j;
      if (g2 >= n_order) continue;
      const int t2 = order[g2];
      if (state[t2].done) continue;
      gram[desc[t2].goff + static_cast<int64_t>(q) * desc[t2].gs] = gsh[e];
    }
    return;
  }
  // the solve of the forward mode: the block solves its tuples, sixteen
  // lanes a tuple (nothing goes to memory but theta*, the state and the
  // accepted frequencies)
  fwd_solve_block<NF, TPB>(gsh, desc, order, n_order, com, ftry, facc, theta, state);
}

// Element (r, c), r >= c, of a packed lower-triangular matrix stored with
// element stride gs.
__device__ __forceinline__ double& P_(double* G, int r, int c, int64_t gs) { return G[(r * (r + 1) / 2 + c) * gs]; }

// In-place Cholesky of the leading K x K block of the packed lower matrix G.
// The solve runs one thread per tuple, one wavefront per SIMD: its loops
// are latency-bound, so independent rows (columns) are taken W at a time,
// which keeps W load and multiply-add chains in flight; each sum keeps the
// order of the plain loop.

// Rows i .. i + W - 1 of column j of the Cholesky factor.
template <int W>
__device__ __forceinline__ void chol_rows(double* G, int i, int j, double inv, int64_t gs) {
  double v[W];
#pragma unroll
  for (int w = 0; w < W; ++w) v[w] = P_(G, i + w, j, gs);
  for (int k = 0; k < j; ++k) {
    const double ljk = P_(G, j, k, gs);
#pragma unroll
    for (int w = 0; w < W; ++w) v[w] -= P_(G, i + w, k, gs) * ljk;
  }
#pragma unroll
  for (int w = 0; w < W; ++w) P_(G, i + w, j, gs) = v[w] * inv;
}

__device__ bool chol_inplace(double* G, int K, int64_t gs) {
  for (int j = 0; j < K; ++j) {
    const double diag = P_(G, j, j, gs);
    double dsum = diag;
    for (int k = 0; k < j; ++k) dsum -= P_(G, j, k, gs) * P_(G, j, k, gs);
    if (!(dsum > PIVOT_TOL * diag)) return false;
    const double ljj = sqrt(dsum);
    const double inv = 1.0 / ljj;
    P_(G, j, j, gs) = ljj;
    int i = j + 1;
    for (; i + 4 <= K; i += 4) chol_rows<4>(G, i, j, inv, gs);
    for (; i < K; ++i) chol_rows<1>(G, i, j, inv, gs);
  }
  return true;
}

// Columns kb .. kb + W - 1 of V = L^{-1} P (P column k = -a_k <phi t' sin_k>
// + b_k <phi t' cos_k>, from the Gram rows of the t' columns).
template <int W>
__device__ __forceinline__ void v_cols(double* G, double* V, const double* th, int K, int n, int kb, int ts0,
                                       int64_t gs) {
  double ak[W], bk[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    ak[w] = th[1 + 2 * (kb + w)];
    bk[w] = th[2 + 2 * (kb + w)];
  }
  for (int j = 0; j < K; ++j) {
    double p[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int rc = ts0 + 2 * (kb + w);
      p[w] = -ak[w] * P_(G, rc + 1, j, gs) + bk[w] * P_(G, rc, j, gs);
    }
    for (int m = 0; m < j; ++m) {
      const double g = P_(G, j, m, gs);
#pragma unroll
      for (int w = 0; w < W; ++w) p[w] -= g * V[(m * n + kb + w) * gs];
    }
    const double inv = 1.0 / P_(G, j, j, gs);
#pragma unroll
    for (int w = 0; w < W; ++w) V[(j * n + kb + w) * gs] = p[w] * inv;
  }
}

// H entries (k, m .. m + W - 1) = <J'_k J'_m> - (V^T V)_km.
template <int W>
__device__ __forceinline__ void h_entries(double* G, const double* V, double* H, const double* th, int K, int n,
                                          int k, int m, int ts0, int64_t gs) {
  auto g = [&](int r1, int r2) { return r1 >= r2 ? P_(G, r1, r2, gs) : P_(G, r2, r1, gs); };
  const double ak = th[1 + 2 * k], bk = th[2 + 2 * k];
  const int kc = ts0 + 2 * k, ks = kc + 1;
  double jj[W];
#pragma unroll
  for (int w = 0; w < W; ++w) {
    const double am = th[1 + 2 * (m + w)], bm = th[2 + 2 * (m + w)];
    const int mc = ts0 + 2 * (m + w), ms = mc + 1;
    jj[w] = ak * am * g(ks, ms) - ak * bm * g(ks, mc) - bk * am * g(kc, ms) + bk * bm * g(kc, mc);
  }
  for (int j = 0; j < K; ++j) {
    const double vk = V[(j * n + k) * gs];
#pragma unroll
    for (int w = 0; w < W; ++w) jj[w] -= vk * V[(j * n + m + w) * gs];
  }
#pragma unroll
  for (int w = 0; w < W; ++w) H[(k * (k + 1) / 2 + m + w) * gs] = jj[w];
}

__global__ __launch_bounds__(BLOCK) void tuple_solve_kernel(const TupleDesc* __restrict__ desc,
                                                            const int32_t* __restrict__ order, int n_tuples,
                                                            const TupleCommon* __restrict__ com,
                                                            double* __restrict__ gram, double* __restrict__ scratch,
                                                            double* __restrict__ ftry, double* __restrict__ facc,
                                                            double* __restrict__ step, double* __restrict__ theta,
                                                            TupleState* __restrict__ state, int mode, int last) {
  const int oi = blockIdx.x * blockDim.x + threadIdx.x;
  if (oi >= n_tuples) return;
  const int ti = order[oi];
  const TupleDesc& d = desc[ti];
  TupleState& S = state[ti];
  if (S.done) return;
  const int n = d.n;
  const int K = 2 * n + 1;
  double* G = gram + d.goff;
  const int64_t gs = d.gs;
  double* ft = ftry + d.foff;
  double* fa = facc + d.foff;
  double* st = step + d.foff;
  double* th = theta + d.thoff;
  const double T = com->T_eff;
  // degenerate trial point: two frequencies merged
  bool degen = false;
  for (int k = 0; k < n; ++k)
    for (int l = k + 1; l < n; ++l) degen |= fabs(ft[k] - ft[l]) * T < MASK_WIDTH;
  // l_0 of the constant model and D from the Gram
  const double D = P_(G, K, K, gs);
  const double l0 = D - P_(G, K, 0, gs) * P_(G, K, 0, gs) / P_(G, 0, 0, gs);
  bool ok = !degen && chol_inplace(G, K, gs);
  double l = 0.0;
  if (ok) {
    // a = L^{-1} g in place on row K; l = D - a.a
    double aa = 0.0;
    for (int i = 0; i < K; ++i) {
      double v = P_(G, K, i, gs);
      for (int k = 0; k < i; ++k) v -= P_(G, i, k, gs) * P_(G, K, k, gs);
      v /= P_(G, i, i, gs);
      P_(G, K, i, gs) = v;
      aa += v * v;
    }
    l = D - aa;
  }
  const bool accept = ok && l <= S.l_acc * (1.0 + ACCEPT_RTOL);
  if (!accept) {
    if (!S.has_acc) {  // the start point itself is degenerate
      S.done = 1;
      S.flags = FREDEC_FLAG_DEGENERATE;
      return;
    }
    for (int k = 0; k < n; ++k) st[k] *= 0.5;
    if (++S.halvings > MAX_HALVINGS || last) {
      S.done = 1;
      return;
    }
    for (int k = 0; k < n; ++k) ft[k] = fa[k] + st[k];
    return;
  }
  // accepted: theta* = L^{-T} a
  for (int i = K - 1; i >= 0; --i) {
    double v = P_(G, K, i, gs);
    for (int k = i + 1; k < K; ++k) v -= P_(G, k, i, gs) * th[k];
    th[i] = v / P_(G, i, i, gs);
  }
  S.has_acc = 1;
  S.l_acc = l;
  S.l0 = l0;
  S.halvings = 0;
  for (int k = 0; k < n; ++k) fa[k] = ft[k];
  if (mode != TUPLE_GN) {
    S.done = 1;
    return;
  }
  // Gauss-Newton step on the frequencies: J'_k = t'(-a_k sin + b_k cos),
  // P = <phi J'>, JJ = <J' J'>, rJ = <x J'> - P^T theta, V = L^{-1} P,
  // H = JJ - V^T V, dnu = H^{-1} rJ, df = dnu / (2 pi sigma_t).
  const int ts0 = K + 1;  // first t' column
  double* V = scratch + d.soff;                      // K x n
  double* H = V + static_cast<int64_t>(K) * n * gs;  // packed n x n
  double* rJ = H + static_cast<int64_t>(n * (n + 1) / 2) * gs;  // n
  {
    int kb = 0;
    for (; kb + 4 <= n; kb += 4) v_cols<4>(G, V, th, K, n, kb, ts0, gs);
    for (; kb < n; ++kb) v_cols<1>(G, V, th, K, n, kb, ts0, gs);
  }
  for (int k = 0; k < n; ++k) {
    const double ak = th[1 + 2 * k], bk = th[2 + 2 * k];
    const int rc = ts0 + 2 * k, rs = ts0 + 2 * k + 1;
    // <x J'_k> - sum_j theta_j P_jk, with P recomputed
    double r = -ak * P_(G, rs, K, gs) + bk * P_(G, rc, K, gs);
    for (int j = 0; j < K; ++j) r -= th[j] * (-ak * P_(G, rs, j, gs) + bk * P_(G, rc, j, gs));
    rJ[k * gs] = r;
  }
  // <J'_k J'_m> from the packed lower Gram (row index >= column index)
  for (int k = 0; k < n; ++k) {
    int m = 0;
    for (; m + 4 <= k + 1; m += 4) h_entries<4>(G, V, H, th, K, n, k, m, ts0, gs);
    for (; m <= k; ++m) h_entries<1>(G, V, H, th, K, n, k, m, ts0, gs);
  }
  if (d.frozen) {
    // frozen frequencies: their J' columns leave the system (row and column
    // of H replaced by the identity's, right-hand side 0, so their step is 0
    // and the others solve the reduced system exactly)
    for (int k = 0; k < n; ++k) {
      if (!(d.frozen >> k & 1)) continue;
      rJ[k * gs] = 0.0;
      for (int m = 0; m < n; ++m) {
        const int i = k > m ? k : m, j = k > m ? m : k;
        H[(i * (i + 1) / 2 + j) * gs] = k == m ? 1.0 : 0.0;
      }
    }
  }
  bool hok = chol_inplace(H, n, gs);
  double big = 0.0;
  if (hok) {
    // solve H dnu = rJ (in place in rJ)
    for (int i = 0; i < n; ++i) {
      double v = rJ[i * gs];
      for (int k = 0; k < i; ++k) v -= H[(i * (i + 1) / 2 + k) * gs] * rJ[k * gs];
      rJ[i * gs] = v / H[(i * (i + 1) / 2 + i) * gs];
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = rJ[i * gs];
      for (int k = i + 1; k < n; ++k) v -= H[(k * (k + 1) / 2 + i) * gs] * rJ[k * gs];
      rJ[i * gs] = v / H[(i * (i + 1) / 2 + i) * gs];
    }
    const double scale = com->inv_two_pi_sigma_t;
    for (int k = 0; k < n; ++k) {
      st[k] = rJ[k * gs] * scale;
      big = fmax(big, fabs(st[k]) * T);
    }
  }
  if (!hok || big < GN_TOL) {
    S.done = 1;
    if (hok) S.flags |= FREDEC_FLAG_CONVERGED;
    return;
  }
  if (last) {  // no pass is left to evaluate the step
    S.done = 1;
    return;
  }
  if (big > GN_CLAMP)
    for (int k = 0; k < n; ++k) st[k] *= GN_CLAMP / big;
  for (int k = 0; k < n; ++k) ft[k] = fa[k] + st[k];
}

__global__ void tuple_finish_kernel(const TupleDesc* __restrict__ desc, int n_tuples,
                                    const TupleCommon* __restrict__ com, const TupleState* __restrict__ state,
                                    const double* __restrict__ facc, double* __restrict__ l_out,
                                    double* __restrict__ z_out, uint8_t* __restrict__ flags_out,
                                    double* __restrict__ f_out, const int8_t* __restrict__ members, int f_stride) {
  const int ti = blockIdx.x * BLOCK + threadIdx.x;
  if (ti >= n_tuples) return;
  const TupleDesc& d = desc[ti];
  const TupleState& S = state[ti];
  const int n = d.n;
  double l = S.has_acc ? S.l_acc : __builtin_nan("");
  double z;
  uint8_t fl = S.flags;
  if (!S.has_acc) {
    z = -__builtin_inf();
    fl |= FREDEC_FLAG_DEGENERATE;
  } else if (!(l > 0.0)) {
    z = __builtin_inf();
    fl |= FREDEC_FLAG_PERFECT;
  } else {
    const double NH = static_cast<double>(com->N - 3 * n - 1);
    z = 0.5 * NH * log(S.l0 / l);
  }
  if (l_out) l_out[ti] = l;
  if (z_out) z_out[ti] = z;
  if (flags_out) flags_out[ti] = fl;
  if (f_out) {
    if (members) {
      double* row = f_out + static_cast<int64_t>(ti) * f_stride;
      for (int k = 0; k < f_stride; ++k) row[k] = __builtin_nan("");
      for (int k = 0; k < n; ++k) row[members[d.foff + k]] = facc[d.foff + k];
    } else {
      for (int k = 0; k < n; ++k) f_out[d.foff + k] = facc[d.foff + k];
    }
  }
}

// Adjoint: <r J_k> and <J_k^2> with J_k = 2 pi t (-a_k sin 2 pi f_k t + b_k cos 2 pi f_k t),
// r = x~ - Phi theta*; dz/df_k = (N_H / l) <r J_k>, h_k = (N_H / l) <J_k^2>.
__global__ __launch_bounds__(BLOCK) void tuple_adjoint_kernel(const TupleDesc* __restrict__ desc,
                                                              const int32_t* __restrict__ order, int n_tuples,
                                                              const TupleCommon* __restrict__ com,
                                                              const double* __restrict__ tau,
                                                              const double* __restrict__ xt,
                                                              const double* __restrict__ wt,
                                                              const double* __restrict__ f,
                                                              const double* __restrict__ theta,
                                                              const TupleState* __restrict__ state,
                                                              double* __restrict__ dzdf, double* __restrict__ hout) {
  __shared__ double2 tab[TRIG_TAB];
  trig_table_fill(tab);
  __syncthreads();
  const int wave = (blockIdx.x * BLOCK + threadIdx.x) >> 6;
  if (wave >= n_tuples) return;
  const int lane = threadIdx.x & 63;
  const int ti = order[wave];
  const TupleDesc& d = desc[ti];
  const TupleState& S = state[ti];
  const int n = d.n;
  const double* fk = f + d.foff;
  const double* th = theta + d.thoff;
  if (!S.has_acc || !(S.l_acc > 0.0)) {
    if (lane < n) {
      if (dzdf) dzdf[d.foff + lane] = __builtin_nan("");
      if (hout) hout[d.foff + lane] = __builtin_nan("");
    }
    return;
  }
  double g[MAXPOOL], h2[MAXPOOL];
#pragma unroll
  for (int k = 0; k < MAXPOOL; ++k) g[k] = h2[k] = 0.0;
  const int64_t N = com->N;
  for (int64_t i = lane; i < N; i += 64) {
    const double ta = tau[i];
    double r = xt[i] - th[0];
    double sv[MAXPOOL], cv[MAXPOOL];
#pragma unroll
    for (int k = 0; k < MAXPOOL; ++k) {
      if (k < n) {
        sincos_tab(fk[k] * ta, tab, sv[k], cv[k]);
        r -= th[1 + 2 * k] * cv[k] + th[2 + 2 * k] * sv[k];
      }
    }
    const double wi = wt[i];
#pragma unroll
    for (int k = 0; k < MAXPOOL; ++k) {
      if (k < n) {
        const double s = sv[k], c = cv[k];
        const double J = 2.0 * M_PI * ta * (-th[1 + 2 * k] * s + th[2 + 2 * k] * c);
        g[k] = __builtin_fma(wi * r, J, g[k]);
        h2[k] = __builtin_fma(wi * J, J, h2[k]);
      }
    }
  }
  const double coef = static_cast<double>(N - 3 * n - 1) / S.l_acc;
#pragma unroll
  for (int k = 0; k < MAXPOOL; ++k) {
    if (k < n) {
      double a = g[k], b = h2[k];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
      }
      if (lane == 0) {
        if (dzdf) dzdf[d.foff + k] = coef * a;
        if (hout) hout[d.foff + k] = coef * b;
      }
    }
  }
}


// Adjoint for tuples of exactly NF <= 6 frequencies, L lanes per tuple.
template <int NF, int L, bool F32>
__global__ __launch_bounds__(BLOCK) void tuple_adjoint_lanes_kernel(const TupleDesc* __restrict__ desc,
                                                                    const int32_t* __restrict__ order, int n_order,
                                                                    const TupleCommon* __restrict__ com,
                                                                    const double* __restrict__ tau,
                                                                    const double* __restrict__ xt,
                                                                    const double* __restrict__ wt,
                                                                    const double* __restrict__ f,
                                                                    const double* __restrict__ theta,
                                                                    const TupleState* __restrict__ state,
                                                                    double* __restrict__ dzdf,
                                                                    double* __restrict__ hout) {
  __shared__ double2 tab[F32 ? 1 : TRIG_TAB];
  if constexpr (!F32) {
    trig_table_fill(tab);
    __syncthreads();
  }
  const int64_t gt = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  const int grp = static_cast<int>(gt / L);
  const int r = static_cast<int>(gt % L);
  const bool in_range = grp < n_order;
  const int ti = in_range ? order[grp] : 0;
  const TupleState& S = state[ti];
  const bool live = in_range && S.has_acc && S.l_acc > 0.0;
  const int64_t foff = desc[ti].foff;
  double fk[NF], th[2 * NF + 1];
#pragma unroll
  for (int k = 0; k < NF; ++k) fk[k] = live ? f[foff + k] : 0.0;
#pragma unroll
  for (int k = 0; k < 2 * NF + 1; ++k) th[k] = live ? theta[desc[ti].thoff + k] : 0.0;
  double g[NF], h2[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) g[k] = h2[k] = 0.0;
  const int64_t N = com->N;
  if (live) {
    // the next sample's tau, w~, x~ are loaded while this one is processed
    double nta = r < N ? tau[r] : 0.0, nwi = r < N ? wt[r] : 0.0, nxi = r < N ? xt[r] : 0.0;
#pragma unroll 1
    for (int64_t i = r; i < N; i += L) {
      const double ta = nta, wi = nwi, xi = nxi;
      if (i + L < N) {
        nta = tau[i + L];
        nwi = wt[i + L];
        nxi = xt[i + L];
      }
      double sv[NF], cv[NF];
      double res = xi - th[0];
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        tuple_sincos<F32>(fk[k] * ta, tab, sv[k], cv[k]);
        res -= th[1 + 2 * k] * cv[k] + th[2 + 2 * k] * sv[k];
      }
      const double tpi = 2.0 * M_PI * ta;
      const double wr = wi * res;
#pragma unroll
      for (int k = 0; k < NF; ++k) {
        const double J = tpi * (-th[1 + 2 * k] * sv[k] + th[2 + 2 * k] * cv[k]);
        g[k] = __builtin_fma(wr, J, g[k]);
        h2[k] = __builtin_fma(wi * J, J, h2[k]);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    g[k] = group_sum<L>(g[k]);
    h2[k] = group_sum<L>(h2[k]);
  }
  if (!in_range || r != 0) return;
  const double coef = static_cast<double>(N - 3 * NF - 1) / S.l_acc;
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    if (dzdf) dzdf[foff + k] = live ? coef * g[k] : __builtin_nan("");
    if (hout) hout[foff + k] = live ? coef * h2[k] : __builtin_nan("");
  }
}

// One step of the preconditioned ascent: f_k += clamp(<r J_k> / <J_k^2>, +-c/T).
__global__ void tuple_ascent_update_kernel(const TupleDesc* __restrict__ desc, int n_tuples,
                                           const TupleCommon* __restrict__ com, const double* __restrict__ g,
                                           const double* __restrict__ h, double* __restrict__ f, double clamp,
                                           TupleState* __restrict__ state) {
  const int ti = blockIdx.x * BLOCK + threadIdx.x;
  if (ti >= n_tuples) return;
  const TupleDesc& d = desc[ti];
  TupleState& S = state[ti];
  if (!S.has_acc) return;
  const double lim = clamp / com->T_eff;
  for (int k = 0; k < d.n; ++k) {
    const double gk = g[d.foff + k], hk = h[d.foff + k];
    if (!isfinite(gk) || !isfinite(hk) || !(hk > 0.0)) continue;
    const double stp = fmin(fmax(gk / hk, -lim), lim);
    f[d.foff + k] += stp;
  }
  // the next forward evaluation starts afresh
  S.done = 0;
  S.has_acc = 0;
  S.l_acc = __builtin_inf();
}

// State of a forward evaluation made by an earlier call, from its l: the
// adjoint kernels need the accepted l and whether there is one.
__global__ void tuple_state_from_l_kernel(int n_tuples, const double* __restrict__ l,
                                          TupleState* __restrict__ state) {
  const int ti = blockIdx.x * BLOCK + threadIdx.x;
  if (ti >= n_tuples) return;
  const double v = l[ti];
  TupleState& S = state[ti];
  S.has_acc = isfinite(v) ? 1 : 0;
  S.l_acc = isfinite(v) ? v : __builtin_inf();
}

__global__ void tuple_init_kernel(int n_tuples, TupleState* __restrict__ state) {
  const int ti = blockIdx.x * BLOCK + threadIdx.x;
  if (ti >= n_tuples) return;
  TupleState s;
  s.l_acc = __builtin_inf();
  s.l0 = 0.0;
  s.halvings = 0;
  s.done = 0;
  s.has_acc = 0;
  s.flags = 0;
  state[ti] = s;
}

__global__ void tuple_common_kernel(const SeriesHdr* __restrict__ hdr, int64_t N, TupleCommon* __restrict__ com) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double sig = sqrt(hdr->stats[3]);
  com->N = N;
  com->T_eff = hdr->T_eff;
  com->inv_sigma_t = 1.0 / sig;
  com->inv_two_pi_sigma_t = 1.0 / (2.0 * M_PI * sig);
}

// l_0 of the constant model as evaluated with the first tuple.
__global__ void tuple_l0_kernel(const TupleState* __restrict__ state, double* __restrict__ l0_out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) l0_out[0] = state[0].l0;
}

__global__ void copy_f64_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

template <int NB, int TV>
hipError_t gram_nb(hipStream_t st, const TupleDesc* desc, const int32_t* order, int n_order, const TupleCommon* com,
                   const double* tau, const double* xt, const double* wt, const double* ftry, const TupleState* state,
                   double* gram, int mode) {
  tuple_gram_kernel<NB, TV><<<n_order, BLOCK, 0, st>>>(desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
  return hipGetLastError();
}

// Column layout of the MFMA Gram kernel for tuples of n frequencies: all C
// columns in ceil(C / 16) blocks (TV = 0), or the T = C - 2 trigonometric
// columns in floor(T / 16) blocks and TV = 2 + T % 16 <= 6 extra columns on
// the VALU, whichever costs fewer issue cycles (a float64 16x16x4 MFMA
// 64, a float64 multiply-add 4, per step of four samples).
void gram_layout(int n, int mode, int& NB, int& TV) {
  const int C = mode == TUPLE_GN ? 4 * n + 2 : 2 * n + 2;
  const int T = C - 2;
  NB = (C + 15) / 16;
  TV = 0;
  const int nbm = T / 16, tail = T % 16;
  if (nbm < 1 || nbm > 4 || tail > 4) return;
  const int cost0 = 64 * NB * (NB + 1) / 2;
  const int cost1 = 64 * nbm * (nbm + 1) / 2 + 4 * (2 + tail) * (nbm + 1);
  if (cost1 < cost0) {
    NB = nbm;
    TV = 2 + tail;
  }
}

template <int NB>
hipError_t gram_tv(int TV, hipStream_t st, const TupleDesc* desc, const int32_t* order, int n_order,
                   const TupleCommon* com, const double* tau, const double* xt, const double* wt, const double* ftry,
                   const TupleState* state, double* gram, int mode) {
  switch (TV) {
    case 2: return gram_nb<NB, 2>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
    case 4: return gram_nb<NB, 4>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
    case 6: return gram_nb<NB, 6>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
    default: return hipErrorInvalidValue;
  }
}

// Lanes per tuple for a group of n_order tuples of N samples: enough groups
// of lanes to give every CU 16 waves, at least 32 samples per lane (fewer
// lanes mean fewer partial sums to add per tuple; at N = 1000 and 10^4
// tuples per size, 16 lanes beat 32 for every size 1..6).
int lanes_for(int n_order, int64_t N, int n_cu) {
  const int64_t want = 16LL * std::max(n_cu, 1) * 64;  // threads for 16 waves per CU
  int L = 4;
  while (L < 64 && static_cast<int64_t>(n_order) * L < want && N / (2 * L) >= 32) L *= 2;
  return L;
}

template <int NF, int L, bool F32>
hipError_t gram_lanes(hipStream_t st, const TupleDesc* desc, const int32_t* order, int n_order,
                      const TupleCommon* com, const double* tau, const double* xt, const double* wt,
                      const double* ftry, TupleState* state, double* gram, double* facc, double* theta,
                      int fuse) {
  const int64_t threads = static_cast<int64_t>(n_order) * L;
  const int blocks = static_cast<int>((threads + BLOCK - 1) / BLOCK);
  tuple_gram_lanes_kernel<NF, L, F32><<<blocks, BLOCK, 0, st>>>(desc, order, n_order, com, tau, xt, wt, ftry, state,
                                                             gram, facc, theta, fuse);
  return hipGetLastError();
}

template <int NF, bool F32>
hipError_t gram_nf(hipStream_t st, int L, const TupleDesc* desc, const int32_t* order, int n_order,
                   const TupleCommon* com, const double* tau, const double* xt, const double* wt,
                   const double* ftry, TupleState* state, double* gram, double* facc, double* theta,
                   int fuse) {
  switch (L) {
    case 4: return gram_lanes<NF, 4, F32>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse);
    case 8: return gram_lanes<NF, 8, F32>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse);
    case 16: return gram_lanes<NF, 16, F32>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse);
    case 32: return gram_lanes<NF, 32, F32>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse);
    case 64: return gram_lanes<NF, 64, F32>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse);
    default: return hipErrorInvalidValue;
  }
}

template <int NF, int L, bool F32>
hipError_t adjoint_lanes(hipStream_t st, const TupleDesc* desc, const int32_t* order, int n_order,
                         const TupleCommon* com, const double* tau, const double* xt, const double* wt,
                         const double* f, const double* theta, const TupleState* state, double* dzdf, double* hout) {
  const int64_t threads = static_cast<int64_t>(n_order) * L;
  const int blocks = static_cast<int>((threads + BLOCK - 1) / BLOCK);
  tuple_adjoint_lanes_kernel<NF, L, F32><<<blocks, BLOCK, 0, st>>>(desc, order, n_order, com, tau, xt, wt, f, theta, state,
                                                                dzdf, hout);
  return hipGetLastError();
}

template <int NF, bool F32>
hipError_t adjoint_nf(hipStream_t st, int L, const TupleDesc* desc, const int32_t* order, int n_order,
                      const TupleCommon* com, const double* tau, const double* xt, const double* wt, const double* f,
                      const double* theta, const TupleState* state, double* dzdf, double* hout) {
  switch (L) {
    case 4: return adjoint_lanes<NF, 4, F32>(st, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
    case 8: return adjoint_lanes<NF, 8, F32>(st, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
    case 16: return adjoint_lanes<NF, 16, F32>(st, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
    case 32: return adjoint_lanes<NF, 32, F32>(st, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
    case 64: return adjoint_lanes<NF, 64, F32>(st, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
    default: return hipErrorInvalidValue;
  }
}

// Residual of each tuple's least-squares fit, r_i = x~_i - Phi(t_i) theta*
// (theta* of tuple k at theta[thoff]: c, a_1, b_1, ...), into r[k N + i],
// and l_k = <r^2> (the weighted sum) into lres[k].  One wavefront per tuple,
// samples over its lanes, trig recomputed per sample.
__global__ __launch_bounds__(BLOCK) void tuple_residual_kernel(const TupleDesc* __restrict__ desc, int n_tuples,
                                                               const TupleCommon* __restrict__ com,
                                                               const double* __restrict__ tau,
                                                               const double* __restrict__ xt,
                                                               const double* __restrict__ wt,
                                                               const double* __restrict__ f,
                                                               const double* __restrict__ theta, double* __restrict__ r,
                                                               double* __restrict__ lres) {
  __shared__ double2 tab[TRIG_TAB];
  trig_table_fill(tab);
  __syncthreads();
  const int k = (blockIdx.x * BLOCK + threadIdx.x) >> 6;
  if (k >= n_tuples) return;
  const int lane = threadIdx.x & 63;
  const TupleDesc& d = desc[k];
  const int n = d.n;
  const double* fk = f + d.foff;
  const double* th = theta + d.thoff;
  const int64_t N = com->N;
  double* rk = r + static_cast<int64_t>(k) * N;
  double acc = 0.0;
  for (int64_t i = lane; i < N; i += 64) {
    const double ta = tau[i];
    double ri = xt[i] - th[0];
    for (int q = 0; q < n; ++q) {
      double sv, cv;
      sincos_tab(fk[q] * ta, tab, sv, cv);
      ri -= th[1 + 2 * q] * cv + th[2 + 2 * q] * sv;
    }
    rk[i] = ri;
    acc = __builtin_fma(wt[i] * ri, ri, acc);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) lres[k] = acc;
}

// Vuong's statistic of the fit `ref` against the fit of every tuple k, for the
// Gaussian noise model with known relative weights and a fitted scale (sample
// i has variance l / (N w~_i)): with the per-sample log-likelihood
// differences d_i = ll_i(ref) - ll_i(k)
//   = -1/2 ln(l_ref / l_k) - (N w~_i / 2)(r_ref,i^2 / l_ref - r_k,i^2 / l_k),
// V_k = sum d / (sqrt(N) omega), omega^2 = mean(d^2) - mean(d)^2.  V_ref = 0;
// V = 0 where omega^2 <= 0 (identical fits); NaN where a fit's l is not
// finite and positive.  One workgroup per tuple; the sums over the samples are
// combined in a fixed tree.
__global__ __launch_bounds__(BLOCK) void tuple_vuong_kernel(int ref, const TupleCommon* __restrict__ com,
                                                            const double* __restrict__ wt,
                                                            const double* __restrict__ r,
                                                            const double* __restrict__ lres, double* __restrict__ V) {
  __shared__ double s1[BLOCK], s2[BLOCK];
  const int k = blockIdx.x;
  const int64_t N = com->N;
  const double lr = lres[ref], lk = lres[k];
  if (k == ref) {
    if (threadIdx.x == 0) V[k] = 0.0;
    return;
  }
  if (!(lr > 0.0 && lk > 0.0 && isfinite(lr) && isfinite(lk))) {
    if (threadIdx.x == 0) V[k] = __builtin_nan("");
    return;
  }
  const double c0 = -0.5 * log(lr / lk);
  const double hN = 0.5 * static_cast<double>(N);
  const double ir = 1.0 / lr, ik = 1.0 / lk;
  const double* rr = r + static_cast<int64_t>(ref) * N;
  const double* rk = r + static_cast<int64_t>(k) * N;
  double a1 = 0.0, a2 = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += BLOCK) {
    const double a = rr[i], b = rk[i];
    const double di = c0 - hN * wt[i] * (a * a * ir - b * b * ik);
    a1 += di;
    a2 = __builtin_fma(di, di, a2);
  }
  s1[threadIdx.x] = a1;
  s2[threadIdx.x] = a2;
  __syncthreads();
  for (int h = BLOCK / 2; h > 0; h >>= 1) {
    if (static_cast<int>(threadIdx.x) < h) {
      s1[threadIdx.x] += s1[threadIdx.x + h];
      s2[threadIdx.x] += s2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double Nd = static_cast<double>(N);
    const double m1 = s1[0] / Nd;
    const double om2 = s2[0] / Nd - m1 * m1;
    V[k] = om2 > 0.0 ? s1[0] / (sqrt(Nd) * sqrt(om2)) : 0.0;
  }
}

// Global-local residual periodogram (Sect. 2): trial frequencies of a chunk of
// the grid, f_j = (j0 + k + 1) df, appended to the refined base frequencies fb
// (tuple k = fb_0 .. fb_{m-1}, f_j, its last member frozen).
__global__ void gl_fill_kernel(const double* __restrict__ fb, int m, double df, int64_t j0, int count,
                               double* __restrict__ ftry) {
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k >= count) return;
  double* f = ftry + static_cast<int64_t>(k) * (m + 1);
  for (int q = 0; q < m; ++q) f[q] = fb[q];
  f[m] = static_cast<double>(j0 + k + 1) * df;
}

// z_j = (N - 3m - 4)/2 ln(l_b / l_j) of the chunk from the refined tuples'
// accepted l (l_b: *lb, or each tuple's constant-model l_0 when lb is null,
// m = 0).  f_j within MASK_WIDTH / T_eff of a refined base frequency: z = 0,
// FLAG_MASKED; a tuple whose start point is degenerate: z = 0, FLAG_SINGULAR;
// l <= 0: z = +inf, FLAG_PERFECT.  Block 0's first thread also writes l_b.
__global__ void gl_finish_kernel(const TupleState* __restrict__ state, int count, const double* __restrict__ fb, int m,
                                 double df, int64_t j0, const TupleCommon* __restrict__ com,
                                 const double* __restrict__ lb, double* __restrict__ z, uint8_t* __restrict__ flags,
                                 double* __restrict__ lb_out) {
  const int k = blockIdx.x * BLOCK + threadIdx.x;
  if (k == 0 && lb_out) *lb_out = lb ? *lb : state[0].l0;
  if (k >= count) return;
  const double T = com->T_eff;
  const double f = static_cast<double>(j0 + k + 1) * df;
  const double NH = static_cast<double>(com->N - 3 * (m + 1) - 1);
  bool masked = false;
  for (int q = 0; q < m; ++q) masked |= fabs(f - fb[q]) * T < MASK_WIDTH;
  const TupleState& S = state[k];
  double zj = 0.0;
  uint8_t fl = 0;
  if (masked) {
    fl = FREDEC_FLAG_MASKED;
  } else if (!S.has_acc) {
    fl = FREDEC_FLAG_SINGULAR;
  } else if (!(S.l_acc > 0.0)) {
    zj = __builtin_inf();
    fl = FREDEC_FLAG_PERFECT;
  } else {
    zj = 0.5 * NH * log((lb ? *lb : S.l0) / S.l_acc);
  }
  z[j0 + k] = zj;
  if (flags) flags[j0 + k] = fl;
}

// Gram matrices of pool subsets at the pool frequencies as sub-blocks of the
// pool's own Gram (Sect. 3: the normal matrix of a subset is the block of the
// pool's normal matrix on the subset's columns).  pg: the pool's packed lower
// Gram in its column order (1, cos/sin of each pool frequency, x~, then in the
// Gauss-Newton mode t' cos/sin of each); tuple ti = order[o] with members
// members[foff ..] (pool indices, increasing) receives the entries of its
// columns in its own order.  One thread per tuple, in launch order (the
// interleaved storage then makes the writes of a group coalesce); the pool
// Gram is staged in LDS.
__global__ __launch_bounds__(BLOCK) void tuple_gather_kernel(const TupleDesc* __restrict__ desc,
                                                             const int32_t* __restrict__ order, int n_tuples,
                                                             const int8_t* __restrict__ members,
                                                             const double* __restrict__ pg, int n_pool, int mode,
                                                             double* __restrict__ gram) {
  extern __shared__ double spg[];
  const bool gn = mode == TUPLE_GN;
  const int CP = gn ? 4 * n_pool + 2 : 2 * n_pool + 2;
  const int npg = CP * (CP + 1) / 2;
  for (int e = threadIdx.x; e < npg; e += BLOCK) spg[e] = pg[e];
  __syncthreads();
  const int o = blockIdx.x * BLOCK + threadIdx.x;
  if (o >= n_tuples) return;
  const TupleDesc& d = desc[order[o]];
  const int n = d.n;
  const int C = gn ? 4 * n + 2 : 2 * n + 2;
  const int K = 2 * n + 1;
  const int8_t* mem = members + d.foff;
  double* G = gram + d.goff;
  const int64_t gs = d.gs;
  auto pcol = [&](int c) {
    if (c == 0) return 0;
    if (c < K) return 1 + 2 * mem[(c - 1) >> 1] + ((c - 1) & 1);
    if (c == K) return 2 * n_pool + 1;
    return 2 * n_pool + 2 + 2 * mem[(c - K - 1) >> 1] + ((c - K - 1) & 1);
  };
  for (int r = 0; r < C; ++r) {
    const int pr = pcol(r);
    for (int c = 0; c <= r; ++c) {
      const int pc = pcol(c);
      const int a = pr > pc ? pr : pc, b = pr > pc ? pc : pr;
      G[(r * (r + 1) / 2 + c) * gs] = spg[a * (a + 1) / 2 + b];
    }
  }
}

}  // namespace

bool tuple_lanes_supported(int n, int mode) { return mode == TUPLE_FWD && n >= 1 && n <= LANES_MAX_N; }

hipError_t launch_tuple_gram(hipStream_t st, int nf, int n_cu, int lanes, const TupleDesc* desc, const int32_t* order,
                             int n_order, int64_t N, const TupleCommon* com, const double* tau, const double* xt,
                             const double* wt, const double* ftry, TupleState* state, double* gram,
                             int mode, bool f32, double* facc, double* theta, bool fuse_solve) {
  if (n_order <= 0) return hipSuccess;
  if (tuple_lanes_supported(nf, mode)) {
    const int L = lanes ? lanes : lanes_for(n_order, N, n_cu);
    if (f32) {
      switch (nf) {
        case 1: return gram_nf<1, true>(st, L, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse_solve ? 1 : 0);
        case 2: return gram_nf<2, true>(st, L, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse_solve ? 1 : 0);
        case 3: return gram_nf<3, true>(st, L, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse_solve ? 1 : 0);
        case 4: return gram_nf<4, true>(st, L, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse_solve ? 1 : 0);
        case 5: return gram_nf<5, true>(st, L, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse_solve ? 1 : 0);
        case 6: return gram_nf<6, true>(st, L, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse_solve ? 1 : 0);
        default: return hipErrorInvalidValue;
      }
    }
    switch (nf) {
      case 1: return gram_nf<1, false>(st, L, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse_solve ? 1 : 0);
      case 2: return gram_nf<2, false>(st, L, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse_solve ? 1 : 0);
      case 3: return gram_nf<3, false>(st, L, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse_solve ? 1 : 0);
      case 4: return gram_nf<4, false>(st, L, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse_solve ? 1 : 0);
      case 5: return gram_nf<5, false>(st, L, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse_solve ? 1 : 0);
      case 6: return gram_nf<6, false>(st, L, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, facc, theta, fuse_solve ? 1 : 0);
      default: return hipErrorInvalidValue;
    }
  }
  int nb = 0, tv = 0;
  gram_layout(nf, mode, nb, tv);
  if (tv > 0) {
    switch (nb) {
      case 1: return gram_tv<1>(tv, st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
      case 2: return gram_tv<2>(tv, st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
      case 3: return gram_tv<3>(tv, st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
      case 4: return gram_tv<4>(tv, st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
      default: return hipErrorInvalidValue;
    }
  }
  switch (nb) {
    case 1: return gram_nb<1, 0>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
    case 2: return gram_nb<2, 0>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
    case 3: return gram_nb<3, 0>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
    case 4: return gram_nb<4, 0>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
    case 5: return gram_nb<5, 0>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
    case 6: return gram_nb<6, 0>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
    case 7: return gram_nb<7, 0>(st, desc, order, n_order, com, tau, xt, wt, ftry, state, gram, mode);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_tuple_solve(hipStream_t st, const TupleDesc* desc, const int32_t* order, int n_tuples,
                              const TupleCommon* com, double* gram, double* scratch, double* ftry, double* facc,
                              double* step, double* theta, TupleState* state, int mode, int last) {
  if (n_tuples <= 0) return hipSuccess;
  // one thread per tuple, serial and latency-bound: small blocks spread the
  // tuples over every CU
  tuple_solve_kernel<<<(n_tuples + 63) / 64, 64, 0, st>>>(desc, order, n_tuples, com, gram, scratch, ftry, facc, step,
                                                          theta, state, mode, last);
  return hipGetLastError();
}

hipError_t launch_tuple_finish(hipStream_t st, const TupleDesc* desc, int n_tuples, const TupleCommon* com,
                               const TupleState* state, const double* facc, double* l_out, double* z_out,
                               uint8_t* flags_out, double* f_out, const int8_t* members, int f_stride) {
  if (n_tuples <= 0) return hipSuccess;
  tuple_finish_kernel<<<(n_tuples + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(desc, n_tuples, com, state, facc, l_out, z_out,
                                                                        flags_out, f_out, members, f_stride);
  return hipGetLastError();
}

hipError_t launch_tuple_adjoint(hipStream_t st, int nf, int n_cu, int lanes, const TupleDesc* desc, const int32_t* order,
                                int n_order, int64_t N, const TupleCommon* com, const double* tau, const double* xt,
                                const double* wt, const double* f, const double* theta, const TupleState* state,
                                double* dzdf, double* hout, bool f32) {
  if (n_order <= 0) return hipSuccess;
  if (tuple_lanes_supported(nf, TUPLE_FWD)) {
    const int L = lanes ? lanes : lanes_for(n_order, N, n_cu);
    if (f32) {
      switch (nf) {
        case 1: return adjoint_nf<1, true>(st, L, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
        case 2: return adjoint_nf<2, true>(st, L, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
        case 3: return adjoint_nf<3, true>(st, L, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
        case 4: return adjoint_nf<4, true>(st, L, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
        case 5: return adjoint_nf<5, true>(st, L, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
        case 6: return adjoint_nf<6, true>(st, L, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
        default: return hipErrorInvalidValue;
      }
    }
    switch (nf) {
      case 1: return adjoint_nf<1, false>(st, L, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
      case 2: return adjoint_nf<2, false>(st, L, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
      case 3: return adjoint_nf<3, false>(st, L, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
      case 4: return adjoint_nf<4, false>(st, L, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
      case 5: return adjoint_nf<5, false>(st, L, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
      case 6: return adjoint_nf<6, false>(st, L, desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
      default: return hipErrorInvalidValue;
    }
  }
  const int blocks = (n_order + 3) / 4;
  tuple_adjoint_kernel<<<blocks, BLOCK, 0, st>>>(desc, order, n_order, com, tau, xt, wt, f, theta, state, dzdf, hout);
  return hipGetLastError();
}

hipError_t launch_tuple_ascent_update(hipStream_t st, const TupleDesc* desc, int n_tuples, const TupleCommon* com,
                                      const double* g, const double* h, double* f, double clamp, TupleState* state) {
  if (n_tuples <= 0) return hipSuccess;
  tuple_ascent_update_kernel<<<(n_tuples + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(desc, n_tuples, com, g, h, f, clamp,
                                                                               state);
  return hipGetLastError();
}

hipError_t launch_tuple_state_from_l(hipStream_t st, int n_tuples, const double* l, TupleState* state) {
  if (n_tuples <= 0) return hipSuccess;
  tuple_state_from_l_kernel<<<(n_tuples + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(n_tuples, l, state);
  return hipGetLastError();
}

hipError_t launch_tuple_init(hipStream_t st, int n_tuples, TupleState* state) {
  if (n_tuples <= 0) return hipSuccess;
  tuple_init_kernel<<<(n_tuples + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(n_tuples, state);
  return hipGetLastError();
}

hipError_t launch_tuple_common(hipStream_t st, const SeriesHdr* hdr, int64_t N, TupleCommon* com) {
  tuple_common_kernel<<<1, 64, 0, st>>>(hdr, N, com);
  return hipGetLastError();
}

hipError_t launch_tuple_gather(hipStream_t st, const TupleDesc* desc, const int32_t* order, int n_tuples,
                               const int8_t* members, const double* pool_gram, int n_pool, int mode, double* gram) {
  if (n_tuples <= 0) return hipSuccess;
  const int CP = mode == TUPLE_GN ? 4 * n_pool + 2 : 2 * n_pool + 2;
  const size_t lds = sizeof(double) * static_cast<size_t>(CP) * (CP + 1) / 2;
  tuple_gather_kernel<<<(n_tuples + BLOCK - 1) / BLOCK, BLOCK, lds, st>>>(desc, order, n_tuples, members, pool_gram,
                                                                          n_pool, mode, gram);
  return hipGetLastError();
}

hipError_t launch_gl_fill(hipStream_t st, const double* fb, int m, double df, int64_t j0, int count, double* ftry) {
  gl_fill_kernel<<<(count + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(fb, m, df, j0, count, ftry);
  return hipGetLastError();
}

hipError_t launch_gl_finish(hipStream_t st, const TupleState* state, int count, const double* fb, int m, double df,
                            int64_t j0, const TupleCommon* com, const double* lb, double* z, uint8_t* flags,
                            double* lb_out) {
  gl_finish_kernel<<<(count + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(state, count, fb, m, df, j0, com, lb, z, flags,
                                                                  lb_out);
  return hipGetLastError();
}

hipError_t launch_tuple_l0(hipStream_t st, const TupleState* state, double* l0_out) {
  tuple_l0_kernel<<<1, 64, 0, st>>>(state, l0_out);
  return hipGetLastError();
}

hipError_t launch_tuple_vuong(hipStream_t st, const TupleDesc* desc, int n_tuples, const TupleCommon* com,
                              const double* tau, const double* xt, const double* wt, const double* f,
                              const double* theta, int ref, double* r, double* lres, double* V) {
  if (n_tuples <= 0) return hipSuccess;
  tuple_residual_kernel<<<(n_tuples + 3) / 4, BLOCK, 0, st>>>(desc, n_tuples, com, tau, xt, wt, f, theta, r, lres);
  tuple_vuong_kernel<<<n_tuples, BLOCK, 0, st>>>(ref, com, wt, r, lres, V);
  return hipGetLastError();
}

hipError_t launch_copy_f64(hipStream_t st, const double* src, double* dst, int64_t n) {
  if (n <= 0) return hipSuccess;
  copy_f64_kernel<<<static_cast<unsigned>((n + BLOCK - 1) / BLOCK), BLOCK, 0, st>>>(src, dst, n);
  return hipGetLastError();
}

}  // namespace fredec
