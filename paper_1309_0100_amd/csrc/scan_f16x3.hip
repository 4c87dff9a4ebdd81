// Residual periodogram scan, reduced-precision MFMA form with split float16
// operands (eq. zpowrel with n = 1, Sects. 3, 5).
//
// The sums against the base columns, U = <q_k cos>, <q_k sin>, are the
// (F x N) by (N x K) product of the generated trial columns with the weighted
// orthonormal base columns, computed on the float16 matrix cores
// (v_mfma_f32_16x16x32_f16, float32 accumulation) with every operand split
// in two float16 parts, x = x_hi + x_lo, and three products per step:
//   A B ~ A_hi B_hi + A_hi B_lo + A_lo B_hi,
// which keeps about 22 significant bits of every product (the dropped
// A_lo B_lo is below 2^-22 of it).  The weight is split between the two
// operands: B = S sqrt(w~) q_k (the preparation kernel's float16 operand
// array, S = 2^12 so that its low parts stay normal) and A = sqrt(w~) cos,
// sqrt(w~) sin; U = D / S.  The float16 matrix cores have sixteen times the
// float32 matrix rate, so the three products cost less than one float32 step.
//
// Per wave: 16 FT consecutive grid frequencies over all samples of the
// series; one MFMA step covers 16 frequencies x 32 samples.  The lane
// (row = lane % 16, kb = lane / 16) generates A for its frequency row at the
// eight samples 8 kb .. 8 kb + 7 of the step: the float32 complex product
// eat[a][s] * bt[row][s] of two phasors computed in float64 and rounded once,
// staged in LDS per tile of 128 samples (eat = sqrt(w~_s) e^{2 pi i (j0 + 1 +
// 16 a) df tau_s}, a = the wave's 16-frequency tile, computed by the block;
// bt = e^{2 pi i row df tau_s}, the same for every workgroup of the series,
// computed once by the preparation and copied), i.e. c' = sqrt(w~) cos and
// s' = sqrt(w~) sin.  The same lane
// accumulates, for its row and its samples,
//   <cos^2> = sum c'^2, <cos sin> = sum c' s'  float32 per tile of 128
//   samples, then float64,
//   h = <r_b cos>, <r_b sin> = sum (sqrt(w~) r_b) c', ...  float64 (the
//   data column enters z linearly),
// reduced over the four kb lanes at the end; <sin^2> = <1> - <cos^2>.  MFMA
// accumulators are added into float32 running sums at the end of every tile
// (U enters z only through U^T U in the Schur block).  The epilogue forms
// U^T U per frequency from the accumulator layout (D[i][j] in lane j + 16
// (i / 4), element i % 4) with cross-lane sums.
// Points where reduced precision loses accuracy (relative Schur pivot below
// RHO_MIN, or l_{m+1} / l_m below LRATIO_MIN) are listed and re-scored in
// float64 by rescore_kernel, as for the other reduced-precision forms.
#include "fredec_internal.h"

namespace fredec {

namespace {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int F16X3_TS = 128;  // samples per table tile (four MFMA steps of 32)

// c = hi + lo with both parts float16: hi = c rounded toward zero (packed
// conversion), lo = the remainder c - hi, which is exact in float32, rounded
// to float16 by one mixed-precision multiply-add (v_fma_mix{lo,hi}_f16:
// fma(hi, -1, c) with hi read as float16 and c as float32).
__device__ __forceinline__ void split8(const float (&c)[8], v8h& hi, v8h& lo) {
  typedef unsigned u4v __attribute__((ext_vector_type(4)));
  u4v H, L;
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const unsigned ph = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(c[e], c[e + 1]));
    unsigned q;
    asm("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(q) : "v"(ph), "v"(c[e]));
    asm("v_fma_mixhi_f16 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "+v"(q) : "v"(ph), "v"(c[e + 1]));
    H[e / 2] = ph;
    L[e / 2] = q;
  }
  hi = __builtin_bit_cast(v8h, H);
  lo = __builtin_bit_cast(v8h, L);
}

// Sum over the 16 lanes of a DPP row, left in every lane of the row: quad
// permutations (lane ^ 1, lane ^ 2), then the half-row and row mirrors.  All
// lanes add the same pairs, so they hold the same value.
template <int CTRL>
__device__ __forceinline__ float dpp_plus(float v) {
  return v + __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float row_sum16(float v) {
  v = dpp_plus<0xB1>(v);   // quad_perm [1,0,3,2]
  v = dpp_plus<0x4E>(v);   // quad_perm [2,3,0,1]
  v = dpp_plus<0x141>(v);  // row_half_mirror
  return dpp_plus<0x140>(v);  // row_mirror
}

// The aux-record values of one sample that the tables need.
struct SampleRec {
  double tau, sw, gr, hc, hs;  // tau, sqrt(w~), sqrt(w~) r_b, cos and sin of 2 pi 16 df tau
};

// Sample `sl` of the tile starting at i0 (neutral values beyond nts).
__device__ __forceinline__ SampleRec fetch_rec(const double* __restrict__ aser, int64_t i0, int nts, int sl) {
  SampleRec r{0.0, 0.0, 0.0, 1.0, 0.0};
  if (sl < nts) {
    const double* a = aser + (i0 + sl) * AUX_STRIDE;
    r.tau = a[0];
    r.hc = a[1];
    r.hs = a[2];
    r.sw = a[3];
    r.gr = a[4];
  }
  return r;
}

// Tables of one tile of TS samples: eat[a][s] = sqrt(w~_s) e^{2 pi i fb tau_s}
// v_s^a (a < AMAX, v_s = e^{2 pi i 16 df tau_s}), computed here in float64
// and rounded to float32 (the weight folded into eat makes every trial value
// c' = sqrt(w~) cos, s' = sqrt(w~) sin); bt[b][s] = e^{2 pi i b df tau_s}
// (b < 16), copied from the preparation's phasor rows of the tile (pts: 16
// rows of TS float2, zero beyond the series); grs[s] = sqrt(w~_s) r_b(tau_s).
// Samples nts .. TS - 1 get zero entries, so that they contribute nothing.
// BLOCK / TS threads per sample, each taking AMAX TS / BLOCK consecutive rows
// of eat (its first row v^(a0) by binary powers of v).
template <int TS, int AMAX>
__device__ __forceinline__ void build_tables(const SampleRec& r, int nts, double fb, const float4* __restrict__ pts,
                                             float2* __restrict__ eat, float2* __restrict__ bt,
                                             double* __restrict__ grs) {
  constexpr int TPS = BLOCK / TS;   // threads per sample
  constexpr int ROWS = AMAX / TPS;  // rows of eat per thread
  constexpr int TSP = TS + 2;
  constexpr int NV = 16 * TS / 2;   // float4 of bt per tile
  static_assert(TPS * ROWS == AMAX && NV % BLOCK == 0, "tile size must divide the block");
  float4 bv[NV / BLOCK];
#pragma unroll
  for (int u = 0; u < NV / BLOCK; ++u) bv[u] = pts[u * BLOCK + threadIdx.x];
  const int sl = threadIdx.x / TPS, part = threadIdx.x % TPS;
  const int a0 = ROWS * part;
  if (sl < nts) {
    double es, ec;
    sincos_rev(fb * r.tau, es, ec);
    double vc = ec * r.sw, vs = es * r.sw;
    double pc = 1.0, ps = 0.0, xc = r.hc, xs = r.hs;  // v^(a0), v^(2^k)
#pragma unroll
    for (int k = 0; (1 << k) < AMAX; ++k) {
      if ((a0 >> k) & 1) {
        const double tc = __builtin_fma(pc, xc, -ps * xs);
        ps = __builtin_fma(pc, xs, ps * xc);
        pc = tc;
      }
      const double nc = __builtin_fma(xc, xc, -xs * xs);
      xs = 2.0 * xc * xs;
      xc = nc;
    }
    {
      const double tc = __builtin_fma(vc, pc, -vs * ps);
      vs = __builtin_fma(vs, pc, vc * ps);
      vc = tc;
    }
#pragma unroll
    for (int k = 0; k < ROWS; ++k) {
      eat[(a0 + k) * TSP + sl] = float2{static_cast<float>(vc), static_cast<float>(vs)};
      const double nc = __builtin_fma(vc, r.hc, -vs * r.hs);
      vs = __builtin_fma(vs, r.hc, vc * r.hs);
      vc = nc;
    }
    if (part == 0) grs[sl] = r.gr;
  } else {
#pragma unroll
    for (int k = 0; k < ROWS; ++k) eat[(a0 + k) * TSP + sl] = float2{0.0f, 0.0f};
    if (part == 0) grs[sl] = 0.0;
  }
#pragma unroll
  for (int u = 0; u < NV / BLOCK; ++u) {
    const int q = u * BLOCK + threadIdx.x;
    const int b = q / (TS / 2), c = q % (TS / 2);
    *reinterpret_cast<float4*>(bt + b * TSP + 2 * c) = bv[u];
  }
}

// Samples per chunk when a scan is split over nsplit sample chunks (whole tiles).
__host__ __device__ inline int64_t f16x3_chunk(int64_t N, int nsplit) {
  return ((N + nsplit - 1) / nsplit + F16X3_TS - 1) / F16X3_TS * F16X3_TS;
}

// Grid point j of series `series` from its sums: e[0..2] = U^T U (cos cos,
// cos sin, sin sin), e[3..6] = <cos^2>, <cos sin>, h_c, h_s.  Writes z and
// the flags, and lists the point for float64 re-scoring where the reduced
// precision loses accuracy.
__device__ __forceinline__ void f16x3_finish(const double* e, int64_t j, int32_t series, const SeriesIn& si,
                                             const SeriesHdr& h, double* zs, uint8_t* fs, Rescore* list,
                                             unsigned long long* count) {
  const double ccr = e[3], csr = e[4], ss = h.W1 - ccr;
  const double Scc = ccr - e[0], Scs = csr - e[1], Sss = ss - e[2];
  double z;
  uint8_t fl;
  double lratio;
  schur_finish(Scc, Scs, Sss, ccr, ss, e[5], e[6], static_cast<double>(j + 1) * si.df, si, h, z, fl, &lratio);
  const double l21 = Scs / sqrt(fmax(Scc, 1e-300));
  const double rho = fmin(Scc / ccr, (Sss - l21 * l21) / ss);
  if (!(fl & FREDEC_FLAG_MASKED) && (!(rho >= RHO_MIN) || !(lratio >= LRATIO_MIN))) {
    const unsigned long long slot = atomicAdd(count + series, 1ull);
    list[si.goff + slot] = Rescore{series, 0, j};
  }
  zs[j] = z;
  if (fs) fs[j] = fl;
}

// nsplit > 1: the work item covers the samples of chunk wk.pad and writes its
// raw sums (the four float64 sums of each grid point, then U per column) to
// `part` for scan_f16x3_reduce_kernel instead of finishing the points.  Every
// (NT, FT) is held to 256 registers, i.e. two waves per SIMD.
template <int NT, int FT, int TS>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2))) void scan_f16x3_kernel(const ScanWork* __restrict__ work,
                                                           const SeriesIn* __restrict__ sin_,
                                                           const SeriesHdr* __restrict__ hdr,
                                                           const double* __restrict__ aux,
                                                           const v8h* __restrict__ b16,
                                                           const float4* __restrict__ pt16,
                                                           double* __restrict__ z_out, uint8_t* __restrict__ flags_out,
                                                           Rescore* __restrict__ list,
                                                           unsigned long long* __restrict__ count,
                                                           double* __restrict__ part, int nsplit) {
  static_assert(FT >= 1 && FT <= 4, "the epilogue gives one lane group per frequency tile");
  static_assert(TS % 32 == 0 && BLOCK % TS == 0, "tiles hold whole MFMA steps");
  static_assert(TS == PT_TS, "tiles of the preparation's phasor rows");
  constexpr int TSP = TS + 2;  // row length (float2) of the transposed tables
  // LDS: the tables during the sample loop; the epilogue reuses the memory
  // for the per-frequency sums (EPF doubles per frequency)
  constexpr int EPF = 7;
  constexpr int TAB_DOUBLES = (4 * FT + 16) * TSP + TS;
  constexpr int EP_DOUBLES = (BLOCK / 64) * 16 * FT * EPF;
  __shared__ double lds[TAB_DOUBLES > EP_DOUBLES ? TAB_DOUBLES : EP_DOUBLES];
  float2* eat = reinterpret_cast<float2*>(lds);
  float2* bt = eat + 4 * FT * TSP;
  double* grs = reinterpret_cast<double*>(bt + 16 * TSP);

  const ScanWork wk = work[blockIdx.x];
  const SeriesIn& si = sin_[wk.series];
  const SeriesHdr& h = hdr[wk.series];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int row = lane & 15;  // frequency row of A, column of B and D
  const int kb = lane >> 4;   // eight-sample block of the MFMA step
  const int64_t N = si.N;
  const int64_t F = si.F;
  const int64_t jw = wk.j0 + static_cast<int64_t>(wave) * 16 * FT;
  double* zs = z_out + si.goff;
  uint8_t* fs = flags_out ? flags_out + si.goff : nullptr;
  int64_t i_lo = 0, i_hi = N;
  if (nsplit > 1) {
    const int64_t nc = f16x3_chunk(N, nsplit);
    i_lo = static_cast<int64_t>(wk.pad) * nc;
    i_hi = i_lo + nc < N ? i_lo + nc : N;
    if (h.status != 0) return;  // the reduction writes NaN
  }
  if (h.status != 0) {
    for (int ft = 0; ft < FT; ++ft) {
      const int64_t j = jw + ft * 16 + row;
      if (kb == 0 && j < F) {
        zs[j] = __builtin_nan("");
        if (fs) fs[j] = FREDEC_FLAG_BADSERIES;
      }
    }
    return;
  }

  v4f accc[FT][NT], accs[FT][NT];  // MFMA accumulators of the current tile
  v4f uoc[FT][NT], uos[FT][NT];    // float32 running sums of the tile results
  float cc32[FT], cs32[FT];
  double cc[FT], cs[FT], hc[FT], hs[FT];
#pragma unroll
  for (int ft = 0; ft < FT; ++ft) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      accc[ft][nt] = accs[ft][nt] = uoc[ft][nt] = uos[ft][nt] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    cc32[ft] = cs32[ft] = 0.0f;
    cc[ft] = cs[ft] = hc[ft] = hs[ft] = 0.0;
  }

  const double fb = static_cast<double>(wk.j0 + 1) * si.df;
  const double* __restrict__ aser = aux + si.aux_off;
  const v8h* __restrict__ bser = b16 + si.b16_off;
  const float4* __restrict__ pser = pt16 + si.pt_off / 2;  // float2 offset, a multiple of 16 PT_TS
  const int slb = threadIdx.x / (BLOCK / TS);  // sample of this thread in the table build
  for (int64_t i0 = i_lo; i0 < i_hi; i0 += TS) {
    const int nts = i_hi - i0 < TS ? static_cast<int>(i_hi - i0) : TS;
    __syncthreads();
    build_tables<TS, 4 * FT>(fetch_rec(aser, i0, nts, slb), nts, fb, pser + (i0 / TS) * (8 * TS), eat, bt, grs);
    __syncthreads();
    const int ng = (nts + 31) >> 5;
    for (int gg = 0; gg < ng; ++gg) {
      const int64_t g = (i0 >> 5) + gg;  // MFMA step of the series
      v8h bh[NT], bl[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        bh[nt] = bser[((g * NT + nt) * 2) * 64 + lane];
        bl[nt] = bser[((g * NT + nt) * 2 + 1) * 64 + lane];
      }
      const int s0 = 32 * gg + 8 * kb;  // first sample of this lane in the tile
      float2 bv[8];
      double g8[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        bv[e] = bt[row * TSP + s0 + e];
        g8[e] = grs[s0 + e];
      }
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) {
        const int a = FT * wave + ft;
        float c[8], s[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float2 ev = eat[a * TSP + s0 + e];
          c[e] = __builtin_fmaf(ev.x, bv[e].x, -ev.y * bv[e].y);
          s[e] = __builtin_fmaf(ev.y, bv[e].x, ev.x * bv[e].y);
        }
        v8h ch, cl, sh, sl;
        split8(c, ch, cl);
        split8(s, sh, sl);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          accc[ft][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ch, bh[nt], accc[ft][nt], 0, 0, 0);
          accs[ft][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(sh, bh[nt], accs[ft][nt], 0, 0, 0);
          accc[ft][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ch, bl[nt], accc[ft][nt], 0, 0, 0);
          accs[ft][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(sh, bl[nt], accs[ft][nt], 0, 0, 0);
          accc[ft][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(cl, bh[nt], accc[ft][nt], 0, 0, 0);
          accs[ft][nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(sl, bh[nt], accs[ft][nt], 0, 0, 0);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          cc32[ft] = __builtin_fmaf(c[e], c[e], cc32[ft]);
          cs32[ft] = __builtin_fmaf(c[e], s[e], cs32[ft]);
          hc[ft] = __builtin_fma(g8[e], static_cast<double>(c[e]), hc[ft]);
          hs[ft] = __builtin_fma(g8[e], static_cast<double>(s[e]), hs[ft]);
        }
      }
    }
    // end of a tile: tile sums into the running sums
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        uoc[ft][nt] += accc[ft][nt];
        uos[ft][nt] += accs[ft][nt];
        accc[ft][nt] = accs[ft][nt] = v4f{0.f, 0.f, 0.f, 0.f};
      }
      cc[ft] += static_cast<double>(cc32[ft]);
      cs[ft] += static_cast<double>(cs32[ft]);
      cc32[ft] = cs32[ft] = 0.0f;
    }
  }

  // Epilogue.  Per frequency row: <cos^2>, <cos sin>, h summed over the four
  // kb lanes (shuffles); U^T U = sum over the 16 column lanes of this lane's
  // products, in float32 (a relative error e of U^T U moves S by e |U|^2,
  // well below the float32 bound where the point is not re-scored) with DPP
  // row sums.  The seven sums of every frequency go to LDS, and one lane per
  // frequency finishes it.
  if (nsplit > 1) {
    // part: [chunk][4][F] doubles, then [chunk][cos, sin][16 NT columns][F]
    // floats; D[i][col] of a tile sits in lane col + 16 (i / 4), element i % 4
    const int64_t c = wk.pad;
    float* pu = reinterpret_cast<float*>(part + static_cast<int64_t>(nsplit) * 4 * F);
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) {
      double v[4] = {cc[ft], cs[ft], hc[ft], hs[ft]};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        v[q] += __shfl_xor(v[q], 16);
        v[q] += __shfl_xor(v[q], 32);
      }
      const int64_t j = jw + ft * 16 + row;
      if (kb == 0 && j < F) {
#pragma unroll
        for (int q = 0; q < 4; ++q) part[(c * 4 + q) * F + j] = v[q];
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int col = 16 * nt + row;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t jf = jw + ft * 16 + 4 * kb + i;
          if (jf < F) {
            pu[(c * 32 * NT + col) * F + jf] = uoc[ft][nt][i];
            pu[(c * 32 * NT + 16 * NT + col) * F + jf] = uos[ft][nt][i];
          }
        }
      }
    }
    return;
  }
  const double inv2 = h.b16_inv * h.b16_inv;  // 1 / S^2
  __syncthreads();  // every wave is done with the tables
  double* ep = lds + wave * 16 * FT * EPF;
#pragma unroll
  for (int ft = 0; ft < FT; ++ft) {
    double v[4] = {cc[ft], cs[ft], hc[ft], hs[ft]};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      v[q] += __shfl_xor(v[q], 16);
      v[q] += __shfl_xor(v[q], 32);
    }
    float p[4][3];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      p[i][0] = p[i][1] = p[i][2] = 0.0f;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const float uc = uoc[ft][nt][i], us = uos[ft][nt][i];
        p[i][0] = __builtin_fmaf(uc, uc, p[i][0]);
        p[i][1] = __builtin_fmaf(uc, us, p[i][1]);
        p[i][2] = __builtin_fmaf(us, us, p[i][2]);
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) p[i][q] = row_sum16(p[i][q]);
    }
    // row = lane & 15 holds the C block and h of frequency row `row`;
    // lane 16 kb + i (i < 4) the U^T U sums of row 4 kb + i
    if (kb == 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) ep[(ft * 16 + row) * EPF + 3 + q] = v[q];
    }
    if (row < 4) {
      const int r = 4 * kb + row;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float pq = row == 0 ? p[0][q] : row == 1 ? p[1][q] : row == 2 ? p[2][q] : p[3][q];
        ep[(ft * 16 + r) * EPF + q] = static_cast<double>(pq) * inv2;
      }
    }
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < 16 * FT) {
    const int64_t j = jw + lane;
    if (j < F) f16x3_finish(ep + lane * EPF, j, wk.series, si, h, zs, fs, list, count);
  }
}

// The chunks' sums of a split scan (one series) added in chunk order, U^T U
// formed in float64, then the finish of scan_f16x3_kernel: one thread per grid
// point.
__global__ __launch_bounds__(BLOCK) void scan_f16x3_reduce_kernel(const SeriesIn* __restrict__ sin_,
                                                                  const SeriesHdr* __restrict__ hdr,
                                                                  const double* __restrict__ part, int nsplit,
                                                                  double* __restrict__ z_out,
                                                                  uint8_t* __restrict__ flags_out,
                                                                  Rescore* __restrict__ list,
                                                                  unsigned long long* __restrict__ count) {
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
  double e[7];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double v = 0.0;
    for (int c = 0; c < nsplit; ++c) v += part[(static_cast<int64_t>(c) * 4 + q) * F + j];
    e[3 + q] = v;
  }
  const float* pu = reinterpret_cast<const float*>(part + static_cast<int64_t>(nsplit) * 4 * F);
  const int NC = 16 * si.NT;
  double p0 = 0.0, p1 = 0.0, p2 = 0.0;
  for (int col = 0; col < NC; ++col) {
    double uc = 0.0, us = 0.0;
    for (int c = 0; c < nsplit; ++c) {
      uc += static_cast<double>(pu[(static_cast<int64_t>(c) * 2 * NC + col) * F + j]);
      us += static_cast<double>(pu[(static_cast<int64_t>(c) * 2 * NC + NC + col) * F + j]);
    }
    p0 = __builtin_fma(uc, uc, p0);
    p1 = __builtin_fma(uc, us, p1);
    p2 = __builtin_fma(us, us, p2);
  }
  const double inv2 = h.b16_inv * h.b16_inv;  // 1 / S^2
  e[0] = p0 * inv2;
  e[1] = p1 * inv2;
  e[2] = p2 * inv2;
  f16x3_finish(e, j, 0, si, h, zs, fs, list, count);
}

template <int NT, int FT>
hipError_t launch_nt(hipStream_t st, int n_work, const ScanWork* work, const SeriesIn* sin, const SeriesHdr* hdr,
                     const double* aux, const void* b16, const void* pt16, double* z, uint8_t* flags, Rescore* list,
                     unsigned long long* count, double* part, int nsplit, int64_t F_split) {
  const int ns = nsplit > 1 && part && F_split > 0 ? nsplit : 1;
  scan_f16x3_kernel<NT, FT, F16X3_TS><<<n_work, BLOCK, 0, st>>>(work, sin, hdr, aux, static_cast<const v8h*>(b16),
                                                               static_cast<const float4*>(pt16), z, flags, list,
                                                               count, part, ns);
  if (ns > 1)
    scan_f16x3_reduce_kernel<<<static_cast<unsigned>((F_split + BLOCK - 1) / BLOCK), BLOCK, 0, st>>>(
        sin, hdr, part, ns, z, flags, list, count);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_scan_f16x3(hipStream_t st, int NT, int FT, int n_work, const ScanWork* work, const SeriesIn* sin,
                             const SeriesHdr* hdr, const double* aux, const void* b16, const void* pt16, double* z,
                             uint8_t* flags, Rescore* list, unsigned long long* count, double* part, int nsplit,
                             int64_t F_split) {
  if (n_work <= 0) return hipSuccess;
#define X(nt, ft)                                                                                              \
  if (NT == nt && FT == ft)                                                                                    \
    return launch_nt<nt, ft>(st, n_work, work, sin, hdr, aux, b16, pt16, z, flags, list, count, part, nsplit, \
                             F_split);
  X(1, 1) X(1, 2) X(1, 4) X(2, 1) X(2, 2) X(3, 1) X(4, 1)
#undef X
  return hipErrorInvalidValue;
}

int scan_f16x3_nsplit(int64_t N, int NT, int64_t F) {
  const int64_t tile = 64 * static_cast<int64_t>(f16x3_freq_tiles(NT));
  const int64_t tiles = (F + tile - 1) / tile;
  if (tiles >= 512) return 1;
  int64_t ns = (512 + tiles - 1) / tiles;
  if (ns > 16) ns = 16;
  if (ns > N / 1024) ns = N / 1024;
  return ns < 2 ? 1 : static_cast<int>(ns);
}

}  // namespace fredec
