// Resident-sample phasor tables of the scan kernels.
#pragma once

#include "fredec_internal.h"

namespace fredec {

// For a block whose 256 lanes t = 16a + b own the grid frequencies
// (j0 + 1 + t) df, the phasor e^{2 pi i (j0 + 1 + t) df tau} of lane t at a
// sample is eash[s][a] * bsh[s][b] with
//   eash[s][a] = e^{2 pi i fb tau_s} (w_s^16)^a,  bsh[s][b] = w_s^b,
//   w_s = e^{2 pi i df tau_s}, fb = (j0 + 1) df,
// built here for the nts samples of a tile (every thread takes one sample
// (threadIdx / 4) and four entries (4 q4 .. 4 q4 + 3) of both tables).
// Sample records (stride P) hold tau at [0] and w_s at [KP + 3], [KP + 4].
// Powers come from repeated squaring and multiplication in float64; e^{2 pi
// i fb tau} from the float64 phase reduction of sincos_rev.
template <int KP>
__device__ __forceinline__ void build_phasor_tables(const double* __restrict__ q_tile, int P, int nts, double fb,
                                                    double2 (*eash)[16], double2 (*bsh)[16]) {
  const int sl = threadIdx.x >> 2, q4 = threadIdx.x & 3;
  if (sl >= nts) return;
  const double* qs = q_tile + static_cast<int64_t>(sl) * P;
  const double wc = qs[KP + 3], ws = qs[KP + 4];
  // p = w^(4 q4) and a = w^(64 q4) by repeated squaring (few values live at
  // a time: the accumulators of the calling lane stay in registers)
  double pc = 1.0, ps = 0.0, ac = 1.0, as = 0.0;
  double xc = wc, xs = ws;  // w^(2^k)
#pragma unroll
  for (int k = 1; k <= 7; ++k) {
    const double nc = xc * xc - xs * xs;
    xs = 2.0 * xc * xs;
    xc = nc;
    if ((k == 2 && (q4 & 1)) || (k == 3 && (q4 & 2))) {
      const double tc = pc * xc - ps * xs;
      ps = pc * xs + ps * xc;
      pc = tc;
    }
    if ((k == 6 && (q4 & 1)) || (k == 7 && (q4 & 2))) {
      const double tc = ac * xc - as * xs;
      as = ac * xs + as * xc;
      ac = tc;
    }
  }
  // B_b for b = 4 q4 .. 4 q4 + 3
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    bsh[sl][4 * q4 + k] = double2{pc, ps};
    const double nc = __builtin_fma(pc, wc, -ps * ws);
    ps = __builtin_fma(ps, wc, pc * ws);
    pc = nc;
  }
  // E0 A_a for a = 4 q4 .. 4 q4 + 3, A_a = (w^16)^a (w^16 by four squarings)
  double hc = wc, hs = ws;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double nc = hc * hc - hs * hs;
    hs = 2.0 * hc * hs;
    hc = nc;
  }
  double es, ec;
  sincos_rev(fb * qs[0], es, ec);
  pc = __builtin_fma(ec, ac, -es * as);
  ps = __builtin_fma(es, ac, ec * as);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    eash[sl][4 * q4 + k] = double2{pc, ps};
    const double nc = __builtin_fma(pc, hc, -ps * hs);
    ps = __builtin_fma(ps, hc, pc * hs);
    pc = nc;
  }
}

// float32 copies of the phasor tables for a block whose lane t = 16a + b owns
// the R frequencies (j0 + 1 + t + 256 r) df, r < R:
//   eat[(s 16 + a) R + r] = e^{2 pi i fb tau_s} (w_s^16)^a (w_s^256)^r,
//   bt[s 16 + b]          = w_s^b,
// evaluated in float64 and rounded once to float32, so the lane's phasor for
// frequency r is the float32 complex product of two correctly rounded unit
// phasors.  TS samples per tile, BLOCK / TS threads per sample, each taking
// 16 TS / BLOCK consecutive values of a and of b.  Sample records (stride P)
// hold tau at [0], w_s^256 at [1], [2] and w_s at [KP + 3], [KP + 4].
template <int KP, int R, int TS>
__device__ __forceinline__ void build_phasor_tables32(const double* __restrict__ q_tile, int P, int nts, double fb,
                                                      float2* __restrict__ eat, float2* __restrict__ bt) {
  constexpr int TPS = BLOCK / TS;  // threads per sample
  constexpr int PER = 16 / TPS;    // values of a and of b per thread
  static_assert(TPS * PER == 16, "tile size must divide the block");
  const int sl = threadIdx.x / TPS, part = threadIdx.x % TPS;
  if (sl >= nts) return;
  const double* qs = q_tile + static_cast<int64_t>(sl) * P;
  const double wc = qs[KP + 3], ws = qs[KP + 4];
  const int eb = PER * part;  // first b (and first a) of this thread
  const int ea = 16 * eb;     // exponent of w in A_eb
  // p = w^eb and a = w^(16 eb) by binary powering; h = w^16
  double pc = 1.0, ps = 0.0, ac = 1.0, as = 0.0, hc = 1.0, hs = 0.0;
  double xc = wc, xs = ws;  // w^(2^k)
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k == 4) {
      hc = xc;
      hs = xs;
    }
    if ((eb >> k) & 1) {
      const double tc = __builtin_fma(pc, xc, -ps * xs);
      ps = __builtin_fma(pc, xs, ps * xc);
      pc = tc;
    }
    if ((ea >> k) & 1) {
      const double tc = __builtin_fma(ac, xc, -as * xs);
      as = __builtin_fma(ac, xs, as * xc);
      ac = tc;
    }
    const double nc = __builtin_fma(xc, xc, -xs * xs);
    xs = 2.0 * xc * xs;
    xc = nc;
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    bt[sl * 16 + eb + k] = float2{static_cast<float>(pc), static_cast<float>(ps)};
    const double nc = __builtin_fma(pc, wc, -ps * ws);
    ps = __builtin_fma(ps, wc, pc * ws);
    pc = nc;
  }
  double es, ec;
  sincos_rev(fb * qs[0], es, ec);
  double vc = __builtin_fma(ec, ac, -es * as);
  double vs = __builtin_fma(es, ac, ec * as);
  const double rc = qs[1], rs = qs[2];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    double uc = vc, us = vs;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      eat[(sl * 16 + eb + k) * R + r] = float2{static_cast<float>(uc), static_cast<float>(us)};
      const double nc = __builtin_fma(uc, rc, -us * rs);
      us = __builtin_fma(us, rc, uc * rs);
      uc = nc;
    }
    const double nc = __builtin_fma(vc, hc, -vs * hs);
    vs = __builtin_fma(vs, hc, vc * hs);
    vc = nc;
  }
}

}  // namespace fredec
