// Internal declarations of the tuple kernels.
#pragma once

#include "fredec_internal.h"

namespace fredec {

constexpr int MAXPOOL = FREDEC_MAX_POOL;
constexpr int TUPLE_FWD = 0;         // columns 1, cos, sin, x
constexpr int TUPLE_GN = 1;          // plus t' cos, t' sin
constexpr double ACCEPT_RTOL = 1e-12;  // a trial point is accepted if l <= l_acc (1 + ACCEPT_RTOL)
constexpr int MAX_HALVINGS = 5;        // consecutive step halvings before stopping
constexpr double GN_TOL = 1e-10;       // stop once max |df_k| T_eff falls below this
constexpr double GN_CLAMP = 0.25;      // largest step max |df_k| T_eff
constexpr int LANES_MAX_N = 6;         // largest tuple size of the lane-group VALU kernels

// The packed Gram matrices and the solve scratch of a size group are stored
// interleaved: element e of the tuple at position j of its group sits at
// goff + e gs (soff + e gs), goff = group base + j, gs = the group's size, so
// that the one-thread-per-tuple solve reads consecutive addresses across a
// wavefront.
struct TupleDesc {
  int64_t foff;   // first frequency of the tuple in the ragged arrays
  int64_t goff;   // first double of its packed Gram matrix
  int64_t soff;   // first double of its solve scratch
  int64_t thoff;  // first double of theta* (2n + 1 values)
  int32_t n;      // frequencies
  int32_t nb;     // 16-column blocks of its Gram
  int32_t gs;     // element stride of its Gram matrix and scratch
  int32_t frozen; // bit k set: the Gauss-Newton step keeps frequency k fixed
};

struct TupleCommon {
  int64_t N;
  double T_eff;
  double inv_sigma_t;
  double inv_two_pi_sigma_t;
};

struct TupleState {
  double l_acc;     // l at the accepted point (+inf before the first)
  double l0;        // l of the constant model
  int32_t halvings;
  int32_t done;
  int32_t has_acc;
  int32_t flags;
};

// Whether tuples of n frequencies in this mode go to the lane-group VALU
// kernels (launches then take a group of tuples of exactly n).
bool tuple_lanes_supported(int n, int mode);
// nf: the exact size of every tuple of the group (it and the mode fix the
// MFMA kernel's column layout otherwise); n_cu sizes the lane groups; N
// samples; lanes: lanes per tuple of the lane-group kernels (0 = sized from
// the tuple count, N and n_cu); f32: the reduced-precision trig of the lane-group kernels (the MFMA
// kernel is float64).  With fuse_solve the lane-group kernels (forward mode)
// also make the tuples' solve from the Gram in registers (theta, facc and the
// state; the Gram itself is not stored, and the solve kernel then skips these
// tuples, which are done); without it they store the Gram.
hipError_t launch_tuple_gram(hipStream_t st, int nf, int n_cu, int lanes, const TupleDesc* desc, const int32_t* order,
                             int n_order, int64_t N, const TupleCommon* com, const double* tau, const double* xt,
                             const double* wt, const double* ftry, TupleState* state, double* gram, int mode,
                             bool f32, double* facc, double* theta, bool fuse_solve);
// The solve for tuples order[0 .. n_tuples).
hipError_t launch_tuple_solve(hipStream_t st, const TupleDesc* desc, const int32_t* order, int n_tuples,
                              const TupleCommon* com, double* gram, double* scratch, double* ftry, double* facc,
                              double* step, double* theta, TupleState* state, int mode, int last);
hipError_t launch_tuple_finish(hipStream_t st, const TupleDesc* desc, int n_tuples, const TupleCommon* com,
                               const TupleState* state, const double* facc, double* l_out, double* z_out,
                               uint8_t* flags_out, double* f_out, const int8_t* members, int f_stride);
hipError_t launch_tuple_adjoint(hipStream_t st, int nf, int n_cu, int lanes, const TupleDesc* desc, const int32_t* order,
                                int n_order, int64_t N, const TupleCommon* com, const double* tau, const double* xt,
                                const double* wt, const double* f, const double* theta, const TupleState* state,
                                double* dzdf, double* hout, bool f32);
hipError_t launch_tuple_ascent_update(hipStream_t st, const TupleDesc* desc, int n_tuples, const TupleCommon* com,
                                      const double* g, const double* h, double* f, double clamp, TupleState* state);
hipError_t launch_tuple_init(hipStream_t st, int n_tuples, TupleState* state);
hipError_t launch_tuple_state_from_l(hipStream_t st, int n_tuples, const double* l, TupleState* state);
hipError_t launch_tuple_l0(hipStream_t st, const TupleState* state, double* l0_out);
hipError_t launch_tuple_common(hipStream_t st, const SeriesHdr* hdr, int64_t N, TupleCommon* com);
// Residuals r [n_tuples x N] and l = <r^2> (lres) of every tuple's fit with
// coefficients theta, then Vuong's statistic of tuple `ref` against each (V).
hipError_t launch_tuple_vuong(hipStream_t st, const TupleDesc* desc, int n_tuples, const TupleCommon* com,
                              const double* tau, const double* xt, const double* wt, const double* f,
                              const double* theta, int ref, double* r, double* lres, double* V);
// Gram matrices of the pool subsets order[0 .. n_tuples) at the pool
// frequencies, gathered from the pool's Gram (packed lower, its own column
// order, element stride 1).
hipError_t launch_tuple_gather(hipStream_t st, const TupleDesc* desc, const int32_t* order, int n_tuples,
                               const int8_t* members, const double* pool_gram, int n_pool, int mode, double* gram);
// Global-local residual periodogram: the chunk's tuples (refined base fb
// [device, m], then the trial frequency) and their statistic z / flags at
// grid indices j0 .. j0 + count (lb: device l of the refined base, null for
// m = 0; lb_out nullable).
hipError_t launch_gl_fill(hipStream_t st, const double* fb, int m, double df, int64_t j0, int count, double* ftry);
hipError_t launch_gl_finish(hipStream_t st, const TupleState* state, int count, const double* fb, int m, double df,
                            int64_t j0, const TupleCommon* com, const double* lb, double* z, uint8_t* flags,
                            double* lb_out);
hipError_t launch_copy_f64(hipStream_t st, const double* src, double* dst, int64_t n);

}  // namespace fredec
