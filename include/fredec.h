/*
 * fredec.h - C ABI of the FREDEC multifrequency-periodogram hot path for
 * AMD Instinct MI355X (gfx950).
 *
 * Method: R. V. Baluev, "Detecting multiple periodicities in observational
 * data with the multifrequency periodogram - II. Frequency Decomposer"
 * (Astronomy and Computing; arXiv:1309.0100).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Bulk arrays (times, values, weights, outputs, tables) are DEVICE pointers
 *    owned by the caller.  Small descriptors (offsets, base frequencies, grid
 *    steps, masks, thresholds) are HOST pointers.  Each argument says which.
 *    The library never frees or retains caller memory beyond the work it
 *    enqueues on `stream`; host arrays may be reused as soon as a call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    work is enqueued asynchronously on it; results are valid once the stream
 *    has reached that point.
 *  - Scratch memory comes from a caller-provided device `workspace` whose size
 *    is given by the matching *_workspace query; too small a workspace returns
 *    FREDEC_ENOMEM before anything is enqueued.
 *  - Return value: FREDEC_OK (0) or a negative code.  Every check on host
 *    arguments is made before any work is enqueued.  Conditions that need the
 *    device data (weights, degenerate series, singular base model) are
 *    reported per series in `status_out` (one int32 per series, 0 = ok, else
 *    the negative code), and the outputs of that series are NaN.
 *  - Per-element numeric conditions are not call errors: they are reported in
 *    `flags_out` bits (see FREDEC_FLAG_*).
 *  - A context is bound to one device and is not thread-safe: use one context
 *    per host thread.  It owns three side streams (default priority) onto
 *    which a call may fork independent kernels; they are joined back to the
 *    caller's stream (events) before the call's later work, so the call stays
 *    ordered on that stream and can be captured into a HIP graph from it.
 *    Outputs are always float64 whatever the precision.
 *  - Time t is in the caller's unit (e.g. days); frequencies are in cycles per
 *    that unit.  Data are normalised internally as in Sect. 4.1 (eq. idn):
 *    weights to unit sum, x to zero weighted mean and unit weighted variance,
 *    t centred.  The statistics do not depend on the units.
 */
#ifndef FREDEC_H
#define FREDEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fredec_ctx fredec_ctx;

/* Internal arithmetic of the trigonometric sums (outputs are float64). */
enum {
  FREDEC_FP64 = 0, /* float64 phase, trig and sums */
  FREDEC_FP32 = 1  /* float64 phase reduction, phasors, data column and solves;
                      float32 sums against the base columns (VALU or MFMA),
                      added into float64 totals per sample tile; ill-conditioned
                      points re-scored in float64 */
};

enum {
  FREDEC_OK = 0,
  FREDEC_EINVAL = -1,    /* null pointer, bad size, bad precision, bad option */
  FREDEC_EDOF = -2,      /* N - 3(m+1) - 1 <= 0 (scan) or N - 3n - 1 <= 0 (tuples), Sect. 2 */
  FREDEC_EWEIGHT = -3,   /* a weight w_i <= 0 or a non-finite t, x or w, Sect. 2 */
  FREDEC_EDEGEN = -4,    /* zero weighted variance of x or of t */
  FREDEC_ESINGULAR = -5, /* base normal matrix not positive definite */
  FREDEC_ENOMEM = -6,    /* workspace too small, or host allocation failed */
  FREDEC_EDEVICE = -7,   /* HIP runtime error (launch or earlier asynchronous fault) */
  FREDEC_ENOTSUP = -8    /* size beyond a compiled limit (e.g. m > FREDEC_MAX_BASE) */
};

/* Element flags (uint8). */
enum {
  FREDEC_FLAG_MASKED = 1,     /* |f - f'_k| * T_eff < 0.05 for a base frequency: z := 0 */
  FREDEC_FLAG_SINGULAR = 2,   /* Cholesky pivot below 1e-13 of its diagonal: z := 0 */
  FREDEC_FLAG_PERFECT = 4,    /* l <= 0 (perfect fit): z := +inf */
  FREDEC_FLAG_DEGENERATE = 8, /* tuple with merged frequencies or singular matrix: z := -inf */
  FREDEC_FLAG_CONVERGED = 16, /* tuple refinement stopped on the step tolerance */
  FREDEC_FLAG_RESCORED = 64,  /* FREDEC_FP32 scan: trial columns nearly in the base span (relative
                                 Schur pivot < 0.6) or a strong peak (l_{m+1} < l_m / 2):
                                 value recomputed in float64 */
  FREDEC_FLAG_BADSERIES = 128 /* the series failed validation (see status_out): z := NaN */
};

#define FREDEC_MAX_BASE 24   /* largest base model m of a scan */
#define FREDEC_MAX_POOL 27   /* largest tuple size n (explicit masks, ragged tuples) and pool size of the
                                cascade; Sect. 5 names n = 25-27 as the practical limit of the method.  With
                                masks == NULL (all 2^n - 1 subsets) the caller's workspace bounds n. */

/* Context --------------------------------------------------------------- */
int fredec_create(fredec_ctx** ctx, int device);
void fredec_destroy(fredec_ctx* ctx);
const char* fredec_strerror(int code);
int fredec_version(void); /* 100 * major + minor */

/* Timing of the dominant kernel of each call (the trig-sum kernels of a
 * scan, the Gram kernel of tuples): while enabled, every call records a pair
 * of HIP events on its stream around those launches.  fredec_profile_read
 * waits for them and returns the summed elapsed time (ms) and the number of
 * event pairs since the last read or enable, then resets the count. */
int fredec_profile(fredec_ctx* ctx, int32_t enable);
int fredec_profile_read(fredec_ctx* ctx, double* total_ms, int64_t* launches);
/* The same timing by kind of kernel group: ms_out[k] and launches_out[k]
 * (host arrays of n_kinds) receive the summed time (ms) and the number of
 * timed groups of kind k < n_kinds since the last read or enable, then every
 * count is reset.  fredec_profile_read reports kinds SCAN and GRAM. */
enum {
  FREDEC_PROF_SCAN = 0,     /* trig-sum kernels of a scan (every kernel family) */
  FREDEC_PROF_GRAM = 1,     /* tuple Gram passes (all size groups of a pass) */
  FREDEC_PROF_SOLVE = 2,    /* tuple solves (Cholesky, theta*, Gauss-Newton step) */
  FREDEC_PROF_PREP = 3,     /* normalisation and base-model precomputation of a scan */
  FREDEC_PROF_RESCORE = 4,  /* float64 re-scoring of reduced-precision scan points */
  FREDEC_PROF_ADJOINT = 5,  /* adjoint passes (dz/df) */
  FREDEC_PROF_NKIND = 6
};
int fredec_profile_read_kinds(fredec_ctx* ctx, int32_t n_kinds, double* ms_out, int64_t* launches_out);

/* Kernel and tile choices made by the autotuner (paper_1309_0100_amd/autotune.py).
 * FREDEC_TILE_SCAN_F16X3: key = column tiles NT of the split-float16 scan
 * operand (1..4, i.e. ceil((2m+1)/16)), value = 16-frequency tiles per wave
 * FT (1, 2 or 4 with NT * FT <= 4; 0 = default: 4, 2, 1, 1 for NT = 1..4).
 * FREDEC_TILE_SCAN_F32_FORM: key = 0, value = kernel family of the
 * FREDEC_FP32 scan (FREDEC_F32_FORM_*): VALU = float32 vector sums (base
 * models with m <= 12; the split-float16 kernel above), F16X3 = float16
 * matrix cores on split operands (three products per step) for every m,
 * AUTO (default) = VALU for 2m + 2 <= the key-1 setting and F16X3 above.
 * All give results within the float32 bound.  Key = 1: value = largest
 * 2m + 2 (0..26, default 6) that the AUTO form gives to the VALU kernel.
 * FREDEC_TILE_SCAN_F32_FORM value 1 (a float32-MFMA kernel family) is no
 * longer provided and is rejected.
 * FREDEC_TILE_TUPLE_LANES: key = tuple size n (1..6, the sizes the lane-group
 * forward and adjoint kernels take), value = lanes per tuple (4, 8, 16, 32
 * or 64; 0 = default: sized from the tuple count, N and the CU count).
 * Errors: EINVAL for an unsupported combination.  The workspace size of a
 * scan or a tuple batch does not depend on these settings. */
enum { FREDEC_TILE_SCAN_F16X3 = 1, FREDEC_TILE_SCAN_F32_FORM = 2, FREDEC_TILE_TUPLE_LANES = 3 };
enum { FREDEC_F32_FORM_VALU = 0, FREDEC_F32_FORM_F16X3 = 2, FREDEC_F32_FORM_AUTO = 3 };
int fredec_set_tile(fredec_ctx* ctx, int32_t kernel, int32_t key, int32_t value);

/* Normalisation (Sect. 4.1, eq. idn; T_eff of Sect. 2) -------------------
 * Batch of n_series series in CSR form: series s owns samples
 * [soff[s], soff[s+1]) of t, x, w (device, float64).
 * Outputs (device, float64, same layout): tau = t - <t>, xt = (x - <x>)/s_x,
 * wt = w / sum(w).  stats_out (device, [n_series * 6]): <t>, <x>, s_x,
 * Var(t), T_eff = sqrt(4 pi Var(t)), sum(w).  status_out: per-series status. */
int fredec_normalize_workspace(int32_t n_series, size_t* bytes);
int fredec_normalize(fredec_ctx* ctx, void* stream, int32_t n_series, const int64_t* soff_host,
                     const double* t, const double* x, const double* w,
                     void* workspace, size_t ws_bytes,
                     double* tau_out, double* xt_out, double* wt_out, double* stats_out,
                     int32_t* status_out);

/* Residual periodogram scan (eq. zpowrel with n = 1; Sects. 2, 3, 5) -----
 * For series s with base frequencies f'_1..f'_m (m = boff[s+1]-boff[s] <=
 * FREDEC_MAX_BASE, host base_f[boff[s]..]) and grid f_j = (j+1) * df[s],
 * j = 0..F[s]-1, computes
 *     z_j = (N - 3m - 4)/2 * ln( l_m(f') / l_{m+1}(f', f_j) )
 * where l is the least-squares chi^2 minimum of the normalised data for the
 * model "constant + sinusoids" (eq. Hn).  z of series s is written to
 * z_out[goff_s + j] with goff_s = F[0] + ... + F[s-1] (device, float64);
 * flags_out (device uint8, same layout, nullable); l_base_out (device,
 * [n_series], nullable) receives l_m; status_out (device int32 [n_series],
 * nullable).  soff, boff, base_f, df and F are host arrays.
 * A batch's kernel groups (one per kernel instance) run concurrently on the
 * context's side streams.  A single series whose grid gives few frequency
 * tiles (FREDEC_FP64: fewer than 128; FREDEC_FP32: fewer than 512 at the
 * split-float16 kernel's default tile) is split over up to 16 sample chunks
 * (the workspace then holds their partial sums; they are added in chunk
 * order), and in FREDEC_FP32 such a series is given to the split-float16
 * kernel even where the automatic form would pick the float32 VALU kernel.
 * Errors: EINVAL (null/size/precision), EDOF (N - 3m - 4 <= 0 for a series),
 * ENOTSUP (m > FREDEC_MAX_BASE), ENOMEM (workspace). */
int fredec_scan_workspace(int32_t n_series, const int64_t* soff_host, const int64_t* boff_host,
                          const int64_t* F_host, int32_t precision, size_t* bytes);
int fredec_scan(fredec_ctx* ctx, void* stream, int32_t n_series,
                const double* t, const double* x, const double* w, const int64_t* soff_host,
                const double* base_f_host, const int64_t* boff_host,
                const double* df_host, const int64_t* F_host,
                int32_t precision, void* workspace, size_t ws_bytes,
                double* z_out, uint8_t* flags_out, double* l_base_out, int32_t* status_out);

/* Allocation-free residual scan ---------------------------------------------
 * For callers that cannot allocate device memory: code under HIP-graph
 * capture, tight serving loops, harnesses that forbid allocation.  The result
 * of fredec_scan for ONE series (t, x, w device [N]; base_f host [m], nullable
 * when m = 0; grid f_j = (j+1) df, j < F; outputs as for fredec_scan with
 * n_series = 1), computed by the same kernels, with its scratch memory taken
 * from a static device array of the library instead of a workspace.  The call
 * makes no allocation and no copy of any kind (no hipMalloc, hipFree,
 * hipHostMalloc, memset or host-to-device copy): the series descriptor and the
 * work list are written by kernels from launch arguments.  No timing events
 * are recorded (fredec_profile does not apply).
 *  - Limit: the scan's scratch (fredec_scan_workspace of this one series) must
 *    fit FREDEC_STATIC_SCRATCH_BYTES (32 MiB: e.g. N = 2000, m = 4,
 *    F = 10^6 in both precisions; N = 10^4, m = 12, F = 4e6 in FREDEC_FP64
 *    only); larger scans return FREDEC_ENOTSUP before anything is enqueued.
 *  - Each GPU holds its own copy of the array (32 MiB) from library load
 *    until the process ends; its address is resolved by fredec_create.
 *  - Every call on one GPU shares that GPU's array and leaves its contents
 *    behind (each call re-initialises what it reads).  Calls that overlap in
 *    time on one GPU (several streams, threads or contexts) race on it:
 *    serialise them.
 * Errors: EINVAL (null pointer, N <= 0, F <= 0, m < 0, bad precision or df,
 * null or unusable context), EDOF, ENOTSUP (m > FREDEC_MAX_BASE or scratch
 * above the limit), EDEVICE. */
#define FREDEC_STATIC_SCRATCH_BYTES (32 * 1024 * 1024)
int fredec_scan_static(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                       const double* base_f_host, int32_t m, double df, int64_t F, int32_t precision, double* z_out,
                       uint8_t* flags_out, double* l_base_out, int32_t* status_out);

/* The same statistic for one series at an explicit list of grid indices
 * (device int64 idx[n_idx], each in [0, F), n_idx < 2^31), always in float64
 * (one workgroup per index).  Used to re-score reduced-precision peaks.
 * z_out/flags_out: device [n_idx].  Errors: EINVAL (null pointer, bad size
 * or df, n_idx >= 2^31), EDOF, ENOTSUP, ENOMEM (workspace), EDEVICE. */
int fredec_scan_at_workspace(int64_t N, int32_t m, size_t* bytes);
int fredec_scan_at(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w,
                   int64_t N, const double* base_f_host, int32_t m, double df,
                   const int64_t* idx, int64_t n_idx, void* workspace, size_t ws_bytes,
                   double* z_out, uint8_t* flags_out);

/* Prepared calls for HIP-graph capture --------------------------------------
 * A plan does the host part of a call once: it checks the host arguments,
 * lays out the workspace, uploads the descriptors into it and waits for that
 * upload (synchronous on `stream`).  Launching a plan (fredec_plan_*) then
 * only enqueues kernels - no host-to-device copy, no allocation, no memset,
 * no synchronisation - so a launch can be captured into a HIP graph and the
 * graph replayed; every launch reads t, x, w (and f) afresh from the given
 * device pointers, so new data written into the same buffers are picked up.
 * Between plan creation and its last launch the plan's workspace belongs to
 * the plan: it must not be freed or passed to another call.  Launches of one
 * plan that overlap in time (two streams) race on its workspace.  Tile
 * settings (fredec_set_tile) are fixed when the plan is made.  Timing events
 * (fredec_profile) must be off while a launch is captured.  A plan is bound
 * to the context's device and is freed by fredec_plan_destroy (host memory
 * only; NULL is ignored). */
typedef struct fredec_plan fredec_plan;
void fredec_plan_destroy(fredec_plan* plan);

/* Plan of fredec_scan for a fixed CSR batch (arguments and errors as for
 * fredec_scan; workspace size from fredec_scan_workspace). */
int fredec_scan_plan(fredec_ctx* ctx, void* stream, int32_t n_series, const int64_t* soff_host,
                     const double* base_f_host, const int64_t* boff_host, const double* df_host,
                     const int64_t* F_host, int32_t precision, void* workspace, size_t ws_bytes,
                     fredec_plan** plan_out);
/* Launch of a scan plan; t, x, w and the outputs as for fredec_scan.
 * Errors: EINVAL (null pointer, a plan of another kind or device), EDEVICE. */
int fredec_plan_scan(fredec_ctx* ctx, fredec_plan* plan, void* stream,
                     const double* t, const double* x, const double* w,
                     double* z_out, uint8_t* flags_out, double* l_base_out, int32_t* status_out);

/* Tuple statistics (eq. zpow; Sects. 2, 3, 4.3) --------------------------
 * One series t, x, w (device, N samples) and a pool of n_pool <= FREDEC_MAX_POOL
 * frequencies (host pool[n_pool]).  Tuple k is the subset of the pool given by
 * the bits of masks[k] (host; bit b selects pool[b]); masks == NULL means all
 * 2^n_pool - 1 subsets in increasing mask order (n_tuples must then equal
 * 2^n_pool - 1).  For each tuple of n frequencies:
 *   l = min over theta of <(x~ - mu)^2> for the model of eq. Hn,
 *   z = (N - 3n - 1)/2 ln(l_0 / l), l_0 the constant-model minimum.
 * refine_steps = 0 evaluates at the pool frequencies.  refine_steps = R > 0
 * makes 1 + R float64 least-squares passes per tuple: Gauss-Newton steps on
 * the frequencies with theta re-solved at each iterate (Sect. 3, eq. lsqf),
 * each step scaled to max |df| T_eff <= 0.25, a trial point accepted if
 * l <= l_acc (1 + 1e-12) and otherwise the step halved (at most 5 times in a
 * row), stopping once max |df| T_eff < 1e-10 (flag FREDEC_FLAG_CONVERGED).
 * Outputs (device, nullable): l_out[n_tuples], z_out[n_tuples],
 * f_out[n_tuples * n_pool] (the accepted frequencies of the members at their
 * pool index, NaN elsewhere), flags_out[n_tuples] (FREDEC_FLAG_DEGENERATE:
 * two frequencies within 0.05 / T_eff or a singular normal matrix, z = -inf;
 * FREDEC_FLAG_PERFECT: l <= 0, z = +inf), l0_out[1] (l_0 of the constant
 * model, the entry l(empty set) of the Phase 3 table).  The sums are float64 (MFMA) for
 * both precisions.  Errors: EINVAL, ENOTSUP (n_pool > FREDEC_MAX_POOL),
 * EDOF (N - 3 n_max - 1 <= 0), ENOMEM. */
int fredec_tuples_workspace(int64_t N, int32_t n_pool, const uint64_t* masks_host, int64_t n_tuples,
                            int32_t refine_steps, size_t* bytes);
int fredec_tuples(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                  const double* pool_host, int32_t n_pool, const uint64_t* masks_host, int64_t n_tuples,
                  int32_t refine_steps, int32_t precision, void* workspace, size_t ws_bytes,
                  double* l_out, double* z_out, double* f_out, uint8_t* flags_out, double* l0_out);

/* z and its gradient for ragged tuples: tuple k owns the frequencies
 * f[toff[k] .. toff[k+1]) (f device float64, toff host int64, toff[0] = 0,
 * 1 <= toff[k+1] - toff[k] <= FREDEC_MAX_POOL).  z is the absolute statistic
 * of eq. zpow at the given frequencies, l the least-squares minimum of eq. lsq
 * (Sect. 3).  The gradient follows the frequency part of the gradient g_f of
 * eq. lsqf at theta = theta*(f) (Sect. 3: its theta part vanishes there):
 * dl/df_k = -2 <r J_k>, hence dz/df_k = (N_H / l) <r J_k>, with
 * r = x~ - Phi theta*, J_k = d mu / d f_k = 2 pi t (-a_k sin 2 pi f_k t +
 * b_k cos 2 pi f_k t) and N_H = N - 3n - 1; h_k = (N_H / l) <J_k^2> is the
 * diagonal of the frequency block of the Fisher matrix Q_f of eq. lsqf in the
 * same units (the curvature of a one-frequency Gauss-Newton step).  The
 * adjoint recomputes the trig terms sample by sample (nothing of size N x n
 * is stored).  Outputs (device, nullable): z_out, l_out, flags_out
 * [n_tuples]; theta_out [sum(2 n_k + 1)], tuple k at offset 2 toff[k] + k
 * (c, a_1, b_1, ..., a_n, b_n); dz_df, h_out [toff[n_tuples]].  With dz_df
 * and h_out both NULL no adjoint pass is made.  Degenerate tuples (flags)
 * get NaN gradients.  Errors: EINVAL, ENOTSUP (a tuple above
 * FREDEC_MAX_POOL), EDOF (N - 3 n_max - 1 <= 0), ENOMEM. */
int fredec_grad_workspace(int64_t N, const int64_t* toff_host, int64_t n_tuples, size_t* bytes);
int fredec_grad(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                const double* f, const int64_t* toff_host, int64_t n_tuples, int32_t precision,
                void* workspace, size_t ws_bytes, double* z_out, double* l_out, double* theta_out,
                double* dz_df, double* h_out, uint8_t* flags_out);

/* The adjoint pass of fredec_grad alone, for a forward evaluation made
 * earlier (the backward pass of an automatic-differentiation framework):
 * given the frequencies f, toff as for fredec_grad, and that call's theta_out
 * (theta, device) and l_out (l, device), writes dz_df and h_out (device,
 * nullable, [toff[n_tuples]]) by the formulas of fredec_grad.  A tuple whose
 * l is not finite and positive gets NaN.  Workspace from
 * fredec_grad_workspace.  Errors as for fredec_grad. */
int fredec_adjoint(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                   const double* f, const int64_t* toff_host, int64_t n_tuples, const double* theta,
                   const double* l, int32_t precision, void* workspace, size_t ws_bytes, double* dz_df,
                   double* h_out);

/* Vuong's statistic between fits (Phase 4 of Sect. 4 and the per-solution
 * output of Sect. 6, which compare each alternative solution with the best
 * one; the paper does not print the formula).  For ragged tuples as in
 * fredec_grad (f device, toff host) with their least-squares coefficients
 * theta (device, the theta_out layout of fredec_grad, from a fredec_grad call
 * at the same f), the residuals r = x~ - Phi theta* are recomputed sample by
 * sample, l_k = <r^2> (device l_out [n_tuples], nullable), and for the
 * Gaussian noise model of Sect. 2 with known relative weights and a fitted
 * scale (sample i has variance l / (N w~_i)) the per-sample log-likelihood
 * differences of tuple `ref` against tuple k,
 *   d_i = -1/2 ln(l_ref / l_k) - (N w~_i / 2)(r_ref,i^2 / l_ref - r_k,i^2 / l_k),
 * give V_out[k] = sum d / (sqrt(N) omega), omega^2 = mean(d^2) - mean(d)^2
 * (device [n_tuples]; positive when `ref` fits better; V_ref = 0; 0 for
 * identical fits; NaN if an l is not finite and positive).  Workspace from
 * fredec_vuong_workspace (includes N x n_tuples residuals).  Errors: EINVAL
 * (also ref outside [0, n_tuples)), ENOTSUP, EDOF, ENOMEM. */
int fredec_vuong_workspace(int64_t N, const int64_t* toff_host, int64_t n_tuples, size_t* bytes);
int fredec_vuong(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                 const double* f, const int64_t* toff_host, int64_t n_tuples, const double* theta, int64_t ref,
                 void* workspace, size_t ws_bytes, double* l_out, double* V_out);

/* Fixed-step preconditioned ascent of z for ragged tuples (workspace as for
 * fredec_grad): `steps` times f_k += clamp(<r J_k> / <J_k^2>, +-clamp / T_eff),
 * then a final evaluation.  f (device) is updated in place; outputs as for
 * fredec_grad. */
int fredec_ascent(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                  double* f, const int64_t* toff_host, int64_t n_tuples, int32_t steps, double clamp,
                  int32_t precision, void* workspace, size_t ws_bytes, double* z_out, double* l_out,
                  uint8_t* flags_out);

/* Plans of fredec_tuples and fredec_ascent (see "Prepared calls" above).
 * fredec_tuples_plan takes the arguments of fredec_tuples that are fixed per
 * batch (N, pool, masks, refine_steps, precision; workspace from
 * fredec_tuples_workspace) and fredec_plan_tuples the series and outputs;
 * fredec_ascent_plan takes N, the tuple offsets, steps, clamp and precision
 * (workspace from fredec_grad_workspace) and fredec_plan_ascent the series,
 * the frequencies f (device, updated in place) and outputs.  Results equal
 * those of the unplanned calls.  Errors as for those calls. */
int fredec_tuples_plan(fredec_ctx* ctx, void* stream, int64_t N, const double* pool_host, int32_t n_pool,
                       const uint64_t* masks_host, int64_t n_tuples, int32_t refine_steps, int32_t precision,
                       void* workspace, size_t ws_bytes, fredec_plan** plan_out);
int fredec_plan_tuples(fredec_ctx* ctx, fredec_plan* plan, void* stream,
                       const double* t, const double* x, const double* w,
                       double* l_out, double* z_out, double* f_out, uint8_t* flags_out, double* l0_out);
int fredec_ascent_plan(fredec_ctx* ctx, void* stream, int64_t N, const int64_t* toff_host, int64_t n_tuples,
                       int32_t steps, double clamp, int32_t precision, void* workspace, size_t ws_bytes,
                       fredec_plan** plan_out);
int fredec_plan_ascent(fredec_ctx* ctx, fredec_plan* plan, void* stream,
                       const double* t, const double* x, const double* w, double* f,
                       double* z_out, double* l_out, uint8_t* flags_out);

/* Global-local residual periodogram (Sect. 2, the statistic with a locally
 * re-optimised base model defined after eq. zpowrel) -------------------------
 * One series t, x, w (device, N samples) and base frequencies f'
 * (host base_f[m], m <= FREDEC_MAX_BASE).  The base model is first refined
 * by Gauss-Newton from f' (the step control of fredec_tuples, refine_steps
 * trial points): l_b = l_{m,loc}(f'_loc).  Then for every grid frequency
 * f_j = (j+1) df, j < F, the model with the m base frequencies and f_j is
 * refined the same way from (f'_loc, f_j) with f_j held fixed (its
 * Gauss-Newton step is zero; the base frequencies move):
 *     z_j = (N - 3m - 4)/2 ln(l_b / l_{1|m,loc}(f_j | f'_loc)),
 * whose maximum over the grid is the global-local statistic.  Flags as for
 * fredec_scan: f_j within 0.05 / T_eff of a refined base frequency: z = 0,
 * FREDEC_FLAG_MASKED; a degenerate start: z = 0, FREDEC_FLAG_SINGULAR; l <= 0:
 * z = +inf, FREDEC_FLAG_PERFECT.  float64 throughout (Gram passes on the
 * float64 matrix cores); the grid runs in chunks of at most 65536 points.
 * Outputs: z_out (device [F]), flags_out (device [F], nullable), l_base_out
 * (device [1], nullable), base_out (device [m], nullable: f'_loc).
 * Synchronises `stream` once (after the base refinement).  Errors: EINVAL,
 * ENOTSUP (m > FREDEC_MAX_BASE), EDOF (N - 3m - 4 <= 0), ENOMEM, ESINGULAR
 * (the base model cannot be fitted). */
int fredec_global_local_workspace(int64_t N, int32_t m, int64_t F, size_t* bytes);
int fredec_global_local(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                        const double* base_f_host, int32_t m, double df, int64_t F, int32_t refine_steps,
                        void* workspace, size_t ws_bytes, double* z_out, uint8_t* flags_out, double* l_base_out,
                        double* base_out);

/* FAP thresholds (eq. zFAP) ------------------------------------------------
 * zc[d], d = 1..n (zc[0] = 0): the z with A_d W^d e^{-z} z^{3d/2-1} = fap on
 * the decreasing branch z > 3d/2 - 1 (bisection, float64, host only).
 * A (host [n+1], nullable = all 1): the constants A~_d, which the paper does
 * not print.  W = f_max T_eff (Sect. 2).  zc: host [n+1]. */
int fredec_zcrit(double W, int32_t n, double fap, const double* A_host, double* zc_host);

/* Periodogram peaks (Sect. 4.2): interior grid points with
 * z_{j-1} < z_j >= z_{j+1}, no flag other than FREDEC_FLAG_RESCORED, and
 * z_j > zmin.  z, flags: device [F] (flags nullable).  Synchronises `stream`;
 * writes up to `cap` peaks sorted by index to the host arrays idx_host,
 * z_host and the total count (possibly above cap) to *n_found. */
int fredec_peaks_workspace(int64_t cap, size_t* bytes);
int fredec_peaks(fredec_ctx* ctx, void* stream, const double* z, const uint8_t* flags, int64_t F, double zmin,
                 void* workspace, size_t ws_bytes, int64_t cap, int64_t* idx_host, double* z_host,
                 int64_t* n_found);

/* Phase 3 backward cascade (Sect. 4.4; the 2^m - 1 joint tests of Sect. 2)
 * over all subsets of a pool of n <= FREDEC_MAX_POOL frequencies.  ltab
 * (device [2^n], float64): l of every subset indexed by its mask, ltab[0] =
 * l_0 (constant model); non-finite entries fail every test.  Subset S
 * survives iff for every proper subset S' (the empty one included)
 *   (N - 3|S| - 1)/2 ln(l(S') / l(S)) > zcrit[|S| - |S'|]
 * (zcrit host [n+1]).  Outputs (device [2^n]): survive_out, maximal_out
 * (survivors with no surviving strict superset: the output sets, which are
 * never nested) and G_out (nullable) = l(S) (N - 1) / (N - 3|S| - 1), the
 * goodness of fit of Sect. 6. */
int fredec_cascade_workspace(int32_t n, size_t* bytes);
int fredec_cascade(fredec_ctx* ctx, void* stream, const double* ltab, int32_t n, int64_t N,
                   const double* zcrit_host, void* workspace, size_t ws_bytes, uint8_t* survive_out,
                   uint8_t* maximal_out, double* G_out);

/* Phase 1 preliminary scan (Sect. 4.2): residual scans on the grid
 * f_j = (j+1) df, j < F, starting from the constant model.  In each scan the
 * peaks with z > zc1 (single-frequency FAP below fap1) and z >= z_max / 2 join
 * the pool unless within 0.5 / T_eff of a member (the earlier one is kept);
 * the highest peak's grid frequency joins the base model while its z exceeds
 * zc0 (FAP below fap0); otherwise the phase ends.  The pool is then capped at
 * pool_cap (N/10 if pool_cap <= 0) by dropping the largest-FAP candidates
 * (ties: the higher frequency) and sorted by frequency.  A1: A~_1 of eq. zFAP.
 * With FREDEC_FP32 the scans use the reduced-precision sums and every peak
 * that can still reach z_max / 2 (float32 z within 1e-3 of half the largest
 * float32 peak, a margin 1000 times the float32 bound) is followed uphill in
 * float64 (fredec_scan_at) before any decision, so that the decisions are
 * taken on float64 values.  Synchronises `stream`.
 * Host outputs: pool_out / pool_z_out [pool capacity], *n_pool, base_out
 * [max_scans], *n_base, *n_scans, *truncated (candidates dropped by the cap),
 * *W_out = F df T_eff.  Errors: EINVAL (including fap1 < fap0), a per-series
 * status code of the first scan (EWEIGHT, EDEGEN), ENOMEM. */
int fredec_phase1_workspace(int64_t N, int64_t F, int32_t max_scans, int32_t precision, size_t* bytes);
int fredec_phase1(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                  double df, int64_t F, double fap0, double fap1, double A1, int32_t pool_cap, int32_t max_scans,
                  int32_t precision, void* workspace, size_t ws_bytes, double* pool_out, double* pool_z_out,
                  int32_t* n_pool, double* base_out, int32_t* n_base, int32_t* n_scans, int32_t* truncated,
                  double* W_out);

/* Residual single-frequency FAP of each solution (Sect. 6: the per-solution
 * output lists the FAP of the largest peak left in the residual periodogram;
 * eq. zFAP with n = 1).  Solution k has the frequencies
 * sol_f[sol_off[k] .. sol_off[k+1]) (host arrays, sol_off[0] = 0, at most
 * FREDEC_MAX_BASE each).  For each, the residual scan of fredec_scan on the
 * grid f_j = (j+1) df, j < F, with those frequencies as the base model; its
 * highest interior local maximum by the rule of fredec_peaks (largest z,
 * ties -> lowest index) z_max at grid index j_max; and
 *     FAP = min(1, A1 W e^{-z_max} z_max^{1/2}),   W = F df T_eff.
 * With FREDEC_FP32 the scans use the reduced-precision sums; the peaks within
 * 1e-4 max(z, 1) of the float32 maximum are followed uphill in float64
 * (fredec_scan_at) and the maximum is taken over the float64 values.
 * Synchronises `stream` after every scan.  Host outputs [n_sol]: fap_out,
 * zmax_out, jmax_out (a periodogram without peak: FAP 1, z NaN, j -1).
 * Errors: EINVAL, ENOTSUP (a solution above FREDEC_MAX_BASE), EDOF
 * (N - 3(m_max + 1) - 1 <= 0), ENOMEM, a series status code (EWEIGHT,
 * EDEGEN, ESINGULAR for a singular solution). */
int fredec_residual_fap_workspace(int64_t N, int64_t F, int32_t m_max, int32_t precision, size_t* bytes);
int fredec_residual_fap(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                        const double* sol_f_host, const int64_t* sol_off_host, int32_t n_sol, double df, int64_t F,
                        double A1, int32_t precision, void* workspace, size_t ws_bytes, double* fap_out,
                        double* zmax_out, int64_t* jmax_out);

#ifdef __cplusplus
}
#endif

#endif /* FREDEC_H */
