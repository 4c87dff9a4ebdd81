// C ABI of the tuple statistics: fredec_tuples (all subsets of a pool, fixed
// or refined frequencies), fredec_grad (z and dz/df of ragged tuples),
// fredec_adjoint (dz/df of an earlier forward evaluation) and fredec_ascent
// (fixed-step preconditioned ascent).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fredec_api_internal.h"
#include "fredec_tuples_internal.h"

using namespace fredec;

namespace {

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

int popcount64(uint64_t v) { return __builtin_popcountll(v); }

// Host-side plan of a tuple batch: descriptors and workspace layout.
struct TuplePlan {
  std::vector<TupleDesc> desc;
  std::vector<int32_t> order;  // tuple indices sorted by (Gram blocks, size)
  struct Group {
    int nb;         // 16-column Gram blocks
    int nf;         // frequencies of every tuple of the group
    int64_t begin;  // first position in `order`
    int count;
  };
  std::vector<Group> groups;
  int64_t N = 0;  // samples of the series
  int32_t precision = FREDEC_FP64;
  int64_t nf = 0, ngram = 0, nscratch = 0, ntheta = 0;
  int max_n = 0;
  size_t off_sin = 0, off_hdr = 0, off_com = 0, off_tau = 0, off_xt = 0, off_wt = 0, off_desc = 0, off_order = 0,
         off_state = 0, off_ftry = 0, off_facc = 0, off_step = 0, off_theta = 0, off_gram = 0, off_scr = 0,
         off_g = 0, off_h = 0, off_members = 0, off_f0 = 0, total = 0;
};

// sizes[k] = number of frequencies of tuple k; gn = whether Gauss-Newton
// columns are needed (refinement).
int make_plan(int64_t N, const std::vector<int>& sizes, bool gn, TuplePlan& P) {
  P.N = N;
  const int64_t nt = static_cast<int64_t>(sizes.size());
  if (nt <= 0 || nt > (int64_t(1) << 30)) return FREDEC_EINVAL;
  P.desc.resize(nt);
  for (int64_t k = 0; k < nt; ++k) {
    const int n = sizes[k];
    if (n < 1) return FREDEC_EINVAL;
    if (n > MAXPOOL) return FREDEC_ENOTSUP;
    P.max_n = std::max(P.max_n, n);
    const int C = gn ? 4 * n + 2 : 2 * n + 2;
    const int K = 2 * n + 1;
    TupleDesc& d = P.desc[k];
    d.n = n;
    d.nb = (C + 15) / 16;
    d.foff = P.nf;
    d.thoff = P.ntheta;
    d.frozen = 0;
    P.nf += n;
    P.ntheta += K;
  }
  if (N - 3 * static_cast<int64_t>(P.max_n) - 1 <= 0) return FREDEC_EDOF;
  // launch order: by column blocks, then size, stable in the tuple index.
  // The blocks grow with the size, so this is a stable counting sort by size
  // (linear: 2^16 - 1 subsets of a pool of 16 are planned in well under 1 ms).
  P.order.resize(nt);
  {
    std::vector<int64_t> first(MAXPOOL + 2, 0);
    for (int64_t k = 0; k < nt; ++k) ++first[P.desc[k].n + 1];
    for (int n = 1; n <= MAXPOOL + 1; ++n) first[n] += first[n - 1];
    for (int64_t k = 0; k < nt; ++k) P.order[first[P.desc[k].n]++] = static_cast<int32_t>(k);
  }
  for (int64_t k = 0; k < nt; ++k) {
    const TupleDesc& d = P.desc[P.order[k]];
    if (P.groups.empty() || P.groups.back().nb != d.nb || P.groups.back().nf != d.n)
      P.groups.push_back(TuplePlan::Group{d.nb, d.n, k, 0});
    P.groups.back().count++;
  }
  // Gram matrices and solve scratch, interleaved within each size group
  for (const auto& g : P.groups) {
    const int n = g.nf;
    const int C = gn ? 4 * n + 2 : 2 * n + 2;
    const int K = 2 * n + 1;
    for (int64_t j = 0; j < g.count; ++j) {
      TupleDesc& d = P.desc[P.order[g.begin + j]];
      d.goff = P.ngram + j;
      d.soff = P.nscratch + j;
      d.gs = static_cast<int32_t>(g.count);
    }
    P.ngram += static_cast<int64_t>(C) * (C + 1) / 2 * g.count;
    P.nscratch += (gn ? static_cast<int64_t>(K) * n + n * (n + 1) / 2 + n : 0) * g.count;
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  P.off_sin = take(sizeof(SeriesIn));
  P.off_hdr = take(sizeof(SeriesHdr));
  P.off_com = take(sizeof(TupleCommon));
  P.off_tau = take(sizeof(double) * N);
  P.off_xt = take(sizeof(double) * N);
  P.off_wt = take(sizeof(double) * N);
  P.off_desc = take(sizeof(TupleDesc) * nt);
  P.off_order = take(sizeof(int32_t) * nt);
  P.off_state = take(sizeof(TupleState) * nt);
  P.off_ftry = take(sizeof(double) * P.nf);
  P.off_facc = take(sizeof(double) * P.nf);
  P.off_step = take(sizeof(double) * P.nf);
  P.off_theta = take(sizeof(double) * P.ntheta);
  P.off_gram = take(sizeof(double) * P.ngram);
  P.off_scr = take(sizeof(double) * P.nscratch);
  P.off_g = take(sizeof(double) * P.nf);
  P.off_h = take(sizeof(double) * P.nf);
  P.off_members = take(P.nf);
  P.off_f0 = take(sizeof(double) * P.nf);
  P.total = off;
  return FREDEC_OK;
}

// Device pointers of a planned workspace.
struct TupleDev {
  SeriesIn* sin;
  SeriesHdr* hdr;
  TupleCommon* com;
  double *tau, *xt, *wt;
  TupleDesc* desc;
  int32_t* order;
  TupleState* state;
  double *ftry, *facc, *step, *theta, *gram, *scr, *g, *h;
  int8_t* members;
  double* f0;  // starting frequencies of a subset batch
};

TupleDev dev_ptrs(void* ws, const TuplePlan& P) {
  TupleDev D;
  D.sin = at<SeriesIn>(ws, P.off_sin);
  D.hdr = at<SeriesHdr>(ws, P.off_hdr);
  D.com = at<TupleCommon>(ws, P.off_com);
  D.tau = at<double>(ws, P.off_tau);
  D.xt = at<double>(ws, P.off_xt);
  D.wt = at<double>(ws, P.off_wt);
  D.desc = at<TupleDesc>(ws, P.off_desc);
  D.order = at<int32_t>(ws, P.off_order);
  D.state = at<TupleState>(ws, P.off_state);
  D.ftry = at<double>(ws, P.off_ftry);
  D.facc = at<double>(ws, P.off_facc);
  D.step = at<double>(ws, P.off_step);
  D.theta = at<double>(ws, P.off_theta);
  D.gram = at<double>(ws, P.off_gram);
  D.scr = at<double>(ws, P.off_scr);
  D.g = at<double>(ws, P.off_g);
  D.h = at<double>(ws, P.off_h);
  D.members = at<int8_t>(ws, P.off_members);
  D.f0 = at<double>(ws, P.off_f0);
  return D;
}

// Series and tuple descriptors into the workspace (asynchronous on `st`).
int upload_descriptors(fredec_ctx* ctx, hipStream_t st, const TuplePlan& P, const TupleDev& D, int64_t N) {
  SeriesIn si;
  std::memset(&si, 0, sizeof(si));
  si.N = N;
  si.F = 1;
  int rc;
  if ((rc = upload(ctx, st, D.sin, &si, sizeof(si)))) return rc;
  if ((rc = upload(ctx, st, D.desc, P.desc.data(), sizeof(TupleDesc) * P.desc.size()))) return rc;
  return upload(ctx, st, D.order, P.order.data(), sizeof(int32_t) * P.order.size());
}

// Normalisation of the series and reset of the per-tuple state (kernels only).
int normalise(hipStream_t st, const TuplePlan& P, const TupleDev& D, const double* t, const double* x,
              const double* w, int64_t N) {
  if (launch_prep(st, 1, 0, 0, D.sin, D.hdr, t, x, w, D.tau, D.xt, D.wt, nullptr, nullptr, nullptr, nullptr,
                  nullptr, nullptr, nullptr, nullptr, 0) !=
      hipSuccess)
    return FREDEC_EDEVICE;
  if (launch_tuple_common(st, D.hdr, N, D.com) != hipSuccess) return FREDEC_EDEVICE;
  if (launch_tuple_init(st, static_cast<int>(P.desc.size()), D.state) != hipSuccess) return FREDEC_EDEVICE;
  return FREDEC_OK;
}

// Launches fn(group, stream) for every size group of the plan.  The groups
// write disjoint outputs, so they run concurrently on the caller's stream and
// the context's side streams (each group, largest estimated work first, onto
// the least loaded stream), which lets the small groups and the last, partly
// filled rounds of the large ones overlap; the side streams are joined back
// to the caller's stream before this returns (also after a failed launch, so
// that no side stream is left forked).
template <class Launch>
int launch_groups(const fredec_ctx* ctx, hipStream_t st, const TuplePlan& P, int mode, Launch&& fn) {
  const int ng = static_cast<int>(P.groups.size());
  const int nst = std::min(ng, 1 + fredec_ctx::NSIDE);
  std::vector<int> idx(ng), on(ng, 0);
  for (int k = 0; k < ng; ++k) idx[k] = k;
  auto work = [&](int k) {
    const int n = P.groups[k].nf;
    const double C = mode == TUPLE_GN ? 4.0 * n + 2.0 : 2.0 * n + 2.0;
    return static_cast<double>(P.groups[k].count) * C * C;
  };
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return work(a) > work(b); });
  std::vector<double> load(nst, 0.0);
  for (int k : idx) {
    const int s = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
    on[k] = s;
    load[s] += work(k);
  }
  if (nst > 1) {
    if (hipEventRecord(ctx->fork_ev, st) != hipSuccess) return FREDEC_EDEVICE;
    for (int s = 1; s < nst; ++s)
      if (hipStreamWaitEvent(ctx->side[s - 1], ctx->fork_ev, 0) != hipSuccess) return FREDEC_EDEVICE;
  }
  int rc = FREDEC_OK;
  for (int k = 0; k < ng && rc == FREDEC_OK; ++k)
    if (!fn(P.groups[k], on[k] == 0 ? st : ctx->side[on[k] - 1])) rc = FREDEC_EDEVICE;
  for (int s = 1; s < nst; ++s) {
    if (hipEventRecord(ctx->join_ev[s - 1], ctx->side[s - 1]) != hipSuccess ||
        hipStreamWaitEvent(st, ctx->join_ev[s - 1], 0) != hipSuccess)
      rc = FREDEC_EDEVICE;
  }
  return rc;
}

// One Gram pass (the size groups concurrently).  fuse_solve: the lane-group
// kernels make the forward solve themselves (else they store the Gram).
int gram_pass(fredec_ctx* ctx, hipStream_t st, const TuplePlan& P, const TupleDev& D, int mode,
              bool fuse_solve = true) {
  ProfScope prof(ctx, st, FREDEC_PROF_GRAM);
  return launch_groups(ctx, st, P, mode, [&](const TuplePlan::Group& g, hipStream_t gs) {
    return launch_tuple_gram(gs, g.nf, ctx->n_cu, g.nf < 8 ? ctx->tuple_lanes[g.nf] : 0, D.desc, D.order + g.begin,
                             g.count, P.N, D.com, D.tau, D.xt, D.wt, D.ftry, D.state, D.gram, mode,
                             P.precision == FREDEC_FP32, D.facc, D.theta, fuse_solve) == hipSuccess;
  });
}

// Adjoint gradient of every tuple (forward state, theta* and f in the
// workspace), the size groups concurrently.
int adjoint_pass(fredec_ctx* ctx, hipStream_t st, const TuplePlan& P, const TupleDev& D, const double* f,
                 double* dzdf, double* hout) {
  ProfScope prof(ctx, st, FREDEC_PROF_ADJOINT);
  return launch_groups(ctx, st, P, TUPLE_FWD, [&](const TuplePlan::Group& g, hipStream_t gs) {
    return launch_tuple_adjoint(gs, g.nf, ctx->n_cu, g.nf < 8 ? ctx->tuple_lanes[g.nf] : 0, D.desc, D.order + g.begin,
                                g.count, P.N, D.com, D.tau, D.xt, D.wt, f, D.theta, D.state, dzdf, hout,
                                P.precision == FREDEC_FP32) == hipSuccess;
  });
}

// The first pass of a batch of pool subsets evaluated at the pool
// frequencies: their Gram matrices are gathered from the pool's Gram.
struct PoolPass {
  const double* pool_gram;  // packed lower Gram of the whole pool (element stride 1)
  int n_pool;
};

// Forward evaluation (and optional Gauss-Newton refinement) of every tuple.
int run_fit(fredec_ctx* ctx, hipStream_t st, const TuplePlan& P, const TupleDev& D, int refine_steps,
            const PoolPass* first = nullptr) {
  const int nt = static_cast<int>(P.desc.size());
  const int mode = refine_steps > 0 ? TUPLE_GN : TUPLE_FWD;
  // the lane-group kernels solve their tuples in a Gram pass; their groups
  // are a prefix of `order` (sorted by size), positions 0 .. fused
  int fused = 0;
  for (const auto& g : P.groups) {
    if (!tuple_lanes_supported(g.nf, mode)) break;
    fused = static_cast<int>(g.begin + g.count);
  }
  for (int it = 0; it <= refine_steps; ++it) {
    int rc = FREDEC_OK;
    int sb = 0;  // first position the solve kernel takes
    if (it == 0 && first) {
      ProfScope prof(ctx, st, FREDEC_PROF_GRAM);
      if (launch_tuple_gather(st, D.desc, D.order, nt, D.members, first->pool_gram, first->n_pool, mode, D.gram) !=
          hipSuccess)
        return FREDEC_EDEVICE;
    } else {
      rc = gram_pass(ctx, st, P, D, mode);
      sb = fused;
    }
    if (rc) return rc;
    if (sb >= nt) continue;
    ProfScope prof(ctx, st, FREDEC_PROF_SOLVE);
    if (launch_tuple_solve(st, D.desc, D.order + sb, nt - sb, D.com, D.gram, D.scr, D.ftry, D.facc, D.step, D.theta,
                           D.state, mode, it == refine_steps ? 1 : 0) != hipSuccess)
      return FREDEC_EDEVICE;
  }
  return FREDEC_OK;
}

int check_series_args(const double* t, const double* x, const double* w, int64_t N) {
  if (!t || !x || !w || N <= 0) return FREDEC_EINVAL;
  return FREDEC_OK;
}

int sizes_from_toff(const int64_t* toff, int64_t n_tuples, std::vector<int>& sizes) {
  if (!toff || n_tuples <= 0 || toff[0] != 0) return FREDEC_EINVAL;
  sizes.resize(n_tuples);
  for (int64_t k = 0; k < n_tuples; ++k) {
    const int64_t n = toff[k + 1] - toff[k];
    if (n < 1) return FREDEC_EINVAL;
    if (n > MAXPOOL) return FREDEC_ENOTSUP;
    sizes[k] = static_cast<int>(n);
  }
  return FREDEC_OK;
}

int sizes_from_masks(int32_t n_pool, const uint64_t* masks, int64_t n_tuples, std::vector<int>& sizes) {
  if (n_pool < 1) return FREDEC_EINVAL;
  if (n_pool > MAXPOOL) return FREDEC_ENOTSUP;
  const uint64_t full = (uint64_t(1) << n_pool) - 1;
  if (!masks && n_tuples != static_cast<int64_t>(full)) return FREDEC_EINVAL;
  if (n_tuples <= 0) return FREDEC_EINVAL;
  sizes.resize(n_tuples);
  for (int64_t k = 0; k < n_tuples; ++k) {
    const uint64_t m = masks ? masks[k] : static_cast<uint64_t>(k + 1);
    if (m == 0 || (m & ~full)) return FREDEC_EINVAL;
    sizes[k] = popcount64(m);
  }
  return FREDEC_OK;
}

// A batch of pool subsets (fredec_tuples) ready to launch.
struct SubsetPlan : fredec_plan {
  SubsetPlan() : fredec_plan(TUPLES) {}
  TuplePlan T;
  int64_t N = 0;
  int32_t n_pool = 0, refine_steps = 0;
  std::vector<double> f0;   // starting frequencies of the members, in bit order
  std::vector<int8_t> mem;  // pool index of each member
  // the whole pool as one tuple, whose Gram gives every subset's first-pass
  // Gram (used when the pool fits the model: N - 3 n_pool - 1 > 0)
  bool use_pool = false;
  TuplePlan Pp;
  size_t off_pool = 0;
  std::vector<double> pool;
};

// Workspace of a batch of pool subsets: the subsets' plan, then the pool's.
int subset_layout(int64_t N, int32_t n_pool, const std::vector<int>& sizes, bool gn, TuplePlan& T, TuplePlan& Pp,
                  bool& use_pool, size_t& off_pool, size_t& total) {
  int rc = make_plan(N, sizes, gn, T);
  if (rc) return rc;
  use_pool = make_plan(N, std::vector<int>(1, n_pool), gn, Pp) == FREDEC_OK;
  off_pool = align_up(T.total);
  total = use_pool ? off_pool + Pp.total : T.total;
  return FREDEC_OK;
}

int subset_build(int64_t N, const double* pool, int32_t n_pool, const uint64_t* masks, int64_t n_tuples,
                 int32_t refine_steps, int32_t precision, void* ws, size_t ws_bytes, SubsetPlan& P) {
  if (!pool || refine_steps < 0) return FREDEC_EINVAL;
  if (precision != FREDEC_FP64 && precision != FREDEC_FP32) return FREDEC_EINVAL;
  std::vector<int> sizes;
  int rc;
  if ((rc = sizes_from_masks(n_pool, masks, n_tuples, sizes))) return rc;
  for (int k = 0; k < n_pool; ++k)
    if (!std::isfinite(pool[k])) return FREDEC_EINVAL;
  size_t total = 0;
  if ((rc = subset_layout(N, n_pool, sizes, refine_steps > 0, P.T, P.Pp, P.use_pool, P.off_pool, total))) return rc;
  P.T.precision = precision;
  P.Pp.precision = precision;
  if (!ws || ws_bytes < total) return FREDEC_ENOMEM;
  P.ws = ws;
  P.ws_bytes = ws_bytes;
  P.N = N;
  P.n_pool = n_pool;
  P.pool.assign(pool, pool + n_pool);
  P.refine_steps = refine_steps;
  P.f0.resize(P.T.nf);
  P.mem.resize(P.T.nf);
  for (int64_t k = 0; k < n_tuples; ++k) {
    const uint64_t m = masks ? masks[k] : static_cast<uint64_t>(k + 1);
    int64_t o = P.T.desc[k].foff;
    for (int b = 0; b < n_pool; ++b)
      if (m >> b & 1) {
        P.f0[o] = pool[b];
        P.mem[o] = static_cast<int8_t>(b);
        ++o;
      }
  }
  return FREDEC_OK;
}

int subset_upload(fredec_ctx* ctx, hipStream_t st, const SubsetPlan& P) {
  const TupleDev D = dev_ptrs(P.ws, P.T);
  int rc;
  if ((rc = upload_descriptors(ctx, st, P.T, D, P.N))) return rc;
  if ((rc = upload(ctx, st, D.f0, P.f0.data(), sizeof(double) * P.T.nf))) return rc;
  if ((rc = upload(ctx, st, D.members, P.mem.data(), P.T.nf))) return rc;
  if (!P.use_pool) return FREDEC_OK;
  const TupleDev Dp = dev_ptrs(static_cast<char*>(P.ws) + P.off_pool, P.Pp);
  if ((rc = upload_descriptors(ctx, st, P.Pp, Dp, P.N))) return rc;
  return upload(ctx, st, Dp.f0, P.pool.data(), sizeof(double) * P.n_pool);
}

// Kernels only (capturable).
int subset_launch(fredec_ctx* ctx, hipStream_t st, const SubsetPlan& P, const double* t, const double* x,
                  const double* w, double* l_out, double* z_out, double* f_out, uint8_t* flags_out, double* l0_out) {
  const TupleDev D = dev_ptrs(P.ws, P.T);
  int rc;
  if ((rc = normalise(st, P.T, D, t, x, w, P.N))) return rc;
  if (launch_copy_f64(st, D.f0, D.ftry, P.T.nf) != hipSuccess) return FREDEC_EDEVICE;
  PoolPass first{nullptr, P.n_pool};
  if (P.use_pool) {
    // the Gram of the whole pool at its frequencies (one tuple)
    const TupleDev Dp = dev_ptrs(static_cast<char*>(P.ws) + P.off_pool, P.Pp);
    if ((rc = normalise(st, P.Pp, Dp, t, x, w, P.N))) return rc;
    if (launch_copy_f64(st, Dp.f0, Dp.ftry, P.n_pool) != hipSuccess) return FREDEC_EDEVICE;
    if ((rc = gram_pass(ctx, st, P.Pp, Dp, P.refine_steps > 0 ? TUPLE_GN : TUPLE_FWD, /*fuse_solve=*/false))) return rc;
    first.pool_gram = Dp.gram;
  }
  if ((rc = run_fit(ctx, st, P.T, D, P.refine_steps, P.use_pool ? &first : nullptr))) return rc;
  if (launch_tuple_finish(st, D.desc, static_cast<int>(P.T.desc.size()), D.com, D.state, D.facc, l_out, z_out,
                          flags_out, f_out, D.members, P.n_pool) != hipSuccess)
    return FREDEC_EDEVICE;
  if (l0_out && launch_tuple_l0(st, D.state, l0_out) != hipSuccess) return FREDEC_EDEVICE;
  return FREDEC_OK;
}

// A batch of ragged tuples for the fixed-step ascent, ready to launch.
struct AscentPlan : fredec_plan {
  AscentPlan() : fredec_plan(ASCENT) {}
  TuplePlan T;
  int64_t N = 0;
  int32_t steps = 0;
  double clamp = 0.0;
};

int ascent_build(int64_t N, const int64_t* toff, int64_t n_tuples, int32_t steps, double clamp, int32_t precision,
                 void* ws, size_t ws_bytes, AscentPlan& P) {
  if (steps < 0 || !(clamp > 0.0) || !std::isfinite(clamp)) return FREDEC_EINVAL;
  if (precision != FREDEC_FP64 && precision != FREDEC_FP32) return FREDEC_EINVAL;
  std::vector<int> sizes;
  int rc;
  if ((rc = sizes_from_toff(toff, n_tuples, sizes))) return rc;
  if ((rc = make_plan(N, sizes, false, P.T))) return rc;
  P.T.precision = precision;
  if (!ws || ws_bytes < P.T.total) return FREDEC_ENOMEM;
  P.ws = ws;
  P.ws_bytes = ws_bytes;
  P.N = N;
  P.steps = steps;
  P.clamp = clamp;
  return FREDEC_OK;
}

// Kernels only (capturable): `steps` times forward, adjoint and update, then
// the final forward evaluation.
int ascent_launch(fredec_ctx* ctx, hipStream_t st, const AscentPlan& P, const double* t, const double* x,
                  const double* w, double* f, double* z_out, double* l_out, uint8_t* flags_out) {
  const TupleDev D = dev_ptrs(P.ws, P.T);
  const int nt = static_cast<int>(P.T.desc.size());
  int rc;
  if ((rc = normalise(st, P.T, D, t, x, w, P.N))) return rc;
  if (launch_copy_f64(st, f, D.ftry, P.T.nf) != hipSuccess) return FREDEC_EDEVICE;
  for (int s = 0; s < P.steps; ++s) {
    if ((rc = run_fit(ctx, st, P.T, D, 0))) return rc;
    if ((rc = adjoint_pass(ctx, st, P.T, D, D.ftry, D.g, D.h))) return rc;
    if (launch_tuple_ascent_update(st, D.desc, nt, D.com, D.g, D.h, D.ftry, P.clamp, D.state) != hipSuccess)
      return FREDEC_EDEVICE;
  }
  if ((rc = run_fit(ctx, st, P.T, D, 0))) return rc;
  if (launch_tuple_finish(st, D.desc, nt, D.com, D.state, D.facc, l_out, z_out, flags_out, nullptr, nullptr, 0) !=
      hipSuccess)
    return FREDEC_EDEVICE;
  if (launch_copy_f64(st, D.ftry, f, P.T.nf) != hipSuccess) return FREDEC_EDEVICE;
  return FREDEC_OK;
}


// Workspace of the global-local residual periodogram: the base model's
// refinement (one tuple of m frequencies, m > 0), then the trial tuples of one
// chunk of the grid (cg tuples of m + 1 frequencies, the last frozen) and of
// the shorter last chunk, which reuses the same memory.
struct GlobalLocalLayout {
  TuplePlan base, chunk, tail;
  int64_t cg = 0, tail_count = 0;
  size_t off_chunk = 0, total = 0;
};

constexpr size_t GL_CHUNK_BYTES = size_t(256) << 20;  // largest chunk workspace (below 65536 tuples)

int gl_layout(int64_t N, int32_t m, int64_t F, GlobalLocalLayout& L) {
  if (N <= 0 || m < 0 || F < 1) return FREDEC_EINVAL;
  if (m > FREDEC_MAX_BASE) return FREDEC_ENOTSUP;
  if (N - 3 * (static_cast<int64_t>(m) + 1) - 1 <= 0) return FREDEC_EDOF;
  int rc;
  if (m > 0 && (rc = make_plan(N, std::vector<int>(1, m), true, L.base))) return rc;
  L.cg = std::min<int64_t>(F, 65536);
  for (;;) {
    L.chunk = TuplePlan();
    if ((rc = make_plan(N, std::vector<int>(static_cast<size_t>(L.cg), m + 1), true, L.chunk))) return rc;
    if (L.chunk.total <= GL_CHUNK_BYTES || L.cg <= 1024) break;
    L.cg = std::max<int64_t>(L.cg / 2, 1024);
  }
  L.tail_count = F % L.cg;
  if (L.tail_count && (rc = make_plan(N, std::vector<int>(static_cast<size_t>(L.tail_count), m + 1), true, L.tail)))
    return rc;
  for (TupleDesc& d : L.chunk.desc) d.frozen = 1 << m;
  for (TupleDesc& d : L.tail.desc) d.frozen = 1 << m;
  L.off_chunk = m > 0 ? align_up(L.base.total) : 0;
  L.total = L.off_chunk + L.chunk.total;
  return FREDEC_OK;
}

}  // namespace

extern "C" {

int fredec_tuples_workspace(int64_t N, int32_t n_pool, const uint64_t* masks, int64_t n_tuples, int32_t refine_steps,
                            size_t* bytes) {
  if (!bytes || N <= 0 || refine_steps < 0) return FREDEC_EINVAL;
  std::vector<int> sizes;
  int rc = sizes_from_masks(n_pool, masks, n_tuples, sizes);
  if (rc) return rc;
  TuplePlan T, Pp;
  bool use_pool = false;
  size_t off_pool = 0, total = 0;
  if ((rc = subset_layout(N, n_pool, sizes, refine_steps > 0, T, Pp, use_pool, off_pool, total))) return rc;
  *bytes = total;
  return FREDEC_OK;
}

int fredec_tuples(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                  const double* pool, int32_t n_pool, const uint64_t* masks, int64_t n_tuples, int32_t refine_steps,
                  int32_t precision, void* ws, size_t ws_bytes, double* l_out, double* z_out, double* f_out,
                  uint8_t* flags_out, double* l0_out) {
  int rc = check_series_args(t, x, w, N);
  if (rc) return rc;
  SubsetPlan P;
  if ((rc = subset_build(N, pool, n_pool, masks, n_tuples, refine_steps, precision, ws, ws_bytes, P))) return rc;
  if (!ctx) return FREDEC_EINVAL;
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = subset_upload(ctx, st, P))) return rc;
  return subset_launch(ctx, st, P, t, x, w, l_out, z_out, f_out, flags_out, l0_out);
}

int fredec_tuples_plan(fredec_ctx* ctx, void* stream, int64_t N, const double* pool, int32_t n_pool,
                       const uint64_t* masks, int64_t n_tuples, int32_t refine_steps, int32_t precision, void* ws,
                       size_t ws_bytes, fredec_plan** plan_out) {
  if (!plan_out) return FREDEC_EINVAL;
  *plan_out = nullptr;
  if (N <= 0) return FREDEC_EINVAL;
  SubsetPlan* P = new (std::nothrow) SubsetPlan();
  if (!P) return FREDEC_ENOMEM;
  int rc = subset_build(N, pool, n_pool, masks, n_tuples, refine_steps, precision, ws, ws_bytes, *P);
  if (!rc && !ctx) rc = FREDEC_EINVAL;
  if (!rc) {
    DeviceGuard g(ctx->device);
    P->device = ctx->device;
    rc = subset_upload(ctx, static_cast<hipStream_t>(stream), *P);
    if (!rc) rc = upload_wait(ctx);
    std::vector<double>().swap(P->f0);
    std::vector<int8_t>().swap(P->mem);
    std::vector<double>().swap(P->pool);
  }
  if (rc) {
    delete P;
    return rc;
  }
  *plan_out = P;
  return FREDEC_OK;
}

int fredec_plan_tuples(fredec_ctx* ctx, fredec_plan* plan, void* stream, const double* t, const double* x,
                       const double* w, double* l_out, double* z_out, double* f_out, uint8_t* flags_out,
                       double* l0_out) {
  if (!ctx || !plan || plan->kind != fredec_plan::TUPLES || plan->device != ctx->device) return FREDEC_EINVAL;
  const SubsetPlan& P = *static_cast<SubsetPlan*>(plan);
  int rc = check_series_args(t, x, w, P.N);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  return subset_launch(ctx, static_cast<hipStream_t>(stream), P, t, x, w, l_out, z_out, f_out, flags_out, l0_out);
}

int fredec_grad_workspace(int64_t N, const int64_t* toff, int64_t n_tuples, size_t* bytes) {
  if (!bytes || N <= 0) return FREDEC_EINVAL;
  std::vector<int> sizes;
  int rc = sizes_from_toff(toff, n_tuples, sizes);
  if (rc) return rc;
  TuplePlan P;
  if ((rc = make_plan(N, sizes, false, P))) return rc;
  *bytes = P.total;
  return FREDEC_OK;
}

int fredec_grad(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                const double* f, const int64_t* toff, int64_t n_tuples, int32_t precision, void* ws, size_t ws_bytes,
                double* z_out, double* l_out, double* theta_out, double* dz_df, double* h_out, uint8_t* flags_out) {
  int rc = check_series_args(t, x, w, N);
  if (rc) return rc;
  if (!f) return FREDEC_EINVAL;
  if (precision != FREDEC_FP64 && precision != FREDEC_FP32) return FREDEC_EINVAL;
  std::vector<int> sizes;
  if ((rc = sizes_from_toff(toff, n_tuples, sizes))) return rc;
  TuplePlan P;
  if ((rc = make_plan(N, sizes, false, P))) return rc;
  P.precision = precision;
  if (!ws || ws_bytes < P.total) return FREDEC_ENOMEM;
  if (!ctx) return FREDEC_EINVAL;
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  TupleDev D = dev_ptrs(ws, P);
  if ((rc = upload_descriptors(ctx, st, P, D, N))) return rc;
  if ((rc = normalise(st, P, D, t, x, w, N))) return rc;
  if (launch_copy_f64(st, f, D.ftry, P.nf) != hipSuccess) return FREDEC_EDEVICE;
  if ((rc = run_fit(ctx, st, P, D, 0))) return rc;
  const int nt = static_cast<int>(n_tuples);
  if (launch_tuple_finish(st, D.desc, nt, D.com, D.state, D.facc, l_out, z_out, flags_out, nullptr, nullptr, 0) !=
      hipSuccess)
    return FREDEC_EDEVICE;
  if (theta_out && launch_copy_f64(st, D.theta, theta_out, P.ntheta) != hipSuccess) return FREDEC_EDEVICE;
  if ((dz_df || h_out) && (rc = adjoint_pass(ctx, st, P, D, D.ftry, dz_df, h_out))) return rc;
  return FREDEC_OK;
}

int fredec_adjoint(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                   const double* f, const int64_t* toff, int64_t n_tuples, const double* theta, const double* l,
                   int32_t precision, void* ws, size_t ws_bytes, double* dz_df, double* h_out) {
  int rc = check_series_args(t, x, w, N);
  if (rc) return rc;
  if (!f || !theta || !l) return FREDEC_EINVAL;
  if (precision != FREDEC_FP64 && precision != FREDEC_FP32) return FREDEC_EINVAL;
  std::vector<int> sizes;
  if ((rc = sizes_from_toff(toff, n_tuples, sizes))) return rc;
  TuplePlan P;
  if ((rc = make_plan(N, sizes, false, P))) return rc;
  P.precision = precision;
  if (!ws || ws_bytes < P.total) return FREDEC_ENOMEM;
  if (!ctx) return FREDEC_EINVAL;
  if (!dz_df && !h_out) return FREDEC_OK;
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  TupleDev D = dev_ptrs(ws, P);
  if ((rc = upload_descriptors(ctx, st, P, D, N))) return rc;
  if ((rc = normalise(st, P, D, t, x, w, N))) return rc;
  if (launch_tuple_state_from_l(st, static_cast<int>(n_tuples), l, D.state) != hipSuccess) return FREDEC_EDEVICE;
  if (launch_copy_f64(st, theta, D.theta, P.ntheta) != hipSuccess) return FREDEC_EDEVICE;
  return adjoint_pass(ctx, st, P, D, f, dz_df, h_out);
}

int fredec_vuong_workspace(int64_t N, const int64_t* toff, int64_t n_tuples, size_t* bytes) {
  if (!bytes || N <= 0) return FREDEC_EINVAL;
  std::vector<int> sizes;
  int rc = sizes_from_toff(toff, n_tuples, sizes);
  if (rc) return rc;
  TuplePlan P;
  if ((rc = make_plan(N, sizes, false, P))) return rc;
  *bytes = P.total + align_up(sizeof(double) * static_cast<size_t>(n_tuples) * N) +
           align_up(sizeof(double) * static_cast<size_t>(n_tuples));
  return FREDEC_OK;
}

int fredec_vuong(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                 const double* f, const int64_t* toff, int64_t n_tuples, const double* theta, int64_t ref, void* ws,
                 size_t ws_bytes, double* l_out, double* V_out) {
  int rc = check_series_args(t, x, w, N);
  if (rc) return rc;
  if (!f || !theta || !V_out) return FREDEC_EINVAL;
  std::vector<int> sizes;
  if ((rc = sizes_from_toff(toff, n_tuples, sizes))) return rc;
  if (ref < 0 || ref >= n_tuples || n_tuples > (int64_t(1) << 30)) return FREDEC_EINVAL;
  TuplePlan P;
  if ((rc = make_plan(N, sizes, false, P))) return rc;
  size_t need = 0;
  fredec_vuong_workspace(N, toff, n_tuples, &need);
  if (!ws || ws_bytes < need) return FREDEC_ENOMEM;
  if (!ctx) return FREDEC_EINVAL;
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  TupleDev D = dev_ptrs(ws, P);
  double* d_r = at<double>(ws, P.total);
  double* d_l = l_out ? l_out : at<double>(ws, P.total + align_up(sizeof(double) * static_cast<size_t>(n_tuples) * N));
  if ((rc = upload_descriptors(ctx, st, P, D, N))) return rc;
  if ((rc = normalise(st, P, D, t, x, w, N))) return rc;
  if (launch_tuple_vuong(st, D.desc, static_cast<int>(n_tuples), D.com, D.tau, D.xt, D.wt, f, theta,
                         static_cast<int>(ref), d_r, d_l, V_out) != hipSuccess)
    return FREDEC_EDEVICE;
  return FREDEC_OK;
}

int fredec_global_local_workspace(int64_t N, int32_t m, int64_t F, size_t* bytes) {
  if (!bytes) return FREDEC_EINVAL;
  GlobalLocalLayout L;
  int rc = gl_layout(N, m, F, L);
  if (rc) return rc;
  *bytes = L.total;
  return FREDEC_OK;
}

int fredec_global_local(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                        const double* base_f, int32_t m, double df, int64_t F, int32_t refine_steps, void* ws,
                        size_t ws_bytes, double* z_out, uint8_t* flags_out, double* l_base_out, double* base_out) {
  int rc = check_series_args(t, x, w, N);
  if (rc) return rc;
  if (!z_out || refine_steps < 0 || !std::isfinite(df) || df == 0.0) return FREDEC_EINVAL;
  if (m > 0 && !base_f) return FREDEC_EINVAL;
  for (int q = 0; q < m; ++q)
    if (!std::isfinite(base_f[q])) return FREDEC_EINVAL;
  GlobalLocalLayout L;
  if ((rc = gl_layout(N, m, F, L))) return rc;
  if (!ws || ws_bytes < L.total) return FREDEC_ENOMEM;
  if (!ctx) return FREDEC_EINVAL;
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double* fb = nullptr;
  const double* lb = nullptr;
  if (m > 0) {
    // the base model refined by Gauss-Newton from base_f: l_{m,loc} and f'_loc
    TupleDev B = dev_ptrs(ws, L.base);
    if ((rc = upload_descriptors(ctx, st, L.base, B, N))) return rc;
    if ((rc = normalise(st, L.base, B, t, x, w, N))) return rc;
    if ((rc = upload(ctx, st, B.ftry, base_f, sizeof(double) * m))) return rc;
    if ((rc = run_fit(ctx, st, L.base, B, refine_steps))) return rc;
    TupleState s0;
    if (hipMemcpyAsync(&s0, B.state, sizeof(s0), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return FREDEC_EDEVICE;
    if (!s0.has_acc) return FREDEC_ESINGULAR;
    fb = B.facc;
    lb = &B.state[0].l_acc;
    if (base_out && launch_copy_f64(st, fb, base_out, m) != hipSuccess) return FREDEC_EDEVICE;
  }
  void* cws = static_cast<char*>(ws) + L.off_chunk;
  const TuplePlan* uploaded = nullptr;
  for (int64_t j0 = 0; j0 < F; j0 += L.cg) {
    const int count = static_cast<int>(std::min<int64_t>(L.cg, F - j0));
    const TuplePlan& P = count == L.cg ? L.chunk : L.tail;
    TupleDev D = dev_ptrs(cws, P);
    if (uploaded != &P) {
      if ((rc = upload_descriptors(ctx, st, P, D, N))) return rc;
      uploaded = &P;
    }
    if ((rc = normalise(st, P, D, t, x, w, N))) return rc;
    if (launch_gl_fill(st, fb, m, df, j0, count, D.ftry) != hipSuccess) return FREDEC_EDEVICE;
    if ((rc = run_fit(ctx, st, P, D, refine_steps))) return rc;
    if (launch_gl_finish(st, D.state, count, fb, m, df, j0, D.com, lb, z_out, flags_out,
                         j0 == 0 ? l_base_out : nullptr) != hipSuccess)
      return FREDEC_EDEVICE;
  }
  return FREDEC_OK;
}

int fredec_ascent(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                  double* f, const int64_t* toff, int64_t n_tuples, int32_t steps, double clamp, int32_t precision,
                  void* ws, size_t ws_bytes, double* z_out, double* l_out, uint8_t* flags_out) {
  int rc = check_series_args(t, x, w, N);
  if (rc) return rc;
  if (!f) return FREDEC_EINVAL;
  AscentPlan P;
  if ((rc = ascent_build(N, toff, n_tuples, steps, clamp, precision, ws, ws_bytes, P))) return rc;
  if (!ctx) return FREDEC_EINVAL;
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = upload_descriptors(ctx, st, P.T, dev_ptrs(ws, P.T), N))) return rc;
  return ascent_launch(ctx, st, P, t, x, w, f, z_out, l_out, flags_out);
}

int fredec_ascent_plan(fredec_ctx* ctx, void* stream, int64_t N, const int64_t* toff, int64_t n_tuples, int32_t steps,
                       double clamp, int32_t precision, void* ws, size_t ws_bytes, fredec_plan** plan_out) {
  if (!plan_out) return FREDEC_EINVAL;
  *plan_out = nullptr;
  if (N <= 0) return FREDEC_EINVAL;
  AscentPlan* P = new (std::nothrow) AscentPlan();
  if (!P) return FREDEC_ENOMEM;
  int rc = ascent_build(N, toff, n_tuples, steps, clamp, precision, ws, ws_bytes, *P);
  if (!rc && !ctx) rc = FREDEC_EINVAL;
  if (!rc) {
    DeviceGuard g(ctx->device);
    P->device = ctx->device;
    rc = upload_descriptors(ctx, static_cast<hipStream_t>(stream), P->T, dev_ptrs(ws, P->T), N);
    if (!rc) rc = upload_wait(ctx);
  }
  if (rc) {
    delete P;
    return rc;
  }
  *plan_out = P;
  return FREDEC_OK;
}

int fredec_plan_ascent(fredec_ctx* ctx, fredec_plan* plan, void* stream, const double* t, const double* x,
                       const double* w, double* f, double* z_out, double* l_out, uint8_t* flags_out) {
  if (!ctx || !plan || plan->kind != fredec_plan::ASCENT || plan->device != ctx->device || !f) return FREDEC_EINVAL;
  const AscentPlan& P = *static_cast<AscentPlan*>(plan);
  int rc = check_series_args(t, x, w, P.N);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  return ascent_launch(ctx, static_cast<hipStream_t>(stream), P, t, x, w, f, z_out, l_out, flags_out);
}

}  // extern "C"
