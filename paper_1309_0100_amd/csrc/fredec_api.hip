// C ABI of libfredec: argument checks, workspace layout, uploads of the small
// per-series descriptors and kernel launches.  See include/fredec.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "fredec_internal.h"
#include "fredec_api_internal.h"

using namespace fredec;

namespace fredec {

DeviceGuard::DeviceGuard(int dev) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) cur = -1;
  if (cur != dev && hipSetDevice(dev) == hipSuccess) prev_ = cur;
}
DeviceGuard::~DeviceGuard() {
  if (prev_ >= 0) (void)hipSetDevice(prev_);
}

// Copy `bytes` of host data to device memory `dst` on `st` through the
// context's pinned staging buffer.
int upload(fredec_ctx* ctx, hipStream_t st, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return FREDEC_OK;
  if (ctx->staging_pending) {
    if (hipEventSynchronize(ctx->staging_done) != hipSuccess) return FREDEC_EDEVICE;
    ctx->staging_pending = false;
  }
  if (bytes > ctx->staging_bytes) {
    if (ctx->staging) (void)hipHostFree(ctx->staging);
    ctx->staging = nullptr;
    ctx->staging_bytes = 0;
    size_t cap = std::max<size_t>(bytes, 1 << 20);
    if (hipHostMalloc(&ctx->staging, cap, hipHostMallocDefault) != hipSuccess) return FREDEC_ENOMEM;
    ctx->staging_bytes = cap;
  }
  std::memcpy(ctx->staging, src, bytes);
  if (hipMemcpyAsync(dst, ctx->staging, bytes, hipMemcpyHostToDevice, st) != hipSuccess) return FREDEC_EDEVICE;
  if (hipEventRecord(ctx->staging_done, st) != hipSuccess) return FREDEC_EDEVICE;
  ctx->staging_pending = true;
  return FREDEC_OK;
}

int upload_wait(fredec_ctx* ctx) {
  if (!ctx->staging_pending) return FREDEC_OK;
  if (hipEventSynchronize(ctx->staging_done) != hipSuccess) return FREDEC_EDEVICE;
  ctx->staging_pending = false;
  return FREDEC_OK;
}

size_t align_up(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

ProfScope::ProfScope(fredec_ctx* ctx, hipStream_t st, int kind) : ctx_(ctx), st_(st) {
  if (!ctx_ || !ctx_->profiling) return;
  if (ctx_->prof_used == ctx_->prof_events.size()) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
    ctx_->prof_events.push_back({a, b, kind});
  }
  idx_ = static_cast<long>(ctx_->prof_used++);
  ctx_->prof_events[idx_].kind = kind;
  (void)hipEventRecord(ctx_->prof_events[idx_].begin, st_);
}
ProfScope::~ProfScope() {
  if (idx_ >= 0) (void)hipEventRecord(ctx_->prof_events[idx_].end, st_);
}

}  // namespace fredec

// Scratch memory of the allocation-free scan (fredec_scan_static).  Each GPU
// the library runs on holds its own copy from module load until the process
// ends.  In host code this name is only a stand-in for the symbol: the device
// address of a GPU's copy comes from hipGetSymbolAddress on that device
// (static_scratch_address) and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[FREDEC_STATIC_SCRATCH_BYTES];

namespace {

struct ScanLayout {
  size_t off_sin = 0, off_hdr = 0, off_work = 0, off_tau = 0, off_xt = 0, off_wt = 0, off_rec = 0, off_phi = 0;
  size_t off_g32 = 0, off_aux = 0, off_b16 = 0, off_pt16 = 0, off_list = 0, off_count = 0, off_chunk = 0;
  size_t off_ppart = 0, off_pm = 0, off_part = 0;
  size_t total = 0;
  int nsplit = 1;  // sample chunks of a single series with few frequency tiles
  int64_t Ntot = 0, rec_total = 0, phi_total = 0, g32_total = 0, aux_total = 0, b16_total = 0, pt16_total = 0,
          n_work = 0, F_total = 0;
  int64_t ptiles = 0, ppart_total = 0, pm_total = 0;  // preparation tiles, Gram partials, basis changes
  int max_nt = 1;
};

// Frequencies per workgroup of the scan kernel used for a series (for the
// reduced-precision form the smallest tile of any of its kernels, which
// bounds the work list of any setting).
int64_t scan_tile(int KP, int32_t precision) {
  if (precision == FREDEC_FP32) return 64;
  return static_cast<int64_t>(BLOCK) * scan_freqs_per_thread(KP);
}

// 16-frequency tiles per wave of the split-float16 scan for NT column tiles
// (the context's setting, else the default).
int f16x3_ft_for(const fredec_ctx* ctx, int NT) {
  return (ctx && NT >= 1 && NT <= 4 && ctx->f16x3_ft[NT]) ? ctx->f16x3_ft[NT] : f16x3_freq_tiles(NT);
}

// Checks the host descriptors of a scan batch and computes the workspace layout.
int scan_layout(int32_t n_series, const int64_t* soff, const int64_t* boff, const int64_t* F, int32_t precision,
                ScanLayout& L, bool allow_split = true) {
  if (n_series <= 0 || !soff || !boff || !F) return FREDEC_EINVAL;
  if (precision != FREDEC_FP64 && precision != FREDEC_FP32) return FREDEC_EINVAL;
  if (soff[0] < 0 || boff[0] < 0) return FREDEC_EINVAL;
  for (int32_t s = 0; s < n_series; ++s) {
    const int64_t N = soff[s + 1] - soff[s];
    const int64_t m = boff[s + 1] - boff[s];
    if (N <= 0 || m < 0 || F[s] <= 0) return FREDEC_EINVAL;
    if (m > MAXM) return FREDEC_ENOTSUP;
    if (N - 3 * m - 4 <= 0) return FREDEC_EDOF;
    const int KP = static_cast<int>(2 * m + 2);
    const int64_t tile = scan_tile(KP, precision);
    if (n_series == 1 && allow_split)
      L.nsplit = precision == FREDEC_FP64 ? scan_f64_nsplit(N, KP, F[s]) : scan_f16x3_nsplit(N, col_tiles(KP), F[s]);
    L.n_work += (F[s] + tile - 1) / tile * L.nsplit;
    L.Ntot += N;
    L.phi_total += N * KP;
    L.rec_total += N * rec_stride(KP);
    L.F_total += F[s];
    {
      SeriesIn d{};
      d.N = N;
      d.KP = KP;
      prep_assign(d, L.ptiles, L.ppart_total, L.pm_total);
    }
    if (precision == FREDEC_FP32) {
      L.g32_total += N * 16 * col_tiles(KP);
      L.aux_total += N * AUX_STRIDE;
      L.b16_total += b16_vectors(N, col_tiles(KP));
      L.pt16_total += pt16_float2(N);
      L.max_nt = std::max(L.max_nt, col_tiles(KP));
    }
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.off_sin = take(sizeof(SeriesIn) * n_series);
  L.off_hdr = take(sizeof(SeriesHdr) * n_series);
  L.off_work = take(sizeof(ScanWork) * L.n_work);
  L.off_tau = take(sizeof(double) * L.Ntot);
  L.off_xt = take(sizeof(double) * L.Ntot);
  L.off_wt = take(sizeof(double) * L.Ntot);
  L.off_rec = take(sizeof(double) * L.rec_total);
  L.off_phi = take(sizeof(double) * L.phi_total);
  L.off_g32 = take(sizeof(float) * L.g32_total);
  L.off_aux = take(sizeof(double) * L.aux_total);
  L.off_b16 = take(16 * L.b16_total);
  L.off_pt16 = take(8 * L.pt16_total);
  L.off_list = take(precision == FREDEC_FP32 ? sizeof(Rescore) * L.F_total : 0);
  L.off_count = take(sizeof(unsigned long long) * n_series);
  L.off_chunk = take(precision == FREDEC_FP32 ? sizeof(int64_t) * (2 * n_series + 3) : 0);
  L.off_ppart = take(sizeof(double) * L.ppart_total);
  L.off_pm = take(sizeof(double) * L.pm_total);
  if (L.nsplit > 1) {
    const int KP0 = static_cast<int>(2 * (boff[1] - boff[0]) + 2);
    L.off_part = take(precision == FREDEC_FP64 ? sizeof(double) * L.nsplit * (2 * KP0 + 3) * F[0]
                                               : static_cast<size_t>(f16x3_part_bytes(L.nsplit, col_tiles(KP0), F[0])));
  } else {
    L.off_part = take(0);
  }
  L.total = off;
  return FREDEC_OK;
}

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// A scan batch ready to launch: layout, per-series descriptors, the work list
// and its grouping by kernel instance.
struct ScanPlan : fredec_plan {
  ScanPlan() : fredec_plan(SCAN) {}
  ScanLayout L;
  int32_t n_series = 0;
  int32_t precision = FREDEC_FP64;
  int64_t base_off = 0;  // soff[0]: t, x, w are indexed from the caller's pointers
  int32_t kp_max = 2;    // largest KP of the series
  int64_t sin_F0 = 0;    // grid size of the first series (a split float64 scan has one series)
  std::vector<SeriesIn> sin;
  std::vector<ScanWork> work;
  // a single series: the work list is written on the device at launch
  // (per_chunk tiles of `work_tile` grid points for each sample chunk)
  // instead of built and uploaded by the host
  bool device_work = false;
  int64_t work_tile = 0, work_per_chunk = 0;
  enum Kind { F64 = 0, F32 = 2, F16X3 = 3 };
  struct Group {
    int kind;        // kernel family
    int key;         // KP (float64, float32 VALU) or column tiles NT (split float16)
    int ft;          // split float16: 16-frequency tiles per wave the work list was cut for
    int64_t begin, end;
    double work = 0.0;  // estimated cost: sum of N F (2 KP + 3) over its series
    int nsplit = 1;     // one series (float64 or split float16): sample chunks (work item pad = chunk)
  };
  std::vector<Group> groups;
};

// Work list of a single series: item k covers sample chunk k / per_chunk and
// the grid points from (k % per_chunk) * tile.
__global__ void fill_work_kernel(ScanWork* work, int64_t n, int64_t tile, int64_t per_chunk) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k < n) {
    ScanWork wk;
    wk.series = 0;
    wk.pad = static_cast<int32_t>(k / per_chunk);
    wk.j0 = (k % per_chunk) * tile;
    work[k] = wk;
  }
}

// Running offsets of the per-series arrays of a scan workspace.
struct SeriesOffsets {
  int64_t goff = 0, rec = 0, phi = 0, g32 = 0, aux = 0, b16 = 0, pt16 = 0, ptile = 0, ppart = 0, pm = 0;
};

// Descriptor of one series (samples [soff, soff + N) of the caller's arrays,
// base frequencies bf[0..m), grid of F points with step df) at the running
// offsets `o`, which it advances.
int series_desc(SeriesIn& d, int64_t soff, int64_t N, const double* bf, int32_t m, double df, int64_t F,
                int32_t precision, SeriesOffsets& o) {
  d.soff = soff;
  d.N = N;
  d.goff = o.goff;
  d.F = F;
  d.df = df;
  if (!std::isfinite(df) || df == 0.0) return FREDEC_EINVAL;
  d.rot_step = static_cast<double>(BLOCK) * df;
  d.rot_tile = 16.0 * df;
  d.m = m;
  d.KP = 2 * m + 2;
  prep_assign(d, o.ptile, o.ppart, o.pm);
  d.NT = col_tiles(d.KP);
  for (int k = 0; k < m; ++k) {
    d.base_f[k] = bf[k];
    if (!std::isfinite(d.base_f[k])) return FREDEC_EINVAL;
  }
  d.rec_off = o.rec;
  d.phi_off = o.phi;
  d.g32_off = o.g32;
  d.aux_off = o.aux;
  d.b16_off = o.b16;
  d.pt_off = o.pt16;
  o.goff += F;
  o.phi += N * d.KP;
  o.rec += N * rec_stride(d.KP);
  if (precision == FREDEC_FP32) {
    o.g32 += N * 16 * d.NT;
    o.aux += N * AUX_STRIDE;
    o.b16 += b16_vectors(N, d.NT);
    o.pt16 += pt16_float2(N);
  }
  return FREDEC_OK;
}

// Kernel family that scans a series with KP = 2m + 2 columns.  F_single: the
// grid of a scan of this one series (0 in a batch).  The automatic form gives
// a single series to the float32 VALU kernel only where its workgroups (256 R
// frequencies each) number at least four per CU; on smaller grids most CUs
// would idle, and the split-float16 kernel (64 FT frequencies per workgroup)
// is much faster (N = 10^4, F = 65536, m = 0: 0.49 against 5.0 ms, measured).
int scan_kind(const fredec_ctx* ctx, int32_t precision, int KP, int64_t F_single = 0) {
  const int form = ctx ? ctx->f32_form : FREDEC_F32_FORM_AUTO;
  const int auto_kp = ctx ? ctx->f32_auto_valu_max_kp : F32_AUTO_VALU_MAX_KP;
  if (precision == FREDEC_FP64) return ScanPlan::F64;
  if (form == FREDEC_F32_FORM_F16X3 || (form == FREDEC_F32_FORM_AUTO && KP > auto_kp)) return ScanPlan::F16X3;
  if (form == FREDEC_F32_FORM_AUTO && F_single > 0) {
    const int64_t tile = static_cast<int64_t>(BLOCK) * scan_f32_freqs_per_thread(KP);
    const int64_t n_cu = std::max(ctx ? ctx->n_cu : 0, 1);
    if ((F_single + tile - 1) / tile < 4 * n_cu) return ScanPlan::F16X3;
  }
  if (KP <= F32_VALU_MAX_KP) return ScanPlan::F32;
  return ScanPlan::F16X3;
}

// Operand sets the preparation writes for a series scanned by kernel family `kind`.
int kind_outputs(int kind) {
  return kind == ScanPlan::F32 ? PREP_G32 : kind == ScanPlan::F16X3 ? PREP_AUX | PREP_F16 : 0;
}

// Grid points per work-list tile of kernel family `kind` (ft: split-float16
// 16-frequency tiles per wave).
int64_t kind_tile(int kind, int KP, int ft, int32_t precision) {
  return kind == ScanPlan::F16X3 ? 64 * static_cast<int64_t>(ft)
         : kind == ScanPlan::F32 ? static_cast<int64_t>(BLOCK) * scan_f32_freqs_per_thread(KP)
                                 : scan_tile(KP, precision);
}

// Host part of a scan: checks, workspace layout, descriptors and work list.
int scan_build(const fredec_ctx* ctx, int32_t n_series, const int64_t* soff, const double* base_f,
               const int64_t* boff, const double* df, const int64_t* F, int32_t precision, void* ws, size_t ws_bytes,
               ScanPlan& P) {
  if (!df) return FREDEC_EINVAL;
  ScanLayout& L = P.L;
  int rc = scan_layout(n_series, soff, boff, F, precision, L);
  if (rc) return rc;
  if (boff[n_series] > boff[0] && !base_f) return FREDEC_EINVAL;
  if (!ws || ws_bytes < L.total) return FREDEC_ENOMEM;
  P.ws = ws;
  P.ws_bytes = ws_bytes;
  P.n_series = n_series;
  P.kp_max = 2;
  P.precision = precision;
  P.base_off = soff[0];
  P.sin_F0 = F[0];
  std::vector<SeriesIn>& sin = P.sin;
  sin.assign(n_series, SeriesIn{});
  std::memset(sin.data(), 0, sizeof(SeriesIn) * n_series);
  SeriesOffsets o;
  for (int32_t s = 0; s < n_series; ++s) {
    const int32_t m = static_cast<int32_t>(boff[s + 1] - boff[s]);
    if ((rc = series_desc(sin[s], soff[s], soff[s + 1] - soff[s], base_f + (boff[s] - boff[0]), m, df[s], F[s],
                          precision, o)))
      return rc;
    if (sin[s].KP > P.kp_max) P.kp_max = sin[s].KP;
  }
  // Work list: tiles grouped by kernel instance (KP for the float64 and the
  // float32 VALU kernels, column tiles NT for the split-float16 kernel), longest series first
  // inside a group.
  auto kind = [&](int32_t s) { return scan_kind(ctx, precision, sin[s].KP, n_series == 1 ? sin[s].F : 0); };
  auto key = [&](int32_t s) { return kind(s) == ScanPlan::F16X3 ? sin[s].NT : sin[s].KP; };
  std::vector<int32_t> order(n_series);
  for (int32_t s = 0; s < n_series; ++s) order[s] = s;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    if (kind(a) != kind(b)) return kind(a) < kind(b);
    if (key(a) != key(b)) return key(a) < key(b);
    return sin[a].N > sin[b].N;
  });
  for (int32_t s = 0; s < n_series; ++s) sin[s].outputs = kind_outputs(kind(s));
  P.work.clear();
  P.device_work = false;
  if (n_series > 1) P.work.reserve(L.n_work);
  P.groups.clear();
  for (int32_t s : order) {
    const int kd = kind(s);
    const int ft = kd == ScanPlan::F16X3 ? f16x3_ft_for(ctx, sin[s].NT) : 0;
    const int64_t tile = kind_tile(kd, sin[s].KP, ft, precision);
    if (P.groups.empty() || P.groups.back().kind != kd || P.groups.back().key != key(s))
      P.groups.push_back(ScanPlan::Group{kd, key(s), ft, static_cast<int64_t>(P.work.size()), 0});
    const int ns = kd == ScanPlan::F64 || kd == ScanPlan::F16X3 ? L.nsplit : 1;
    P.groups.back().nsplit = ns;
    if (n_series == 1) {
      P.device_work = true;
      P.work_tile = tile;
      P.work_per_chunk = (sin[s].F + tile - 1) / tile;
      P.groups.back().end = P.work_per_chunk * ns;
    } else {
      for (int c = 0; c < ns; ++c)
        for (int64_t j0 = 0; j0 < sin[s].F; j0 += tile) P.work.push_back(ScanWork{s, c, j0});
      P.groups.back().end = static_cast<int64_t>(P.work.size());
    }
    P.groups.back().work +=
        static_cast<double>(sin[s].N) * static_cast<double>(sin[s].F) * static_cast<double>(2 * sin[s].KP + 3);
  }
  return FREDEC_OK;
}

// Descriptors and work list into the workspace (asynchronous on `st`).
int scan_upload(fredec_ctx* ctx, hipStream_t st, const ScanPlan& P) {
  int rc;
  if ((rc = upload(ctx, st, at<SeriesIn>(P.ws, P.L.off_sin), P.sin.data(), sizeof(SeriesIn) * P.sin.size())))
    return rc;
  if (P.device_work) return FREDEC_OK;
  return upload(ctx, st, at<ScanWork>(P.ws, P.L.off_work), P.work.data(), sizeof(ScanWork) * P.work.size());
}

// Kernel launches of a scan whose descriptors are in the workspace: no host
// to device copies, allocations or synchronisation (capturable).
int scan_launch(fredec_ctx* ctx, hipStream_t st, const ScanPlan& P, const ScanPlan::Group* groups, size_t n_groups,
                const double* t, const double* x, const double* w, double* z_out, uint8_t* flags_out,
                double* l_base_out, int32_t* status_out, bool timed = true) {
  fredec_ctx* prof_ctx = timed ? ctx : nullptr;
  const ScanLayout& L = P.L;
  void* ws = P.ws;
  SeriesIn* d_sin = at<SeriesIn>(ws, L.off_sin);
  SeriesHdr* d_hdr = at<SeriesHdr>(ws, L.off_hdr);
  ScanWork* d_work = at<ScanWork>(ws, L.off_work);
  double* d_tau = at<double>(ws, L.off_tau);
  double* d_xt = at<double>(ws, L.off_xt);
  double* d_wt = at<double>(ws, L.off_wt);
  double* d_rec = at<double>(ws, L.off_rec);
  double* d_phi = at<double>(ws, L.off_phi);
  float* d_g32 = at<float>(ws, L.off_g32);
  double* d_aux = at<double>(ws, L.off_aux);
  void* d_b16 = at<char>(ws, L.off_b16);
  void* d_pt16 = at<char>(ws, L.off_pt16);
  Rescore* d_list = at<Rescore>(ws, L.off_list);
  unsigned long long* d_count = at<unsigned long long>(ws, L.off_count);
  int64_t* d_chunk = at<int64_t>(ws, L.off_chunk);
  const bool f32 = P.precision == FREDEC_FP32;
  // soff is absolute into t/x/w; the normalised copies use the same indexing
  // shifted by soff[0] (the batch is contiguous).
  const int64_t base_off = P.base_off;
  // per series, the prep kernel writes only what its scan kernel reads (SeriesIn::outputs)
  const int flags = PREP_BASE | PREP_REC64 | PREP_G32 | PREP_AUX | PREP_F16;
  if (f32 && launch_zero_u64(st, d_count, P.n_series) != hipSuccess) return FREDEC_EDEVICE;
  if (P.device_work && n_groups > 0) {
    const int64_t n = groups[0].end;
    hipLaunchKernelGGL(fill_work_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st, d_work, n,
                       P.work_tile, P.work_per_chunk);
    if (hipGetLastError() != hipSuccess) return FREDEC_EDEVICE;
  }
  {
    ProfScope prof(prof_ctx, st, FREDEC_PROF_PREP);
    if (launch_prep(st, P.n_series, P.kp_max, L.ptiles, d_sin, d_hdr, t, x, w, d_tau - base_off, d_xt - base_off,
                    d_wt - base_off, d_rec, d_phi, d_g32, d_aux, d_b16, d_pt16, at<double>(ws, L.off_ppart),
                    at<double>(ws, L.off_pm), flags) != hipSuccess)
      return FREDEC_EDEVICE;
  }
  {
    ProfScope prof(prof_ctx, st, FREDEC_PROF_SCAN);
    // The groups write disjoint outputs: with several of them, they run
    // concurrently on the caller's stream and the context's side streams
    // (each group, largest estimated work first, onto the least loaded
    // stream), joined back to the caller's stream with events before the
    // re-scoring (capturable fork/join), so that one group's last, partly
    // filled round overlaps the others.
    const int nst = static_cast<int>(std::min<size_t>(n_groups, 1 + fredec_ctx::NSIDE));
    int on_small[64];
    std::vector<int> on_big;
    int* on = n_groups <= 64 ? on_small : (on_big.assign(n_groups, 0), on_big.data());
    {
      double load[1 + fredec_ctx::NSIDE] = {};
      int order_small[64];
      std::vector<int> order_big;
      int* order = n_groups <= 64 ? order_small : (order_big.assign(n_groups, 0), order_big.data());
      for (size_t g = 0; g < n_groups; ++g) order[g] = static_cast<int>(g);
      std::sort(order, order + n_groups, [&](int a, int b) { return groups[a].work > groups[b].work; });
      for (size_t q = 0; q < n_groups; ++q) {
        int best = 0;
        for (int k = 1; k < nst; ++k)
          if (load[k] < load[best]) best = k;
        on[order[q]] = best;
        load[best] += groups[order[q]].work;
      }
    }
    if (nst > 1) {
      if (hipEventRecord(ctx->fork_ev, st) != hipSuccess) return FREDEC_EDEVICE;
      for (int k = 1; k < nst; ++k)
        if (hipStreamWaitEvent(ctx->side[k - 1], ctx->fork_ev, 0) != hipSuccess) return FREDEC_EDEVICE;
    }
    int rc = FREDEC_OK;
    for (size_t g = 0; g < n_groups && rc == FREDEC_OK; ++g) {
      const ScanPlan::Group& gr = groups[g];
      const hipStream_t gs = on[g] == 0 ? st : ctx->side[on[g] - 1];
      const int n = static_cast<int>(gr.end - gr.begin);
      hipError_t err;
      if (gr.kind == ScanPlan::F16X3)
        err = launch_scan_f16x3(gs, gr.key, gr.ft, n, d_work + gr.begin, d_sin, d_hdr, d_aux, d_b16, d_pt16, z_out,
                                flags_out, d_list, d_count, at<double>(ws, L.off_part), gr.nsplit,
                                P.n_series == 1 ? P.sin_F0 : 0);
      else if (gr.kind == ScanPlan::F32)
        err = launch_scan_f32(gs, gr.key, n, d_work + gr.begin, d_sin, d_hdr, d_rec, d_g32, z_out, flags_out, d_list,
                              d_count);
      else
        err = launch_scan_f64(gs, gr.key, n, d_work + gr.begin, d_sin, d_hdr, d_rec, z_out, flags_out,
                              at<double>(ws, L.off_part), gr.nsplit, P.n_series == 1 ? P.sin_F0 : 0);
      if (err != hipSuccess) rc = FREDEC_EDEVICE;
    }
    // join (also after a failed launch, so that no side stream stays forked)
    for (int k = 1; k < nst; ++k)
      if (hipEventRecord(ctx->join_ev[k - 1], ctx->side[k - 1]) != hipSuccess ||
          hipStreamWaitEvent(st, ctx->join_ev[k - 1], 0) != hipSuccess)
        rc = FREDEC_EDEVICE;
    if (rc) return rc;
  }
  if (f32) {
    ProfScope prof(prof_ctx, st, FREDEC_PROF_RESCORE);
    if (launch_rescore(st, L.max_nt, 4 * std::max(ctx->n_cu, 1), P.n_series, d_sin, d_hdr, d_rec, d_list, d_count,
                       d_chunk, z_out, flags_out) != hipSuccess)
      return FREDEC_EDEVICE;
  }
  if (launch_copy_stats(st, P.n_series, d_hdr, d_sin, l_base_out, status_out, nullptr) != hipSuccess)
    return FREDEC_EDEVICE;
  return FREDEC_OK;
}

// ------------------------------------------------------------ static scratch
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[MAX_DEVICES] = {};

// Device address of the calling device's copy of `scratch`; `dev` must be
// the current device.  Looked up once per device.
int static_scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return FREDEC_ENOTSUP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FREDEC_EDEVICE;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return FREDEC_OK;
}

// The descriptor of the single series of fredec_scan_static, written by the
// device (kernel argument) instead of a host-to-device copy.
__global__ void store_series_kernel(SeriesIn d, SeriesIn* dst) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *dst = d;
}

}  // namespace

extern "C" {

int fredec_version(void) { return 100; }

const char* fredec_strerror(int code) {
  switch (code) {
    case FREDEC_OK: return "ok";
    case FREDEC_EINVAL: return "invalid argument";
    case FREDEC_EDOF: return "too few samples for the model (N - 3n - 1 <= 0)";
    case FREDEC_EWEIGHT: return "non-positive weight or non-finite input";
    case FREDEC_EDEGEN: return "degenerate series (zero variance of x or t)";
    case FREDEC_ESINGULAR: return "singular base model";
    case FREDEC_ENOMEM: return "workspace too small or allocation failure";
    case FREDEC_EDEVICE: return "HIP runtime error";
    case FREDEC_ENOTSUP: return "size beyond a compiled limit";
    default: return "unknown error";
  }
}

int fredec_create(fredec_ctx** out, int device) {
  if (!out) return FREDEC_EINVAL;
  *out = nullptr;
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev) return FREDEC_EDEVICE;
  fredec_ctx* ctx = new (std::nothrow) fredec_ctx();
  if (!ctx) return FREDEC_ENOMEM;
  ctx->device = device;
  DeviceGuard g(device);
  hipDeviceProp_t prop;
  bool ok = hipGetDeviceProperties(&prop, device) == hipSuccess &&
            hipEventCreateWithFlags(&ctx->staging_done, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming) == hipSuccess;
  for (int i = 0; ok && i < fredec_ctx::NSIDE; ++i)
    ok = hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&ctx->join_ev[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    fredec_destroy(ctx);
    return FREDEC_EDEVICE;
  }
  ctx->n_cu = prop.multiProcessorCount;
  // the device address of this device's static scratch array (fredec_scan_static)
  if (static_scratch_address(device, &ctx->static_scratch) != FREDEC_OK) {
    fredec_destroy(ctx);
    return FREDEC_EDEVICE;
  }
  *out = ctx;
  return FREDEC_OK;
}

int fredec_set_tile(fredec_ctx* ctx, int32_t kernel, int32_t key, int32_t value) {
  if (!ctx) return FREDEC_EINVAL;
  if (kernel == FREDEC_TILE_SCAN_F16X3) {
    if (key < 1 || key > 4) return FREDEC_EINVAL;
    if (value != 0 && !f16x3_tile_supported(key, value)) return FREDEC_EINVAL;
    ctx->f16x3_ft[key] = value;
    return FREDEC_OK;
  }
  if (kernel == FREDEC_TILE_SCAN_F32_FORM) {
    if (key == 0) {
      if (value != FREDEC_F32_FORM_VALU && value != FREDEC_F32_FORM_F16X3 && value != FREDEC_F32_FORM_AUTO)
        return FREDEC_EINVAL;
      ctx->f32_form = value;
      return FREDEC_OK;
    }
    if (key == 1) {
      if (value < 0 || value > F32_VALU_MAX_KP) return FREDEC_EINVAL;
      ctx->f32_auto_valu_max_kp = value;
      return FREDEC_OK;
    }
    return FREDEC_EINVAL;
  }
  if (kernel == FREDEC_TILE_TUPLE_LANES) {
    if (key < 1 || key > 6) return FREDEC_EINVAL;
    if (value != 0 && value != 4 && value != 8 && value != 16 && value != 32 && value != 64) return FREDEC_EINVAL;
    ctx->tuple_lanes[key] = value;
    return FREDEC_OK;
  }
  return FREDEC_EINVAL;
}

int fredec_profile(fredec_ctx* ctx, int32_t enable) {
  if (!ctx) return FREDEC_EINVAL;
  ctx->profiling = enable != 0;
  ctx->prof_used = 0;
  return FREDEC_OK;
}

int fredec_profile_read_kinds(fredec_ctx* ctx, int32_t n_kinds, double* ms_out, int64_t* launches_out) {
  if (!ctx || n_kinds < 1 || !ms_out || !launches_out) return FREDEC_EINVAL;
  DeviceGuard g(ctx->device);
  for (int k = 0; k < n_kinds; ++k) {
    ms_out[k] = 0.0;
    launches_out[k] = 0;
  }
  int rc = FREDEC_OK;
  for (size_t k = 0; k < ctx->prof_used; ++k) {
    const auto& e = ctx->prof_events[k];
    float ms = 0.0f;
    if (hipEventSynchronize(e.end) != hipSuccess || hipEventElapsedTime(&ms, e.begin, e.end) != hipSuccess) {
      rc = FREDEC_EDEVICE;
      break;
    }
    if (e.kind >= 0 && e.kind < n_kinds) {
      ms_out[e.kind] += ms;
      launches_out[e.kind] += 1;
    }
  }
  ctx->prof_used = 0;
  return rc;
}

int fredec_profile_read(fredec_ctx* ctx, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches) return FREDEC_EINVAL;
  double ms[FREDEC_PROF_NKIND];
  int64_t n[FREDEC_PROF_NKIND];
  const int rc = fredec_profile_read_kinds(ctx, FREDEC_PROF_NKIND, ms, n);
  if (rc) return rc;
  *total_ms = ms[FREDEC_PROF_SCAN] + ms[FREDEC_PROF_GRAM];
  *launches = n[FREDEC_PROF_SCAN] + n[FREDEC_PROF_GRAM];
  return FREDEC_OK;
}

void fredec_destroy(fredec_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  for (auto& e : ctx->prof_events) {
    (void)hipEventDestroy(e.begin);
    (void)hipEventDestroy(e.end);
  }
  if (ctx->staging_pending) (void)hipEventSynchronize(ctx->staging_done);
  if (ctx->staging) (void)hipHostFree(ctx->staging);
  if (ctx->staging_done) (void)hipEventDestroy(ctx->staging_done);
  for (int i = 0; i < fredec_ctx::NSIDE; ++i) {
    if (ctx->side[i]) (void)hipStreamDestroy(ctx->side[i]);
    if (ctx->join_ev[i]) (void)hipEventDestroy(ctx->join_ev[i]);
  }
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  delete ctx;
}

// ------------------------------------------------------------ normalisation
int fredec_normalize_workspace(int32_t n_series, size_t* bytes) {
  if (!bytes || n_series <= 0) return FREDEC_EINVAL;
  *bytes = align_up(sizeof(SeriesIn) * n_series) + align_up(sizeof(SeriesHdr) * n_series);
  return FREDEC_OK;
}

int fredec_normalize(fredec_ctx* ctx, void* stream, int32_t n_series, const int64_t* soff, const double* t,
                     const double* x, const double* w, void* ws, size_t ws_bytes, double* tau_out, double* xt_out,
                     double* wt_out, double* stats_out, int32_t* status_out) {
  if (!soff || !t || !x || !w || !tau_out || !xt_out || !wt_out || n_series <= 0) return FREDEC_EINVAL;
  if (soff[0] < 0) return FREDEC_EINVAL;
  for (int32_t s = 0; s < n_series; ++s)
    if (soff[s + 1] - soff[s] <= 0) return FREDEC_EINVAL;
  size_t need = 0;
  fredec_normalize_workspace(n_series, &need);
  if (!ws || ws_bytes < need) return FREDEC_ENOMEM;
  if (!ctx) return FREDEC_EINVAL;
  std::vector<SeriesIn> sin(n_series);
  std::memset(sin.data(), 0, sizeof(SeriesIn) * n_series);
  for (int32_t s = 0; s < n_series; ++s) {
    sin[s].soff = soff[s];
    sin[s].N = soff[s + 1] - soff[s];
  }
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  SeriesIn* d_sin = at<SeriesIn>(ws, 0);
  SeriesHdr* d_hdr = at<SeriesHdr>(ws, align_up(sizeof(SeriesIn) * n_series));
  int rc = upload(ctx, st, d_sin, sin.data(), sizeof(SeriesIn) * n_series);
  if (rc) return rc;
  // the prep kernel writes the normalised series at the caller's offsets
  if (launch_prep(st, n_series, 0, 0, d_sin, d_hdr, t, x, w, tau_out, xt_out, wt_out, nullptr, nullptr, nullptr,
                  nullptr, nullptr, nullptr, nullptr, nullptr, 0) != hipSuccess)
    return FREDEC_EDEVICE;
  if (launch_copy_stats(st, n_series, d_hdr, d_sin, nullptr, status_out, stats_out) != hipSuccess)
    return FREDEC_EDEVICE;
  return FREDEC_OK;
}

// ------------------------------------------------------------ scan
int fredec_scan_workspace(int32_t n_series, const int64_t* soff, const int64_t* boff, const int64_t* F,
                          int32_t precision, size_t* bytes) {
  if (!bytes) return FREDEC_EINVAL;
  ScanLayout L;
  int rc = scan_layout(n_series, soff, boff, F, precision, L);
  if (rc) return rc;
  *bytes = L.total;
  return FREDEC_OK;
}

int fredec_scan(fredec_ctx* ctx, void* stream, int32_t n_series, const double* t, const double* x, const double* w,
                const int64_t* soff, const double* base_f, const int64_t* boff, const double* df, const int64_t* F,
                int32_t precision, void* ws, size_t ws_bytes, double* z_out, uint8_t* flags_out, double* l_base_out,
                int32_t* status_out) {
  // host-side checks first (they need no device), the context last
  if (!t || !x || !w || !z_out) return FREDEC_EINVAL;
  ScanPlan P;
  int rc = scan_build(ctx, n_series, soff, base_f, boff, df, F, precision, ws, ws_bytes, P);
  if (rc) return rc;
  if (!ctx) return FREDEC_EINVAL;
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if ((rc = scan_upload(ctx, st, P))) return rc;
  return scan_launch(ctx, st, P, P.groups.data(), P.groups.size(), t, x, w, z_out, flags_out, l_base_out,
                     status_out);
}

int fredec_scan_plan(fredec_ctx* ctx, void* stream, int32_t n_series, const int64_t* soff, const double* base_f,
                     const int64_t* boff, const double* df, const int64_t* F, int32_t precision, void* ws,
                     size_t ws_bytes, fredec_plan** plan_out) {
  if (!plan_out) return FREDEC_EINVAL;
  *plan_out = nullptr;
  ScanPlan* P = new (std::nothrow) ScanPlan();
  if (!P) return FREDEC_ENOMEM;
  int rc = scan_build(ctx, n_series, soff, base_f, boff, df, F, precision, ws, ws_bytes, *P);
  if (!rc && !ctx) rc = FREDEC_EINVAL;
  if (!rc) {
    DeviceGuard g(ctx->device);
    P->device = ctx->device;
    rc = scan_upload(ctx, static_cast<hipStream_t>(stream), *P);
    if (!rc) rc = upload_wait(ctx);
    // the descriptors are on the device now; the host copies are not needed
    std::vector<SeriesIn>().swap(P->sin);
    std::vector<ScanWork>().swap(P->work);
  }
  if (rc) {
    delete P;
    return rc;
  }
  *plan_out = P;
  return FREDEC_OK;
}

int fredec_plan_scan(fredec_ctx* ctx, fredec_plan* plan, void* stream, const double* t, const double* x,
                     const double* w, double* z_out, uint8_t* flags_out, double* l_base_out, int32_t* status_out) {
  if (!ctx || !plan || plan->kind != fredec_plan::SCAN || !t || !x || !w || !z_out) return FREDEC_EINVAL;
  if (plan->device != ctx->device) return FREDEC_EINVAL;
  DeviceGuard g(ctx->device);
  const ScanPlan& P = *static_cast<ScanPlan*>(plan);
  return scan_launch(ctx, static_cast<hipStream_t>(stream), P, P.groups.data(), P.groups.size(), t, x, w, z_out,
                     flags_out, l_base_out, status_out);
}

void fredec_plan_destroy(fredec_plan* plan) { delete plan; }

// ------------------------------------------------------------ allocation-free scan
int fredec_scan_static(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                       const double* base_f, int32_t m, double df, int64_t F, int32_t precision, double* z_out,
                       uint8_t* flags_out, double* l_base_out, int32_t* status_out) {
  if (!t || !x || !w || !z_out || N <= 0 || m < 0 || F <= 0) return FREDEC_EINVAL;
  if (m > 0 && !base_f) return FREDEC_EINVAL;
  const int64_t soff[2] = {0, N}, boff[2] = {0, m}, Fs[1] = {F};
  ScanPlan P;  // no host allocation: its vectors stay empty
  int rc = scan_layout(1, soff, boff, Fs, precision, P.L, /*allow_split=*/false);
  if (rc) return rc;
  if (P.L.total > static_cast<size_t>(FREDEC_STATIC_SCRATCH_BYTES)) return FREDEC_ENOTSUP;
  SeriesIn d;
  std::memset(&d, 0, sizeof(d));
  SeriesOffsets o;
  if ((rc = series_desc(d, 0, N, base_f, m, df, F, precision, o))) return rc;
  if (!ctx || !ctx->static_scratch) return FREDEC_EINVAL;
  const int kd = scan_kind(ctx, precision, d.KP, F);
  d.outputs = kind_outputs(kd);
  const int ft = kd == ScanPlan::F16X3 ? f16x3_ft_for(ctx, d.NT) : 0;
  const int64_t tile = kind_tile(kd, d.KP, ft, precision);
  const int64_t n_work = (F + tile - 1) / tile;  // <= P.L.n_work (laid out for the smallest tile)
  P.ws = ctx->static_scratch;
  P.ws_bytes = FREDEC_STATIC_SCRATCH_BYTES;
  P.n_series = 1;
  P.precision = precision;
  P.kp_max = d.KP;
  P.base_off = 0;
  const ScanPlan::Group gr{kd, kd == ScanPlan::F16X3 ? d.NT : d.KP, ft, 0, n_work};
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(store_series_kernel, dim3(1), dim3(64), 0, st, d, at<SeriesIn>(P.ws, P.L.off_sin));
  if (hipGetLastError() != hipSuccess) return FREDEC_EDEVICE;
  hipLaunchKernelGGL(fill_work_kernel, dim3(static_cast<unsigned>((n_work + 255) / 256)), dim3(256), 0, st,
                     at<ScanWork>(P.ws, P.L.off_work), n_work, tile, n_work);
  if (hipGetLastError() != hipSuccess) return FREDEC_EDEVICE;
  return scan_launch(ctx, st, P, &gr, 1, t, x, w, z_out, flags_out, l_base_out, status_out, /*timed=*/false);
}

int fredec_scan_at_workspace(int64_t N, int32_t m, size_t* bytes) {
  if (!bytes || N <= 0 || m < 0) return FREDEC_EINVAL;
  if (m > MAXM) return FREDEC_ENOTSUP;
  const int KP = 2 * m + 2;
  SeriesIn d{};
  d.N = N;
  d.KP = KP;
  int64_t ptile = 0, ppart = 0, pmo = 0;
  prep_assign(d, ptile, ppart, pmo);
  *bytes = align_up(sizeof(SeriesIn)) + align_up(sizeof(SeriesHdr)) + 3 * align_up(sizeof(double) * N) +
           align_up(sizeof(double) * N * rec_stride(KP)) + align_up(sizeof(double) * N * KP) +
           align_up(sizeof(double) * ppart) + align_up(sizeof(double) * pmo);
  return FREDEC_OK;
}

int fredec_scan_at(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                   const double* base_f, int32_t m, double df, const int64_t* idx, int64_t n_idx, void* ws,
                   size_t ws_bytes, double* z_out, uint8_t* flags_out) {
  if (!t || !x || !w || !z_out || N <= 0 || m < 0 || n_idx < 0 || n_idx > 0x7fffffff) return FREDEC_EINVAL;
  if (n_idx > 0 && !idx) return FREDEC_EINVAL;
  if (m > 0 && !base_f) return FREDEC_EINVAL;
  if (!std::isfinite(df) || df == 0.0) return FREDEC_EINVAL;
  if (m > MAXM) return FREDEC_ENOTSUP;
  if (N - 3 * static_cast<int64_t>(m) - 4 <= 0) return FREDEC_EDOF;
  size_t need = 0;
  fredec_scan_at_workspace(N, m, &need);
  if (!ws || ws_bytes < need) return FREDEC_ENOMEM;
  SeriesIn si;
  std::memset(&si, 0, sizeof(si));
  si.N = N;
  si.F = 1;
  si.df = df;
  si.rot_step = static_cast<double>(BLOCK) * df;
  si.rot_tile = 16.0 * df;
  si.m = m;
  si.KP = 2 * m + 2;
  si.NT = col_tiles(si.KP);
  int64_t ptile = 0, ppart = 0, pmo = 0;
  prep_assign(si, ptile, ppart, pmo);
  for (int k = 0; k < m; ++k) {
    if (!std::isfinite(base_f[k])) return FREDEC_EINVAL;
    si.base_f[k] = base_f[k];
  }
  if (!ctx) return FREDEC_EINVAL;
  if (n_idx == 0) return FREDEC_OK;
  size_t off = 0;
  SeriesIn* d_sin = at<SeriesIn>(ws, off);
  off += align_up(sizeof(SeriesIn));
  SeriesHdr* d_hdr = at<SeriesHdr>(ws, off);
  off += align_up(sizeof(SeriesHdr));
  double* d_tau = at<double>(ws, off);
  off += align_up(sizeof(double) * N);
  double* d_xt = at<double>(ws, off);
  off += align_up(sizeof(double) * N);
  double* d_wt = at<double>(ws, off);
  off += align_up(sizeof(double) * N);
  double* d_rec = at<double>(ws, off);
  off += align_up(sizeof(double) * N * rec_stride(si.KP));
  double* d_phi = at<double>(ws, off);
  off += align_up(sizeof(double) * N * si.KP);
  double* d_ppart = at<double>(ws, off);
  off += align_up(sizeof(double) * ppart);
  double* d_pm = at<double>(ws, off);
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  int rc = upload(ctx, st, d_sin, &si, sizeof(si));
  if (rc) return rc;
  if (launch_prep(st, 1, si.KP, ptile, d_sin, d_hdr, t, x, w, d_tau, d_xt, d_wt, d_rec, d_phi, nullptr, nullptr,
                  nullptr, nullptr, d_ppart, d_pm, PREP_BASE | PREP_REC64) != hipSuccess)
    return FREDEC_EDEVICE;
  if (launch_scan_at_f64(st, si.KP, d_sin, d_hdr, d_rec, idx, n_idx, z_out, flags_out) != hipSuccess)
    return FREDEC_EDEVICE;
  return FREDEC_OK;
}

}  // extern "C"
