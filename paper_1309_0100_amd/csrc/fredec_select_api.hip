// C ABI of the selection steps: FAP thresholds (eq. zFAP), periodogram peaks,
// the Phase 1 preliminary scan (Sect. 4.2) and the Phase 3 backward cascade
// (Sect. 4.4).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fredec_api_internal.h"
#include "fredec_select_internal.h"

using namespace fredec;

namespace {

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

// log of the bound A W^d e^{-z} z^{3d/2 - 1} of eq. zFAP
double log_fap(double z, int d, double W, double A) {
  return std::log(A) + d * std::log(W) - z + (1.5 * d - 1.0) * std::log(z);
}

// z with log_fap(z) = log(fap) on the decreasing branch z > 3d/2 - 1, by bisection
double zcrit_one(int d, double W, double fap, double A) {
  double lo = std::max(1.5 * d - 1.0, 1e-300);
  const double target = std::log(fap);
  if (log_fap(lo, d, W, A) <= target) return lo;
  double hi = std::max(2.0 * lo, 1.0);
  while (log_fap(hi, d, W, A) > target) hi *= 2.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (log_fap(mid, d, W, A) > target)
      lo = mid;
    else
      hi = mid;
  }
  return hi;
}

int sync_read(hipStream_t st, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return FREDEC_OK;
  if (hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st) != hipSuccess) return FREDEC_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return FREDEC_EDEVICE;
  return FREDEC_OK;
}

__global__ void zero_count_kernel(unsigned long long* c) { *c = 0ull; }

// Device buffers of the float64 hill climb: grid indices, their z and flags
// (3 per peak) and the fredec_scan_at workspace.
struct ClimbBuffers {
  int64_t* idx;
  double* z;
  uint8_t* fl;
  void* at_ws;
  size_t at_bytes;
};

// Float64 hill climb from each reduced-precision peak in `pk` to the float64
// local maximum of the scan with base model `base` (fredec_scan_at on the
// point and its neighbours until neither neighbour is higher).  Replaces `pk`
// by the float64 maxima reached that are interior, carry no flag other than
// FREDEC_FLAG_RESCORED and have z > zmin, sorted by index without repeats.
// The buffers hold 3 entries per peak.
int climb_f64(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
              const std::vector<double>& base, double df, int64_t F, const ClimbBuffers& cb, double zmin,
              std::vector<Peak>& pk) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t np = static_cast<int64_t>(pk.size());
  int rc;
  std::vector<int64_t> cur(np);
  for (int64_t k = 0; k < np; ++k) cur[k] = pk[k].j;
  std::vector<char> active(np, 1);
  std::vector<double> zc(np, 0.0);
  std::vector<uint8_t> fc(np, 0);
  for (int iter = 0; iter < 64; ++iter) {
    std::vector<int64_t> idx;
    std::vector<int64_t> who;
    for (int64_t k = 0; k < np; ++k)
      if (active[k]) {
        for (int o = -1; o <= 1; ++o) idx.push_back(std::min<int64_t>(std::max<int64_t>(cur[k] + o, 0), F - 1));
        who.push_back(k);
      }
    if (who.empty()) break;
    if ((rc = upload(ctx, st, cb.idx, idx.data(), sizeof(int64_t) * idx.size()))) return rc;
    if ((rc = fredec_scan_at(ctx, stream, t, x, w, N, base.empty() ? nullptr : base.data(),
                             static_cast<int32_t>(base.size()), df, cb.idx, static_cast<int64_t>(idx.size()),
                             cb.at_ws, cb.at_bytes, cb.z, cb.fl)))
      return rc;
    std::vector<double> zv(idx.size());
    std::vector<uint8_t> fv(idx.size());
    if ((rc = sync_read(st, zv.data(), cb.z, sizeof(double) * zv.size()))) return rc;
    if ((rc = sync_read(st, fv.data(), cb.fl, fv.size()))) return rc;
    for (size_t q = 0; q < who.size(); ++q) {
      const int64_t k = who[q];
      const double zl = zv[3 * q], zm = zv[3 * q + 1], zr = zv[3 * q + 2];
      const int64_t j = cur[k];
      if (j <= 0 || j >= F - 1) {
        active[k] = 0;
        zc[k] = -1.0;  // not an interior point
        continue;
      }
      if (zl >= zm) {
        cur[k] = j - 1;
      } else if (zr > zm) {
        cur[k] = j + 1;
      } else {
        active[k] = 0;
        zc[k] = zm;
        fc[k] = fv[3 * q + 1];
      }
    }
  }
  std::vector<Peak> out;
  for (int64_t k = 0; k < np; ++k)
    if (!active[k] && zc[k] > zmin && (fc[k] & ~FREDEC_FLAG_RESCORED) == 0) out.push_back(Peak{cur[k], zc[k]});
  std::sort(out.begin(), out.end(), [](const Peak& a, const Peak& b) { return a.j < b.j; });
  out.erase(std::unique(out.begin(), out.end(), [](const Peak& a, const Peak& b) { return a.j == b.j; }), out.end());
  pk.swap(out);
  return FREDEC_OK;
}

// Largest scan workspace over the base models m = 0 .. mmax of one series
// (a single float64 scan of few frequency tiles holds partial sums of its
// sample chunks, so a smaller base can need more); bases that leave no
// degrees of freedom are skipped.
int scan_ws_upto(int64_t N, int64_t F, int mmax, int32_t precision, size_t* bytes) {
  *bytes = 0;
  const int64_t soff[2] = {0, N};
  const int64_t Fs[1] = {F};
  for (int m = 0; m <= mmax; ++m) {
    const int64_t boff[2] = {0, m};
    size_t b = 0;
    const int rc = fredec_scan_workspace(1, soff, boff, Fs, precision, &b);
    if (rc == FREDEC_EDOF) break;
    if (rc) return rc;
    *bytes = std::max(*bytes, b);
  }
  return *bytes ? FREDEC_OK : FREDEC_EDOF;
}

struct Phase1Layout {
  size_t scan_ws = 0, at_ws = 0;
  size_t off_scan = 0, off_at = 0, off_z = 0, off_fl = 0, off_lb = 0, off_st = 0, off_peaks = 0, off_count = 0,
         off_idx = 0, off_zat = 0, off_flat = 0, total = 0;
  int64_t peak_cap = 0;
};

int phase1_layout(int64_t N, int64_t F, int32_t max_scans, int32_t precision, Phase1Layout& L) {
  if (N <= 0 || F < 3 || max_scans < 1) return FREDEC_EINVAL;
  const int mmax = std::min<int>(max_scans - 1, FREDEC_MAX_BASE);
  if (precision != FREDEC_FP64 && precision != FREDEC_FP32) return FREDEC_EINVAL;
  int rc = scan_ws_upto(N, F, mmax, precision, &L.scan_ws);
  if (rc) return rc;
  if ((rc = fredec_scan_at_workspace(N, mmax, &L.at_ws))) return rc;
  // interior maxima with z_{j-1} < z_j cannot be adjacent: at most
  // ceil((F - 2) / 2) of them, so every peak above the threshold is kept
  L.peak_cap = std::max<int64_t>((F - 1) / 2, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.off_scan = take(L.scan_ws);
  L.off_at = take(L.at_ws);
  L.off_z = take(sizeof(double) * F);
  L.off_fl = take(F);
  L.off_lb = take(sizeof(double));
  L.off_st = take(sizeof(int32_t));
  L.off_peaks = take(sizeof(Peak) * L.peak_cap);
  L.off_count = take(sizeof(unsigned long long));
  L.off_idx = take(sizeof(int64_t) * 3 * L.peak_cap);
  L.off_zat = take(sizeof(double) * 3 * L.peak_cap);
  L.off_flat = take(3 * L.peak_cap);
  L.total = off;
  return FREDEC_OK;
}


struct FapLayout {
  size_t scan_ws = 0, at_ws = 0;
  size_t off_scan = 0, off_at = 0, off_z = 0, off_fl = 0, off_lb = 0, off_st = 0, off_part = 0, off_best = 0,
         off_peaks = 0, off_count = 0, off_idx = 0, off_zat = 0, off_flat = 0, total = 0;
  int64_t peak_cap = 0;
};

int fap_layout(int64_t N, int64_t F, int32_t m_max, int32_t precision, FapLayout& L) {
  if (N <= 0 || F < 3 || m_max < 0) return FREDEC_EINVAL;
  if (m_max > FREDEC_MAX_BASE) return FREDEC_ENOTSUP;
  if (N - 3 * (static_cast<int64_t>(m_max) + 1) - 1 <= 0) return FREDEC_EDOF;
  int rc = scan_ws_upto(N, F, m_max, precision, &L.scan_ws);
  if (rc) return rc;
  if ((rc = fredec_scan_at_workspace(N, m_max, &L.at_ws))) return rc;
  L.peak_cap = std::max<int64_t>((F - 1) / 2, 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  L.off_scan = take(L.scan_ws);
  L.off_at = take(L.at_ws);
  L.off_z = take(sizeof(double) * F);
  L.off_fl = take(F);
  L.off_lb = take(sizeof(double));
  L.off_st = take(sizeof(int32_t));
  L.off_part = take(sizeof(Peak) * peak_max_parts(F));
  L.off_best = take(sizeof(Peak));
  L.off_peaks = take(precision == FREDEC_FP32 ? sizeof(Peak) * L.peak_cap : 0);
  L.off_count = take(sizeof(unsigned long long));
  L.off_idx = take(precision == FREDEC_FP32 ? sizeof(int64_t) * 3 * L.peak_cap : 0);
  L.off_zat = take(precision == FREDEC_FP32 ? sizeof(double) * 3 * L.peak_cap : 0);
  L.off_flat = take(precision == FREDEC_FP32 ? 3 * L.peak_cap : 0);
  L.total = off;
  return FREDEC_OK;
}

// Largest base model among the solutions, or a negative code.
int fap_check(const double* sol_f, const int64_t* sol_off, int32_t n_sol, int32_t* m_max) {
  if (!sol_off || n_sol < 1 || sol_off[0] != 0) return FREDEC_EINVAL;
  int64_t mm = 0;
  for (int32_t k = 0; k < n_sol; ++k) {
    const int64_t m = sol_off[k + 1] - sol_off[k];
    if (m < 0) return FREDEC_EINVAL;
    if (m > FREDEC_MAX_BASE) return FREDEC_ENOTSUP;
    mm = std::max(mm, m);
  }
  if (sol_off[n_sol] > 0 && !sol_f) return FREDEC_EINVAL;
  for (int64_t q = 0; q < sol_off[n_sol]; ++q)
    if (!std::isfinite(sol_f[q])) return FREDEC_EINVAL;
  *m_max = static_cast<int32_t>(mm);
  return FREDEC_OK;
}

}  // namespace

extern "C" {

int fredec_zcrit(double W, int32_t n, double fap, const double* A, double* zc) {
  if (!zc || n < 1 || !(W > 0.0) || !(fap > 0.0) || !(fap < 1.0) || !std::isfinite(W)) return FREDEC_EINVAL;
  zc[0] = 0.0;
  for (int d = 1; d <= n; ++d) {
    const double a = A ? A[d] : 1.0;
    if (!(a > 0.0)) return FREDEC_EINVAL;
    zc[d] = zcrit_one(d, W, fap, a);
  }
  return FREDEC_OK;
}

int fredec_peaks_workspace(int64_t cap, size_t* bytes) {
  if (!bytes || cap < 1) return FREDEC_EINVAL;
  *bytes = align_up(sizeof(unsigned long long)) + align_up(sizeof(Peak) * cap);
  return FREDEC_OK;
}

int fredec_peaks(fredec_ctx* ctx, void* stream, const double* z, const uint8_t* flags, int64_t F, double zmin,
                 void* ws, size_t ws_bytes, int64_t cap, int64_t* idx_host, double* z_host, int64_t* n_found) {
  if (!z || F < 1 || cap < 1 || !idx_host || !z_host || !n_found) return FREDEC_EINVAL;
  size_t need = 0;
  fredec_peaks_workspace(cap, &need);
  if (!ws || ws_bytes < need) return FREDEC_ENOMEM;
  if (!ctx) return FREDEC_EINVAL;
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  unsigned long long* d_count = at<unsigned long long>(ws, 0);
  Peak* d_peaks = at<Peak>(ws, align_up(sizeof(unsigned long long)));
  zero_count_kernel<<<1, 1, 0, st>>>(d_count);
  if (hipGetLastError() != hipSuccess) return FREDEC_EDEVICE;
  if (launch_peaks(st, z, flags, F, zmin, d_peaks, d_count, cap) != hipSuccess) return FREDEC_EDEVICE;
  unsigned long long cnt = 0;
  int rc = sync_read(st, &cnt, d_count, sizeof(cnt));
  if (rc) return rc;
  const int64_t n = std::min<int64_t>(static_cast<int64_t>(cnt), cap);
  std::vector<Peak> pk(n);
  if ((rc = sync_read(st, pk.data(), d_peaks, sizeof(Peak) * n))) return rc;
  std::sort(pk.begin(), pk.end(), [](const Peak& a, const Peak& b) { return a.j < b.j; });
  for (int64_t k = 0; k < n; ++k) {
    idx_host[k] = pk[k].j;
    z_host[k] = pk[k].z;
  }
  *n_found = static_cast<int64_t>(cnt);
  return FREDEC_OK;
}

int fredec_cascade_workspace(int32_t n, size_t* bytes) {
  if (!bytes || n < 1) return FREDEC_EINVAL;
  if (n > FREDEC_MAX_POOL) return FREDEC_ENOTSUP;
  *bytes = align_up(size_t(1) << n);
  return FREDEC_OK;
}

int fredec_cascade(fredec_ctx* ctx, void* stream, const double* ltab, int32_t n, int64_t N, const double* zcrit,
                   void* ws, size_t ws_bytes, uint8_t* survive_out, uint8_t* maximal_out, double* G_out) {
  if (!ltab || !zcrit || !survive_out || !maximal_out || N <= 0 || n < 1) return FREDEC_EINVAL;
  if (n > FREDEC_MAX_POOL) return FREDEC_ENOTSUP;
  size_t need = 0;
  fredec_cascade_workspace(n, &need);
  if (!ws || ws_bytes < need) return FREDEC_ENOMEM;
  CascadeParams p;
  std::memset(&p, 0, sizeof(p));
  for (int d = 0; d <= n; ++d) {
    if (!std::isfinite(zcrit[d])) return FREDEC_EINVAL;
    p.zc[d] = zcrit[d];
  }
  if (!ctx) return FREDEC_EINVAL;
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (launch_cascade(st, ltab, n, N, p, survive_out, static_cast<uint8_t*>(ws), maximal_out, G_out) != hipSuccess)
    return FREDEC_EDEVICE;
  return FREDEC_OK;
}

int fredec_phase1_workspace(int64_t N, int64_t F, int32_t max_scans, int32_t precision, size_t* bytes) {
  if (!bytes) return FREDEC_EINVAL;
  Phase1Layout L;
  int rc = phase1_layout(N, F, max_scans, precision, L);
  if (rc) return rc;
  *bytes = L.total;
  return FREDEC_OK;
}

int fredec_phase1(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                  double df, int64_t F, double fap0, double fap1, double A1, int32_t pool_cap, int32_t max_scans,
                  int32_t precision, void* ws, size_t ws_bytes, double* pool_out, double* pool_z_out,
                  int32_t* n_pool, double* base_out, int32_t* n_base, int32_t* n_scans, int32_t* truncated,
                  double* W_out) {
  if (!t || !x || !w || N <= 0 || F < 3 || !pool_out || !pool_z_out || !n_pool || !base_out || !n_base ||
      !n_scans || !truncated || !W_out)
    return FREDEC_EINVAL;
  if (!(fap1 >= fap0 && fap0 > 0.0 && fap1 < 1.0) || !(A1 > 0.0) || !std::isfinite(df) || df == 0.0 ||
      max_scans < 1)
    return FREDEC_EINVAL;
  if (precision != FREDEC_FP64 && precision != FREDEC_FP32) return FREDEC_EINVAL;
  Phase1Layout L;
  int rc = phase1_layout(N, F, max_scans, precision, L);
  if (rc) return rc;
  if (!ws || ws_bytes < L.total) return FREDEC_ENOMEM;
  if (!ctx) return FREDEC_EINVAL;
  const int32_t cap = pool_cap > 0 ? pool_cap : static_cast<int32_t>(N / 10);
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* d_z = at<double>(ws, L.off_z);
  uint8_t* d_fl = at<uint8_t>(ws, L.off_fl);
  double* d_lb = at<double>(ws, L.off_lb);
  int32_t* d_st = at<int32_t>(ws, L.off_st);
  Peak* d_pk = at<Peak>(ws, L.off_peaks);
  unsigned long long* d_cnt = at<unsigned long long>(ws, L.off_count);
  int64_t* d_idx = at<int64_t>(ws, L.off_idx);
  double* d_zat = at<double>(ws, L.off_zat);
  uint8_t* d_flat = at<uint8_t>(ws, L.off_flat);

  std::vector<double> base, pf, pz;
  int scans = 0;
  double T = 0.0, W = 0.0, zc1 = 0.0, zc0 = 0.0;
  const int64_t soff[2] = {0, N};
  while (scans < max_scans && N - 3 * (static_cast<int64_t>(base.size()) + 1) - 1 > 0 &&
         static_cast<int>(base.size()) <= FREDEC_MAX_BASE) {
    const int64_t boff[2] = {0, static_cast<int64_t>(base.size())};
    if ((rc = fredec_scan(ctx, stream, 1, t, x, w, soff, base.empty() ? nullptr : base.data(), boff, &df, &F,
                          precision, at<void>(ws, L.off_scan), L.scan_ws, d_z, d_fl, d_lb, d_st)))
      return rc;
    ++scans;
    if (scans == 1) {
      // T_eff and status of the series from the preparation kernel
      int32_t status = 0;
      if ((rc = sync_read(st, &status, d_st, sizeof(status)))) return rc;
      if (status) return status;
      double stats[6];
      // the scan workspace begins with SeriesIn[1] then SeriesHdr[1]
      const SeriesHdr* hdr = at<const SeriesHdr>(ws, L.off_scan + align_up(sizeof(SeriesIn)));
      if ((rc = sync_read(st, stats, hdr->stats, sizeof(stats)))) return rc;
      T = stats[4];
      W = static_cast<double>(F) * df * T;
      zc1 = zcrit_one(1, std::fabs(W), fap1, A1);
      zc0 = zcrit_one(1, std::fabs(W), fap0, A1);
      *W_out = std::fabs(W);
    }
    // peaks above the candidate threshold (a little below it for float32
    // sums; the decisions below use float64 values)
    const double zmin = precision == FREDEC_FP32 ? zc1 * (1.0 - 1e-4) : zc1;
    zero_count_kernel<<<1, 1, 0, st>>>(d_cnt);
    if (hipGetLastError() != hipSuccess) return FREDEC_EDEVICE;
    if (launch_peaks(st, d_z, d_fl, F, zmin, d_pk, d_cnt, L.peak_cap) != hipSuccess) return FREDEC_EDEVICE;
    unsigned long long cnt = 0;
    if ((rc = sync_read(st, &cnt, d_cnt, sizeof(cnt)))) return rc;
    if (static_cast<int64_t>(cnt) > L.peak_cap) return FREDEC_EDEVICE;  // cannot happen (see phase1_layout)
    const int64_t np = static_cast<int64_t>(cnt);
    std::vector<Peak> pk(np);
    if ((rc = sync_read(st, pk.data(), d_pk, sizeof(Peak) * np))) return rc;
    if (precision == FREDEC_FP32 && np > 0) {
      // Only peaks at or above half the largest one enter the decisions
      // below.  The float32 values are within 1e-6 (relative) of float64, so
      // a peak more than 1e-3 below half the largest float32 peak cannot
      // reach half the largest float64 peak after re-scoring: it is dropped
      // before the float64 hill climb (thousands of peaks per scan otherwise).
      double zmax32 = 0.0;
      for (const Peak& p : pk) zmax32 = std::max(zmax32, p.z);
      const double zkeep = 0.5 * zmax32 * (1.0 - 1e-3);
      pk.erase(std::remove_if(pk.begin(), pk.end(), [&](const Peak& p) { return p.z < zkeep; }), pk.end());
      ClimbBuffers cb{d_idx, d_zat, d_flat, at<void>(ws, L.off_at), L.at_ws};
      if ((rc = climb_f64(ctx, stream, t, x, w, N, base, df, F, cb, zc1, pk))) return rc;
    }
    if (pk.empty()) break;
    // descending z, ties -> lower index
    std::sort(pk.begin(), pk.end(), [](const Peak& a, const Peak& b) { return a.z != b.z ? a.z > b.z : a.j < b.j; });
    const double zmax = pk[0].z;
    for (const Peak& p : pk) {
      if (!(p.z > zc1 && p.z >= 0.5 * zmax)) continue;
      const double fj = static_cast<double>(p.j + 1) * df;
      bool merged = false;
      for (double q : pf) merged |= std::fabs(fj - q) * T < 0.5;
      if (merged) continue;
      pf.push_back(fj);
      pz.push_back(p.z);
    }
    if (zmax > zc0)
      base.push_back(static_cast<double>(pk[0].j + 1) * df);
    else
      break;
  }
  // cap: keep the smallest FAP (largest z), ties -> lower frequency
  std::vector<int> ord(pf.size());
  for (size_t k = 0; k < pf.size(); ++k) ord[k] = static_cast<int>(k);
  std::sort(ord.begin(), ord.end(), [&](int a, int b) { return pz[a] != pz[b] ? pz[a] > pz[b] : pf[a] < pf[b]; });
  const int keep = std::min<int>(static_cast<int>(pf.size()), cap);
  std::vector<std::pair<double, double>> sel;
  for (int k = 0; k < keep; ++k) sel.push_back({pf[ord[k]], pz[ord[k]]});
  std::stable_sort(sel.begin(), sel.end(), [](const std::pair<double, double>& a, const std::pair<double, double>& b) {
    return a.first < b.first;
  });
  for (int k = 0; k < keep; ++k) {
    pool_out[k] = sel[k].first;
    pool_z_out[k] = sel[k].second;
  }
  *n_pool = keep;
  *truncated = static_cast<int32_t>(pf.size()) - keep;
  for (size_t k = 0; k < base.size(); ++k) base_out[k] = base[k];
  *n_base = static_cast<int32_t>(base.size());
  *n_scans = scans;
  return FREDEC_OK;
}

// ------------------------------------------------------------ residual FAP
int fredec_residual_fap_workspace(int64_t N, int64_t F, int32_t m_max, int32_t precision, size_t* bytes) {
  if (!bytes) return FREDEC_EINVAL;
  if (precision != FREDEC_FP64 && precision != FREDEC_FP32) return FREDEC_EINVAL;
  FapLayout L;
  int rc = fap_layout(N, F, m_max, precision, L);
  if (rc) return rc;
  *bytes = L.total;
  return FREDEC_OK;
}

int fredec_residual_fap(fredec_ctx* ctx, void* stream, const double* t, const double* x, const double* w, int64_t N,
                        const double* sol_f, const int64_t* sol_off, int32_t n_sol, double df, int64_t F, double A1,
                        int32_t precision, void* ws, size_t ws_bytes, double* fap_out, double* zmax_out,
                        int64_t* jmax_out) {
  if (!t || !x || !w || N <= 0 || F < 3 || !fap_out || !zmax_out || !jmax_out) return FREDEC_EINVAL;
  if (!(A1 > 0.0) || !std::isfinite(A1) || !std::isfinite(df) || df == 0.0) return FREDEC_EINVAL;
  if (precision != FREDEC_FP64 && precision != FREDEC_FP32) return FREDEC_EINVAL;
  int32_t m_max = 0;
  int rc = fap_check(sol_f, sol_off, n_sol, &m_max);
  if (rc) return rc;
  if (N - 3 * (static_cast<int64_t>(m_max) + 1) - 1 <= 0) return FREDEC_EDOF;
  FapLayout L;
  if ((rc = fap_layout(N, F, m_max, precision, L))) return rc;
  if (!ws || ws_bytes < L.total) return FREDEC_ENOMEM;
  if (!ctx) return FREDEC_EINVAL;
  DeviceGuard g(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* d_z = at<double>(ws, L.off_z);
  uint8_t* d_fl = at<uint8_t>(ws, L.off_fl);
  double* d_lb = at<double>(ws, L.off_lb);
  int32_t* d_st = at<int32_t>(ws, L.off_st);
  Peak* d_part = at<Peak>(ws, L.off_part);
  Peak* d_best = at<Peak>(ws, L.off_best);
  Peak* d_pk = at<Peak>(ws, L.off_peaks);
  unsigned long long* d_cnt = at<unsigned long long>(ws, L.off_count);
  const int64_t soff[2] = {0, N};
  double W = 0.0;
  for (int32_t k = 0; k < n_sol; ++k) {
    std::vector<double> base(sol_f + sol_off[k], sol_f + sol_off[k + 1]);
    const int64_t boff[2] = {0, static_cast<int64_t>(base.size())};
    if ((rc = fredec_scan(ctx, stream, 1, t, x, w, soff, base.empty() ? nullptr : base.data(), boff, &df, &F,
                          precision, at<void>(ws, L.off_scan), L.scan_ws, d_z, d_fl, d_lb, d_st)))
      return rc;
    int32_t status = 0;
    if ((rc = sync_read(st, &status, d_st, sizeof(status)))) return rc;
    if (status) return status;
    if (k == 0) {
      double stats[6];
      // the scan workspace begins with SeriesIn[1] then SeriesHdr[1]
      const SeriesHdr* hdr = at<const SeriesHdr>(ws, L.off_scan + align_up(sizeof(SeriesIn)));
      if ((rc = sync_read(st, stats, hdr->stats, sizeof(stats)))) return rc;
      W = std::fabs(static_cast<double>(F) * df * stats[4]);
    }
    if (launch_peak_max(st, d_z, d_fl, F, d_part, d_best) != hipSuccess) return FREDEC_EDEVICE;
    Peak best{-1, 0.0};
    if ((rc = sync_read(st, &best, d_best, sizeof(best)))) return rc;
    if (best.j >= 0 && precision == FREDEC_FP32) {
      // the float32 peaks that can be the highest (within the float32 error
      // bound of its maximum), followed uphill in float64
      const double zmin = best.z - 1e-4 * std::max(std::fabs(best.z), 1.0);
      zero_count_kernel<<<1, 1, 0, st>>>(d_cnt);
      if (hipGetLastError() != hipSuccess) return FREDEC_EDEVICE;
      if (launch_peaks(st, d_z, d_fl, F, zmin, d_pk, d_cnt, L.peak_cap) != hipSuccess) return FREDEC_EDEVICE;
      unsigned long long cnt = 0;
      if ((rc = sync_read(st, &cnt, d_cnt, sizeof(cnt)))) return rc;
      if (static_cast<int64_t>(cnt) > L.peak_cap) return FREDEC_EDEVICE;  // cannot happen: peaks are not adjacent
      std::vector<Peak> pk(static_cast<size_t>(cnt));
      if ((rc = sync_read(st, pk.data(), d_pk, sizeof(Peak) * pk.size()))) return rc;
      ClimbBuffers cb{at<int64_t>(ws, L.off_idx), at<double>(ws, L.off_zat), at<uint8_t>(ws, L.off_flat),
                      at<void>(ws, L.off_at), L.at_ws};
      if ((rc = climb_f64(ctx, stream, t, x, w, N, base, df, F, cb, -HUGE_VAL, pk))) return rc;
      best = Peak{-1, 0.0};
      for (const Peak& p : pk)  // sorted by index: ties keep the lower one
        if (best.j < 0 || p.z > best.z) best = p;
    }
    if (best.j < 0) {
      fap_out[k] = 1.0;
      zmax_out[k] = std::nan("");
      jmax_out[k] = -1;
    } else {
      fap_out[k] = std::min(1.0, std::exp(log_fap(best.z, 1, W, A1)));
      zmax_out[k] = best.z;
      jmax_out[k] = best.j;
    }
  }
  return FREDEC_OK;
}

}  // extern "C"
