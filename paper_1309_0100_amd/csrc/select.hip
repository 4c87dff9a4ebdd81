// Selection steps: periodogram peaks (Sect. 4.2, Phase 1) and the backward
// cascade of relative tests over all subsets of the pool (Sect. 4.4, Phase 3;
// the 2^m - 1 joint tests of Sect. 2).
#include "fredec_internal.h"
#include "fredec_select_internal.h"

namespace fredec {

namespace {

// Interior local maxima z_{j-1} < z_j >= z_{j+1} with no flag and z_j > zmin,
// appended (unordered) to `out`; the caller sorts.
__global__ void peaks_kernel(const double* __restrict__ z, const uint8_t* __restrict__ flags, int64_t F, double zmin,
                             Peak* __restrict__ out, unsigned long long* __restrict__ count, int64_t cap) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x + 1;
  if (j >= F - 1) return;
  const double zj = z[j];
  const bool fl = flags ? (flags[j] & ~FREDEC_FLAG_RESCORED) != 0 : false;
  if (!fl && zj > zmin && zj > z[j - 1] && zj >= z[j + 1]) {
    const unsigned long long slot = atomicAdd(count, 1ull);
    if (static_cast<int64_t>(slot) < cap) out[slot] = Peak{j, zj};
  }
}

// Survival of every subset S (mask 1..2^n-1): for all proper subsets S'
// (including the empty one, l(0) = l_0) the relative statistic
//   z_{S|S'} = (N - 3|S| - 1)/2 ln(l(S') / l(S))
// must exceed zcrit[|S| - |S'|].  Subsets are visited in decreasing mask
// order and the first failure ends the test (the early exit of Sect. 4.4;
// the outcome equals the full set of tests).  Also writes the goodness of
// fit G = l(S) (N - 1) / (N - 3|S| - 1) (Sect. 6).
__global__ void cascade_kernel(const double* __restrict__ ltab, int n, int64_t N, CascadeParams p,
                               uint8_t* __restrict__ surv, double* __restrict__ G) {
  const uint64_t S = static_cast<uint64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  const uint64_t full = (uint64_t(1) << n) - 1;
  if (S > full) return;
  if (S == 0) {
    surv[0] = 0;
    if (G) G[0] = __builtin_nan("");
    return;
  }
  const int k = __builtin_popcountll(S);
  const double NH = static_cast<double>(N - 3 * k - 1);
  const double lS = ltab[S];
  if (G) G[S] = lS * static_cast<double>(N - 1) / NH;
  bool ok = NH > 0.0 && lS > 0.0 && isfinite(lS);
  uint64_t sub = (S - 1) & S;
  while (ok) {
    const int d = k - __builtin_popcountll(sub);
    const double zrel = 0.5 * NH * log(ltab[sub] / lS);
    ok = zrel > p.zc[d];
    if (sub == 0) break;
    sub = (sub - 1) & S;
  }
  surv[S] = ok ? 1 : 0;
}

// sup[S] |= sup[S | 2^b] for S without bit b: after passes b = 0..n-1,
// sup[S] = 1 iff some superset of S (S included) survives.
__global__ void superset_pass_kernel(uint8_t* __restrict__ sup, int n, int b) {
  const uint64_t S = static_cast<uint64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  if (S >= (uint64_t(1) << n)) return;
  if (!(S >> b & 1)) sup[S] |= sup[S | (uint64_t(1) << b)];
}

// maximal[S]: S survives and no strict superset does.
__global__ void maximal_kernel(const uint8_t* __restrict__ surv, const uint8_t* __restrict__ sup, int n,
                               uint8_t* __restrict__ maximal) {
  const uint64_t S = static_cast<uint64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  if (S >= (uint64_t(1) << n)) return;
  bool m = surv[S] != 0;
  for (int b = 0; b < n && m; ++b)
    if (!(S >> b & 1) && sup[S | (uint64_t(1) << b)]) m = false;
  maximal[S] = m ? 1 : 0;
}

__global__ void copy_u8_kernel(const uint8_t* __restrict__ a, uint8_t* __restrict__ b, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x;
  if (i < n) b[i] = a[i];
}

unsigned grid_of(uint64_t n) { return static_cast<unsigned>((n + BLOCK - 1) / BLOCK); }

// The better of two peaks: the larger z, then the lower index; j < 0 marks none.
__device__ __forceinline__ Peak better(const Peak& a, const Peak& b) {
  if (a.j < 0) return b;
  if (b.j < 0) return a;
  return (a.z > b.z || (a.z == b.z && a.j < b.j)) ? a : b;
}

// Block tree reduction of one peak per thread (BLOCK threads).
__device__ Peak block_best(Peak p, Peak* sh) {
  sh[threadIdx.x] = p;
  __syncthreads();
  for (int s = BLOCK / 2; s > 0; s >>= 1) {
    if (static_cast<int>(threadIdx.x) < s) sh[threadIdx.x] = better(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  return sh[0];
}

// Highest interior local maximum of z (the peak rule of peaks_kernel) within
// each block's grid points: part[blockIdx.x] (j = -1 if none).
__global__ void peak_max_partial_kernel(const double* __restrict__ z, const uint8_t* __restrict__ flags, int64_t F,
                                        Peak* __restrict__ part) {
  __shared__ Peak sh[BLOCK];
  const int64_t j = static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x + 1;
  Peak p{-1, 0.0};
  if (j < F - 1) {
    const double zj = z[j];
    const bool fl = flags ? (flags[j] & ~FREDEC_FLAG_RESCORED) != 0 : false;
    if (!fl && zj > z[j - 1] && zj >= z[j + 1]) p = Peak{j, zj};
  }
  const Peak b = block_best(p, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// The best of n partial results (one block).
__global__ void peak_max_final_kernel(const Peak* __restrict__ part, int64_t n, Peak* __restrict__ out) {
  __shared__ Peak sh[BLOCK];
  Peak p{-1, 0.0};
  for (int64_t k = threadIdx.x; k < n; k += BLOCK) p = better(p, part[k]);
  const Peak b = block_best(p, sh);
  if (threadIdx.x == 0) *out = b;
}

}  // namespace

hipError_t launch_peaks(hipStream_t st, const double* z, const uint8_t* flags, int64_t F, double zmin, Peak* out,
                        unsigned long long* count, int64_t cap) {
  if (F < 3) return hipSuccess;
  peaks_kernel<<<grid_of(static_cast<uint64_t>(F - 2)), BLOCK, 0, st>>>(z, flags, F, zmin, out, count, cap);
  return hipGetLastError();
}

int64_t peak_max_parts(int64_t F) { return F < 3 ? 1 : static_cast<int64_t>(grid_of(static_cast<uint64_t>(F - 2))); }

hipError_t launch_peak_max(hipStream_t st, const double* z, const uint8_t* flags, int64_t F, Peak* part, Peak* out) {
  const int64_t np = peak_max_parts(F);
  if (F >= 3) peak_max_partial_kernel<<<static_cast<unsigned>(np), BLOCK, 0, st>>>(z, flags, F, part);
  peak_max_final_kernel<<<1, BLOCK, 0, st>>>(part, F >= 3 ? np : 0, out);
  return hipGetLastError();
}

hipError_t launch_cascade(hipStream_t st, const double* ltab, int n, int64_t N, const CascadeParams& p, uint8_t* surv,
                          uint8_t* sup, uint8_t* maximal, double* G) {
  const uint64_t M = uint64_t(1) << n;
  cascade_kernel<<<grid_of(M), BLOCK, 0, st>>>(ltab, n, N, p, surv, G);
  copy_u8_kernel<<<grid_of(M), BLOCK, 0, st>>>(surv, sup, static_cast<int64_t>(M));
  for (int b = 0; b < n; ++b) superset_pass_kernel<<<grid_of(M), BLOCK, 0, st>>>(sup, n, b);
  maximal_kernel<<<grid_of(M), BLOCK, 0, st>>>(surv, sup, n, maximal);
  return hipGetLastError();
}

}  // namespace fredec
