"""Plain FP64 CPU oracle for the FREDEC multifrequency periodogram.

TEST INFRASTRUCTURE ONLY.  This module is imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``.
The product path (the C-ABI library and its Python binding) never imports,
links or calls it, and this module imports nothing from the product.

Everything is float64 NumPy, serial, written directly from the definitions of
Baluev, "Detecting multiple periodicities in observational data with the
multifrequency periodogram - II. Frequency Decomposer" (Astronomy and
Computing, arXiv:1309.0100).  Each function cites the passage it follows.

Readings of points where the paper is silent or garbled (all listed again in
the design notes of the repository):

* z ratio (eqs. zpow, zpowrel): the printed ratio (D-l_0)/(D-l_n) is garbled;
  l is a chi^2 minimum, so the statistic is z = (N_H/2) ln(l_ref / l) >= 0.
* Factor 2 in eq. lsq: l = D - g^T Q^{-1} g with g = <x phi>, Q = <phi phi^T>
  (the least-squares residual).
* N_H = N - 3 * (number of frequencies in the larger model) - 1, also for the
  fixed-frequency statistics; the residual scan uses N - 3m - 4.
* Time is centred (tau = t - <t>) but kept in its own unit; frequencies keep
  the user's unit.  This is eq. idn up to a joint rescaling of t and f.
* Grid f_j = (j+1) * df, j = 0..F-1 (f = 0 is excluded).
* Removable singularity near a base frequency: |f - f'| * T_eff < 0.05 gives
  z := 0 and flag bit 0.  A Cholesky pivot below PIVOT_TOL times its diagonal
  gives z := 0 and flag bit 1; l <= 0 gives z := +inf and flag bit 2.
* Tuples with two frequencies closer than 0.05 / T_eff, or a non-SPD normal
  matrix, get z := -inf and flag bit 3.
* FAP constants A~_n of eq. zFAP are not printed: caller-supplied, default 1
  (parity with the paper unpinned for them).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

TWO_PI = 2.0 * np.pi
PIVOT_TOL = 1e-13      # relative Cholesky pivot threshold
MASK_WIDTH = 0.05      # |f - f'| * T_eff below this is masked (removable singularity)
MERGE_WIDTH = 0.5      # Phase 1 candidates closer than this (in 1/T_eff) are merged

FLAG_MASKED = 1
FLAG_SINGULAR = 2
FLAG_PERFECT = 4
FLAG_DEGENERATE = 8


# ----------------------------------------------------------------- Sect. 2, 4.1
@dataclass
class Normalized:
    tau: np.ndarray    # t - <t>
    xt: np.ndarray     # (x - <x>) / s_x
    wt: np.ndarray     # w / sum(w)
    tbar: float
    xbar: float
    sx: float
    var_t: float
    T_eff: float

    @property
    def N(self) -> int:
        return int(self.tau.shape[0])


def normalize(t, x, w) -> Normalized:
    """Initial normalisation, Sect. 4.1 eq. idn: <1> = 1, <x> = 0, <x^2> = 1,
    <t> = 0 (time centred, not rescaled).  Effective span T_eff = sqrt(4 pi
    Var(t)) with the weighted (population) variance, Sect. 2."""
    t = np.asarray(t, np.float64)
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    if not (np.all(np.isfinite(t)) and np.all(np.isfinite(x)) and np.all(np.isfinite(w))):
        raise ValueError("non-finite input")
    if np.any(w <= 0):
        raise ValueError("weights must be positive (Sect. 2: Var eps_i = kappa / w_i)")
    wt = w / np.sum(w)
    tbar = float(np.sum(wt * t))
    tau = t - tbar
    xbar = float(np.sum(wt * x))
    d = x - xbar
    sx2 = float(np.sum(wt * d * d))
    var_t = float(np.sum(wt * tau * tau))
    # zero variance up to rounding: below (1e-14)^2 of the second moment
    if sx2 <= 1e-28 * float(np.sum(wt * x * x)) or var_t <= 1e-28 * float(np.sum(wt * t * t)):
        raise ValueError("degenerate series: zero weighted variance of x or t")
    sx = math.sqrt(sx2)
    return Normalized(tau, d / sx, wt, tbar, xbar, sx, var_t, math.sqrt(4.0 * math.pi * var_t))


# ------------------------------------------------------------------ Sect. 2, 3
def design(tau, freqs) -> np.ndarray:
    """Basis of model H_n, eq. Hn: columns 1, cos(2 pi f_k t), sin(2 pi f_k t)."""
    freqs = np.atleast_1d(np.asarray(freqs, np.float64))
    cols = [np.ones_like(tau)]
    for f in freqs:
        ph = TWO_PI * f * tau
        cols.append(np.cos(ph))
        cols.append(np.sin(ph))
    return np.stack(cols, axis=1)


def cholesky_checked(Q, rel_tol=PIVOT_TOL, pivots=False):
    """Textbook Cholesky Q = L L^T over a stack of matrices (..., n, n).
    Returns (L, ok) where ok is False if any pivot falls below rel_tol times
    its diagonal entry (Sect. 3: Q = L L^T); with pivots=True also the
    relative pivots d_j / Q_jj (..., n), the conditioning of each column
    against the ones before it."""
    Q = np.asarray(Q, np.float64)
    n = Q.shape[-1]
    L = np.zeros_like(Q)
    ok = np.ones(Q.shape[:-2], bool)
    rel = np.zeros(Q.shape[:-1])
    for j in range(n):
        d = Q[..., j, j] - np.sum(L[..., j, :j] ** 2, axis=-1)
        ok &= d > rel_tol * Q[..., j, j]
        rel[..., j] = d / Q[..., j, j]
        ljj = np.sqrt(np.where(d > 0, d, 1.0))
        L[..., j, j] = ljj
        for i in range(j + 1, n):
            L[..., i, j] = (Q[..., i, j] - np.sum(L[..., i, :j] * L[..., j, :j], axis=-1)) / ljj
    return (L, ok, rel) if pivots else (L, ok)


def forward_subst(L, g):
    """a = L^{-1} g for lower-triangular L over a stack."""
    n = L.shape[-1]
    a = np.zeros(np.broadcast_shapes(L.shape[:-1], np.shape(g)))
    for i in range(n):
        a[..., i] = (g[..., i] - np.sum(L[..., i, :i] * a[..., :i], axis=-1)) / L[..., i, i]
    return a


def back_subst(L, a):
    """theta = L^{-T} a for lower-triangular L over a stack."""
    n = L.shape[-1]
    th = np.zeros_like(a)
    for i in range(n - 1, -1, -1):
        th[..., i] = (a[..., i] - np.sum(L[..., i + 1:, i] * th[..., i + 1:], axis=-1)) / L[..., i, i]
    return th


@dataclass
class Fit:
    l: float           # min_theta chi^2 (normalised data: l_0 = 1)
    theta: np.ndarray  # theta* = (c, a_1, b_1, ..., a_n, b_n)
    ok: bool


def lsq(nrm: Normalized, freqs) -> Fit:
    """Linear least squares at fixed frequencies, Sect. 3 eqs. lsq, grad,
    fisher: g = <x phi>, Q = <phi phi^T>, Q = L L^T, a = L^{-1} g,
    l = D - a.a with D = <x^2>, theta* = L^{-T} a."""
    Phi = design(nrm.tau, freqs)
    Wphi = Phi * nrm.wt[:, None]
    Q = Wphi.T @ Phi
    g = Wphi.T @ nrm.xt
    D = float(np.sum(nrm.wt * nrm.xt * nrm.xt))
    L, ok = cholesky_checked(Q)
    a = forward_subst(L, g)
    th = back_subst(L, a)
    return Fit(D - float(a @ a), th, bool(ok))


def n_dof(N: int, n_freq: int) -> int:
    """N_H = N - dim H_n = N - 3n - 1 (Sect. 2, below eq. zpow)."""
    return N - 3 * n_freq - 1


# ------------------------------------------------------------ residual scan
def grid(df: float, F: int, idx=None) -> np.ndarray:
    j = np.arange(F, dtype=np.int64) if idx is None else np.asarray(idx, np.int64)
    return (j + 1).astype(np.float64) * df


@dataclass
class ScanResult:
    z: np.ndarray
    flags: np.ndarray
    l_base: float
    T_eff: float
    freqs: np.ndarray
    rho: np.ndarray = None  # smaller relative Cholesky pivot of the two trial columns per frequency


def scan(t, x, w, base_f, df: float, F: int, idx=None, block: int = 256) -> ScanResult:
    """Residual periodogram z_{1|m}(f | f'), eq. zpowrel with n = 1: for every
    grid frequency f the model H_{m+1} with frequencies f' U {f} is fitted by
    plain least squares (full normal matrix and Cholesky per frequency) and
    z = (N - 3m - 4)/2 * ln(l_m(f') / l_{m+1}(f', f))."""
    nrm = normalize(t, x, w)
    base_f = np.atleast_1d(np.asarray(base_f, np.float64))
    m = base_f.size
    N = nrm.N
    NH = n_dof(N, m + 1)
    if NH <= 0:
        raise ValueError("too few samples for the residual scan (N - 3m - 4 <= 0)")
    base = lsq(nrm, base_f)
    if not base.ok:
        raise ValueError("singular base model")
    lm = base.l
    f = grid(df, F, idx)
    z = np.zeros(f.size)
    flags = np.zeros(f.size, np.uint8)
    rho = np.zeros(f.size)
    Phi_b = design(nrm.tau, base_f)
    D = float(np.sum(nrm.wt * nrm.xt * nrm.xt))
    for s in range(0, f.size, block):
        fb = f[s:s + block]
        ph = TWO_PI * fb[:, None] * nrm.tau[None, :]
        Phi = np.concatenate([np.broadcast_to(Phi_b, (fb.size,) + Phi_b.shape),
                              np.cos(ph)[:, :, None], np.sin(ph)[:, :, None]], axis=2)
        WPhi = Phi * nrm.wt[None, :, None]
        Q = np.matmul(np.transpose(WPhi, (0, 2, 1)), Phi)
        g = np.einsum('bnk,n->bk', WPhi, nrm.xt)
        L, ok, rel = cholesky_checked(Q, pivots=True)
        rho[s:s + block] = np.min(rel[:, -2:], axis=1)
        a = forward_subst(L, g)
        l1 = D - np.sum(a * a, axis=1)
        zb = np.zeros(fb.size)
        fl = np.zeros(fb.size, np.uint8)
        good = ok & (l1 > 0)
        zb[good] = 0.5 * NH * np.log(lm / l1[good])
        fl[~ok] |= FLAG_SINGULAR
        zb[~ok] = 0.0
        perfect = ok & (l1 <= 0)
        fl[perfect] |= FLAG_PERFECT
        zb[perfect] = np.inf
        if m:
            near = np.any(np.abs(fb[:, None] - base_f[None, :]) * nrm.T_eff < MASK_WIDTH, axis=1)
            fl[near] = FLAG_MASKED
            zb[near] = 0.0
        z[s:s + block] = zb
        flags[s:s + block] = fl
    return ScanResult(z, flags, lm, nrm.T_eff, f, rho)


# ------------------------------------------------------------------ tuples
def tuple_fit(nrm: Normalized, freqs):
    """Absolute statistic of eq. zpow at fixed frequencies:
    z_n(f) = (N - 3n - 1)/2 * ln(l_0 / l_n(f)), with l_0 the constant-model
    minimum (= 1 after eq. idn).  Returns (z, l, theta, flag)."""
    freqs = np.atleast_1d(np.asarray(freqs, np.float64))
    n = freqs.size
    NH = n_dof(nrm.N, n)
    l0 = lsq(nrm, []).l
    fs = np.sort(freqs)
    if n > 1 and np.any(np.diff(fs) * nrm.T_eff < MASK_WIDTH):
        return -np.inf, np.nan, None, FLAG_DEGENERATE
    fit = lsq(nrm, freqs)
    if not fit.ok:
        return -np.inf, np.nan, None, FLAG_DEGENERATE
    if fit.l <= 0:
        return np.inf, fit.l, fit.theta, FLAG_PERFECT
    return 0.5 * NH * math.log(l0 / fit.l), fit.l, fit.theta, 0


def model_jacobian(nrm: Normalized, freqs, theta):
    """Derivatives of the model of eq. Hn with respect to the frequencies:
    J_k = d mu / d f_k = 2 pi t (-a_k sin 2 pi f_k t + b_k cos 2 pi f_k t)."""
    freqs = np.atleast_1d(np.asarray(freqs, np.float64))
    J = np.empty((nrm.N, freqs.size))
    for k, f in enumerate(freqs):
        ph = TWO_PI * f * nrm.tau
        a, b = theta[1 + 2 * k], theta[2 + 2 * k]
        J[:, k] = TWO_PI * nrm.tau * (-a * np.sin(ph) + b * np.cos(ph))
    return J


def tuple_grad(nrm: Normalized, freqs):
    """z and its gradient by the envelope theorem on l = min_theta chi^2:
    dl/df_k = -2 <r J_k> with r = x - Phi theta*, hence
    dz/df_k = (N_H / l) <r J_k>;  also the diagonal curvature
    h_k = (N_H / l) <J_k^2>.  Returns (z, l, grad, h)."""
    freqs = np.atleast_1d(np.asarray(freqs, np.float64))
    z, l, th, flag = tuple_fit(nrm, freqs)
    if flag & FLAG_DEGENERATE:
        return z, l, np.full(freqs.size, np.nan), np.full(freqs.size, np.nan)
    NH = n_dof(nrm.N, freqs.size)
    r = nrm.xt - design(nrm.tau, freqs) @ th
    J = model_jacobian(nrm, freqs, th)
    g = (nrm.wt * r) @ J
    h = nrm.wt @ (J * J)
    return z, l, NH / l * g, NH / l * h


def gn_step(nrm: Normalized, freqs, theta, frozen=()):
    """One Gauss-Newton step of Sect. 3 (eq. lsqf): with xi = (theta, f) and
    J~ = [Phi, J_1..J_n], Q_f = <J~ J~^T> and g_f = <r J~> (its theta part
    vanishes at theta*); the step is Q_f^{-1} g_f and its f part is returned.
    Frequencies whose index is in `frozen` are held fixed: their columns J_k
    are left out of J~ and their step is 0."""
    freqs = np.atleast_1d(np.asarray(freqs, np.float64))
    free = [k for k in range(freqs.size) if k not in set(frozen)]
    Phi = design(nrm.tau, freqs)
    J = model_jacobian(nrm, freqs, theta)[:, free]
    Jt = np.concatenate([Phi, J], axis=1)
    r = nrm.xt - Phi @ theta
    WJ = Jt * nrm.wt[:, None]
    Qf = WJ.T @ Jt
    gf = WJ.T @ r
    L, ok = cholesky_checked(Qf)
    step = np.zeros(freqs.size)
    if not ok:
        return step, False
    step[free] = back_subst(L, forward_subst(L, gf))[Phi.shape[1]:]
    return step, True


@dataclass
class Refined:
    f: np.ndarray
    l: float
    z: float
    converged: bool    # the iteration stopped on the step tolerance
    passes: int
    flag: int


def gn_refine(nrm: Normalized, f0, steps: int, clamp: float = 0.25, max_halvings: int = 5,
              tol: float = 1e-10, accept_rtol: float = 1e-12, frozen=()) -> Refined:
    """Local refinement l_{n,loc} of Sect. 3 (and the local statistic of
    Sect. 2): Gauss-Newton steps on f with theta re-solved at every iterate.
    Step control (not given in the paper): the step is scaled so that
    max |df_k| T_eff <= clamp; a trial point whose l exceeds the accepted l by
    more than accept_rtol is rejected and the step halved (at most
    max_halvings times in a row); the iteration stops once
    max |df_k| T_eff < tol.  `steps` trial evaluations follow the evaluation
    at f0, so 1 + steps least-squares fits are made in total.  The
    frequencies with an index in `frozen` stay at their start values."""
    f0 = np.atleast_1d(np.asarray(f0, np.float64))
    n = f0.size
    T = nrm.T_eff
    NH = n_dof(nrm.N, n)
    l0 = lsq(nrm, []).l
    f_acc = f0.copy()
    l_acc = np.inf
    th_acc = None
    step = np.zeros(n)
    f_try = f0.copy()
    halvings = 0
    done = False
    converged = False      # stopped because the step fell below tol
    passes = 0
    for _ in range(steps + 1):
        if done:
            break
        passes += 1
        fs = np.sort(f_try)
        degenerate = n > 1 and np.any(np.diff(fs) * T < MASK_WIDTH)
        fit = None if degenerate else lsq(nrm, f_try)
        if fit is not None and fit.ok and fit.l <= l_acc * (1.0 + accept_rtol):
            f_acc, l_acc, th_acc = f_try.copy(), fit.l, fit.theta
            step, ok = gn_step(nrm, f_acc, th_acc, frozen)
            halvings = 0
            big = np.max(np.abs(step)) * T
            if not ok or big < tol:
                done = True
                converged = ok
                continue
            if big > clamp:
                step = step * (clamp / big)
        else:
            if th_acc is None:      # the start point itself is degenerate
                return Refined(f0, np.nan, -np.inf, False, passes, FLAG_DEGENERATE)
            step = 0.5 * step
            halvings += 1
            if halvings > max_halvings:
                done = True
                continue
        f_try = f_acc + step
    if l_acc <= 0:
        return Refined(f_acc, l_acc, np.inf, converged, passes, FLAG_PERFECT)
    return Refined(f_acc, l_acc, 0.5 * NH * math.log(l0 / l_acc), converged, passes, 0)


def ascent(nrm: Normalized, f0, steps: int = 20, clamp: float = 0.1):
    """Fixed-step preconditioned ascent of z over the frequencies (not in the
    paper; used by the differentiable refinement workload): each step moves
    f_k by <r J_k> / <J_k^2> (the Gauss-Newton step for f_k alone with theta
    fixed), clipped to |df_k| <= clamp / T_eff.  Returns (f, z, l)."""
    f = np.atleast_1d(np.asarray(f0, np.float64)).copy()
    T = nrm.T_eff
    for _ in range(steps):
        z, l, g, h = tuple_grad(nrm, f)
        if not np.all(np.isfinite(g)):
            break
        d = g / h
        f = f + np.clip(d, -clamp / T, clamp / T)
    z, l, _, _ = tuple_fit(nrm, f)
    return f, z, l


# --------------------------------------------------------------- FAP, eq. zFAP
def log_fap(z: float, d: int, W: float, A: float = 1.0) -> float:
    """log of the bound FAP_d(z) ~ A_d W^d e^{-z} z^{3d/2 - 1}, eq. zFAP."""
    return math.log(A) + d * math.log(W) - z + (1.5 * d - 1.0) * math.log(z)


def zcrit(d: int, W: float, fap: float, A: float = 1.0) -> float:
    """Threshold z_crit with FAP_d(z_crit) = fap on the decreasing branch
    z > 3d/2 - 1 of eq. zFAP (bisection in float64)."""
    lo = max(1.5 * d - 1.0, 1e-300)
    target = math.log(fap)
    if log_fap(lo if lo > 0 else 1e-300, d, W, A) <= target:
        return lo
    hi = max(2.0 * lo, 1.0)
    while log_fap(hi, d, W, A) > target:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if log_fap(mid, d, W, A) > target:
            lo = mid
        else:
            hi = mid
    return hi


def zcrit_table(n: int, W: float, fap: float, A=None) -> np.ndarray:
    """zc[d] for d = 1..n (zc[0] unused)."""
    A = np.ones(n + 1) if A is None else np.asarray(A, np.float64)
    out = np.zeros(n + 1)
    for d in range(1, n + 1):
        out[d] = zcrit(d, W, fap, float(A[d]))
    return out


# ------------------------------------------------------------ Phase 1, Sect. 4.2
def local_maxima(z: np.ndarray, flags: np.ndarray) -> np.ndarray:
    """Interior grid points with z_{j-1} < z_j >= z_{j+1} and no flag."""
    j = np.arange(1, z.size - 1)
    ok = (z[j] > z[j - 1]) & (z[j] >= z[j + 1]) & (flags[j] == 0)
    return j[ok]


@dataclass
class Phase1Result:
    pool: np.ndarray        # candidate frequencies, ascending
    pool_z: np.ndarray      # z of each candidate in the scan that found it
    base: np.ndarray        # SLICK base frequencies in order of addition
    n_scans: int
    truncated: int          # candidates dropped by the cap
    W: float


def phase1(t, x, w, df: float, F: int, fap0: float = 0.05, fap1: float = 0.1, A1: float = 1.0,
           pool_cap: int | None = None, max_scans: int = 64, scan_fn=None) -> Phase1Result:
    """Preliminary scan of Sect. 4.2 (QUICK + SLICK): residual periodograms are
    computed in sequence; each adds its largest peak to the base model while
    its FAP_1 < FAP_0.  Every peak with FAP_1 < FAP_1-threshold and height at
    least half of the maximum peak joins the pool.  The pool is capped at N/10
    by dropping the largest-FAP candidates.  Rules for ties, merging and the
    final scan are readings (see module docstring of the repository design)."""
    if not (fap1 >= fap0 > 0):
        raise ValueError("FAP_1 >= FAP_0 required (Sect. 4)")
    scan_fn = scan if scan_fn is None else scan_fn
    nrm = normalize(t, x, w)
    N = nrm.N
    W = F * df * nrm.T_eff
    zc1 = zcrit(1, W, fap1, A1)
    zc0 = zcrit(1, W, fap0, A1)
    cap = N // 10 if pool_cap is None else pool_cap
    base: list[float] = []
    pool_f: list[float] = []
    pool_z: list[float] = []
    scans = 0
    while scans < max_scans and n_dof(N, len(base) + 1) > 0:
        res = scan_fn(t, x, w, np.asarray(base), df, F)
        scans += 1
        pk = local_maxima(res.z, res.flags)
        if pk.size == 0:
            break
        zp = res.z[pk]
        order = np.lexsort((pk, -zp))          # descending z, ties -> lower index
        jmax = pk[order[0]]
        zmax = res.z[jmax]
        for o in order:
            zj = zp[o]
            if not (zj > zc1 and zj >= 0.5 * zmax):
                continue
            fj = res.freqs[pk[o]]
            if any(abs(fj - q) * nrm.T_eff < MERGE_WIDTH for q in pool_f):
                continue
            pool_f.append(fj)
            pool_z.append(zj)
        if zmax > zc0:
            base.append(res.freqs[jmax])
        else:
            break
    pf = np.asarray(pool_f)
    pz = np.asarray(pool_z)
    truncated = 0
    if pf.size > cap:
        keep = np.lexsort((pf, -pz))[:cap]     # smallest FAP (largest z), ties -> lower f
        truncated = pf.size - cap
        pf, pz = pf[keep], pz[keep]
    order = np.argsort(pf, kind="stable")
    return Phase1Result(pf[order], pz[order], np.asarray(base), scans, truncated, W)


# ------------------------------------------------------------ Phase 2, Sect. 4.3
def phase2(nrm: Normalized, pool, refine_steps: int = 0):
    """Forward cascade of Sect. 4.3: l_{m,loc} for every non-empty subset of
    the pool (bit k of the mask selects pool[k]).  Returns the table
    l[0..2^n-1] with l[0] = l_0 and the refined frequencies."""
    pool = np.asarray(pool, np.float64)
    n = pool.size
    ltab = np.empty(1 << n)
    ltab[0] = lsq(nrm, []).l
    fout = np.full((1 << n, n), np.nan)
    for mask in range(1, 1 << n):
        members = [k for k in range(n) if mask >> k & 1]
        f0 = pool[members]
        if refine_steps > 0:
            r = gn_refine(nrm, f0, refine_steps)
            ltab[mask] = r.l if r.flag == 0 else np.nan
            fout[mask, members] = r.f
        else:
            z, l, _, flag = tuple_fit(nrm, f0)
            ltab[mask] = l if flag == 0 else np.nan
            fout[mask, members] = f0
    return ltab, fout


# ------------------------------------------------------------ Phase 3, Sect. 4.4
def popcount(m: int) -> int:
    return bin(m).count("1")


def proper_subsets(S: int) -> np.ndarray:
    """Every proper subset S' of the mask S, the empty set included."""
    subs = []
    sub = (S - 1) & S
    while True:
        subs.append(sub)
        if sub == 0:
            break
        sub = (sub - 1) & S
    return np.asarray(subs, np.int64)


def survives(ltab, S: int, N: int, zc) -> bool:
    """Sect. 4.4 / Sect. 2: the subset S passes every relative test against
    its proper subsets S' (including the empty one):
    z_{S|S'} = (N - 3|S| - 1)/2 * ln(l(S') / l(S)) > z_crit[|S| - |S'|]."""
    k = popcount(S)
    NH = n_dof(N, k)
    lS = ltab[S]
    if not np.isfinite(lS) or lS <= 0 or NH <= 0:
        return False
    subs = proper_subsets(S)
    d = k - np.array([popcount(int(s)) for s in subs])
    with np.errstate(invalid="ignore", divide="ignore"):
        zrel = 0.5 * NH * np.log(ltab[subs] / lS)
    return bool(np.all(zrel > zc[d]))


def supersets(R: int, n: int) -> np.ndarray:
    """Every subset S of {0..n-1} that contains the mask R: R joined with each
    subset of the remaining bits."""
    free = [b for b in range(n) if not R >> b & 1]
    T = np.zeros(1 << len(free), np.int64)
    k = np.arange(1 << len(free), dtype=np.int64)
    for j, b in enumerate(free):
        T |= ((k >> j) & 1) << b
    return T | R


def survive_table(ltab, n: int, N: int, zc) -> np.ndarray:
    """The rule of survives() for every subset at once (Sect. 4.4, Sect. 2):
    for each non-empty removed set R and each S containing it, the test of S
    against S' = S minus R at depth |R|.  survive[S] is True iff S passes all
    of them; survive[0] is False."""
    ltab = np.asarray(ltab, np.float64)
    M = 1 << n
    pc = np.array([popcount(S) for S in range(M)], np.int64)
    NH = N - 3 * pc - 1
    with np.errstate(invalid="ignore"):
        ok = np.isfinite(ltab) & (ltab > 0) & (NH > 0)
    ok[0] = False
    for R in range(1, M):
        S = supersets(R, n)
        with np.errstate(invalid="ignore", divide="ignore"):
            zrel = 0.5 * NH[S] * np.log(ltab[S ^ R] / ltab[S])
        ok[S] &= zrel > zc[pc[R]]
    return ok


def maximal_sets(surv: np.ndarray, n: int) -> list[int]:
    """Survivors with no surviving strict superset (Sect. 4.4): the output
    sets, in increasing mask order.  A set has a surviving strict superset
    iff one of its one-element extensions survives or has one."""
    M = 1 << n
    has_sup = np.zeros(M, bool)
    for S in range(M - 1, 0, -1):
        for k in range(n):
            if not S >> k & 1:
                T = S | (1 << k)
                if surv[T] or has_sup[T]:
                    has_sup[S] = True
                    break
    return [S for S in range(1, M) if surv[S] and not has_sup[S]]


def phase3(ltab, n: int, N: int, zc) -> tuple[np.ndarray, np.ndarray, int]:
    """Backward cascade of Sect. 4.4 / the 2^m - 1 joint tests of Sect. 2:
    subset S survives iff for every proper subset S' (including the empty
    one) z_{S|S'} = (N - 3|S| - 1)/2 * ln(l(S') / l(S)) > z_crit[|S| - |S'|].
    Returns (survive[2^n] bool, maximal masks sorted by size then G, number of
    tests evaluated without early exit = 3^n - 2^n)."""
    ltab = np.asarray(ltab, np.float64)
    surv = np.zeros(1 << n, bool)
    tests = 0
    for S in range(1, 1 << n):
        tests += (1 << popcount(S)) - 1
        surv[S] = survives(ltab, S, N, zc)
    maximal = maximal_sets(surv, n)
    G = {S: ltab[S] * (N - 1) / n_dof(N, popcount(S)) for S in maximal}
    maximal.sort(key=lambda S: (popcount(S), G[S], S))
    return surv, np.asarray(maximal, np.int64), tests


def goodness(l: float, N: int, m: int) -> float:
    """G = l_{m,loc} N_H0 / N_Hm, Sect. 6 item 2."""
    return l * (N - 1) / n_dof(N, m)


# ------------------------------------------- Phase 4 and the report of Sect. 6
def residual_fap(t, x, w, freqs, df: float, F: int, A1: float = 1.0):
    """Single-frequency FAP of the highest peak left in the residual
    periodogram of a solution (Sect. 6, last item of the per-solution output):
    the residual scan on the grid with the solution's frequencies as the base
    model, its highest interior local maximum z_max (ties -> lowest index),
    and FAP_1(z_max) of eq. zFAP with W = f_max T_eff, capped at 1.  Returns
    (fap, z_max, grid index of that peak); (1, nan, -1) when the periodogram
    has no peak."""
    res = scan(t, x, w, np.atleast_1d(np.asarray(freqs, np.float64)), df, F)
    pk = local_maxima(res.z, res.flags)
    if pk.size == 0:
        return 1.0, float("nan"), -1
    j = int(pk[np.argmax(res.z[pk])])
    z = float(res.z[j])
    W = F * df * res.T_eff
    return min(1.0, math.exp(log_fap(z, 1, W, A1))), z, j


def loglik_terms(nrm: Normalized, freqs) -> np.ndarray:
    """Per-sample Gaussian log-likelihood of the least-squares fit of model
    H_n at the given frequencies, with the relative weights known and the
    noise scale fitted by maximum likelihood (the noise model of Sect. 2):
    sample i has variance l / (N w~_i), so
        ll_i = -1/2 ln(2 pi l / (N w~_i)) - N w~_i r_i^2 / (2 l),
    r = x~ - Phi theta*, l = <r^2> (normalised data)."""
    fit = lsq(nrm, freqs)
    r = nrm.xt - design(nrm.tau, freqs) @ fit.theta
    l = float(np.sum(nrm.wt * r * r))
    N = nrm.N
    return -0.5 * np.log(TWO_PI * l / (N * nrm.wt)) - N * nrm.wt * r * r / (2.0 * l)


def vuong(nrm: Normalized, f_ref, f_alt) -> float:
    """Vuong's statistic for two non-nested fits (Phase 4 of Sect. 4 and
    Sect. 6): with d_i = ll_i(ref) - ll_i(alt) the per-sample log-likelihood
    differences, V = sum d / (sqrt(N) omega), omega^2 = mean(d^2) - mean(d)^2;
    positive when the reference fits better.  The paper does not print the
    formula: this is the plain statistic, without a correction for the
    numbers of parameters.  0 when omega = 0 (identical fits)."""
    d = loglik_terms(nrm, f_ref) - loglik_terms(nrm, f_alt)
    N = d.size
    om2 = float(np.mean(d * d) - np.mean(d) ** 2)
    if om2 <= 0.0:
        return 0.0
    return float(np.sum(d) / (math.sqrt(N) * math.sqrt(om2)))


def phase4(nrm: Normalized, solutions, vuong_max: float = 5.0):
    """Phase 4 of Sect. 4 with the report of Sect. 6: the solutions (lists of
    frequencies) in chi^2-increase order grouped by their number of
    frequencies (within a group G and chi^2 have the same order), G of each
    (Sect. 6), the Vuong statistic of the smallest-G solution against each,
    and whether the solution is kept by the filter V < vuong_max (default 5).
    Returns a list of dicts in output order."""
    rows = []
    for k, f in enumerate(solutions):
        f = np.sort(np.atleast_1d(np.asarray(f, np.float64)))
        l = lsq(nrm, f).l
        rows.append({"index": k, "freqs": f, "m": f.size, "l": l, "G": goodness(l, nrm.N, f.size)})
    best = min(rows, key=lambda r: (r["G"], r["index"]))
    for r in rows:
        r["vuong"] = 0.0 if r is best else vuong(nrm, best["freqs"], r["freqs"])
        r["keep"] = r["vuong"] < vuong_max
    rows.sort(key=lambda r: (r["m"], r["l"], r["index"]))
    return rows


# --------------------------------------- global-local residual periodogram, Sect. 2
@dataclass
class GlobalLocalResult:
    z: np.ndarray           # z*_{1|m,loc}(f_j | f'_loc)
    flags: np.ndarray
    l_base: float           # l_{m,loc}(f'_loc)
    base: np.ndarray        # the base frequencies at that local minimum
    freqs: np.ndarray


def global_local_scan(t, x, w, base_loc, df: float, F: int, refine_steps: int = 8, idx=None) -> GlobalLocalResult:
    """The residual periodogram with a locally re-optimised base model
    (Sect. 2, after eq. zpowrel): for every grid frequency f_j,
        z*_{1|m,loc}(f_j | f'_loc) = (N - 3m - 4)/2 ln(l_{m,loc}(f'_loc) / l_{1|m,loc}(f_j | f'_loc)),
    l_{m,loc}: the base model's chi^2 minimum near f'_loc (Gauss-Newton from
    f'_loc); l_{1|m,loc}(f_j): the minimum of the model with the m base
    frequencies and f_j near f'_loc with f_j held fixed (Gauss-Newton over the
    base frequencies, started at the refined base).  Both refinements make
    1 + refine_steps least-squares fits at most (gn_refine).  Flags as for
    scan(): f_j within MASK_WIDTH / T_eff of a refined base frequency gives
    z := 0 and FLAG_MASKED; a degenerate start gives z := 0 and
    FLAG_SINGULAR; l <= 0 gives z := +inf and FLAG_PERFECT.  The maximum of
    z* over the grid is the global-local statistic z*_{1|m,loc}(*|f'_loc)."""
    nrm = normalize(t, x, w)
    base_loc = np.atleast_1d(np.asarray(base_loc, np.float64))
    m = base_loc.size
    NH = n_dof(nrm.N, m + 1)
    if m:
        rb = gn_refine(nrm, base_loc, refine_steps)
        lb, fb = rb.l, rb.f
    else:
        lb, fb = lsq(nrm, []).l, base_loc
    f = grid(df, F, idx)
    z = np.zeros(f.size)
    flags = np.zeros(f.size, np.uint8)
    for q, fj in enumerate(f):
        if m and np.any(np.abs(fj - fb) * nrm.T_eff < MASK_WIDTH):
            flags[q] = FLAG_MASKED
            continue
        r = gn_refine(nrm, np.concatenate([fb, [fj]]), refine_steps, frozen=(m,))
        if r.flag & FLAG_DEGENERATE:
            flags[q] = FLAG_SINGULAR
        elif r.flag & FLAG_PERFECT:
            z[q], flags[q] = np.inf, FLAG_PERFECT
        else:
            z[q] = 0.5 * NH * math.log(lb / r.l)
    return GlobalLocalResult(z, flags, lb, fb, f)
