"""Pins of the FP64 oracle against facts that do not come from the oracle:
library routines solving the same definition by other means (lstsq, scipy's
floating-mean Lomb-Scargle, numpy's FFT), closed forms, invariants of the
definitions, finite differences and counts.  CPU only."""
import json
import math
import os

import numpy as np
import pytest
import scipy.signal

import oracle as O
from paper_1309_0100_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _series(seed=1, N=60, span=100.0, n_sin=2, noise=1.0):
    return synth.random_series(seed, N, span=span, n_sin=n_sin, noise=noise)


def lstsq_l(t, x, w, freqs):
    """Weighted least-squares residual via an SVD solver, on the raw data;
    the residual of the constant model is the normaliser."""
    sw = np.sqrt(w)

    def resid(fs):
        cols = [np.ones_like(t)]
        for f in fs:
            cols += [np.cos(2 * np.pi * f * t), np.sin(2 * np.pi * f * t)]
        A = np.stack(cols, 1) * sw[:, None]
        b = x * sw
        th, *_ = np.linalg.lstsq(A, b, rcond=None)
        r = b - A @ th
        return float(r @ r)

    return resid(freqs) / resid([])


# ------------------------------------------------------------------ eq. idn
def test_normalisation_identities():
    s = _series(3, 80)
    n = O.normalize(s.t, s.x, s.w)
    assert abs(n.wt.sum() - 1) < 1e-15
    assert abs(np.sum(n.wt * n.xt)) < 1e-14
    assert abs(np.sum(n.wt * n.xt ** 2) - 1) < 1e-14
    assert abs(np.sum(n.wt * n.tau)) < 1e-12
    assert abs(n.T_eff - math.sqrt(4 * math.pi * np.average((s.t - np.average(s.t, weights=s.w)) ** 2, weights=s.w))) < 1e-9
    for om in [0.1, 1.7, 13.0]:
        c, sn = np.cos(om * n.tau), np.sin(om * n.tau)
        assert abs(np.sum(n.wt * c * c) + np.sum(n.wt * sn * sn) - 1) < 1e-14


def test_normalize_rejects_bad_input():
    s = _series(3, 20)
    with pytest.raises(ValueError):
        O.normalize(s.t, s.x, np.where(np.arange(20) == 3, 0.0, s.w))
    with pytest.raises(ValueError):
        O.normalize(s.t, np.ones(20), s.w)
    with pytest.raises(ValueError):
        O.normalize(np.full(20, 2.0), s.x, s.w)
    with pytest.raises(ValueError):
        O.normalize(s.t, np.where(np.arange(20) == 1, np.nan, s.x), s.w)


# ------------------------------------------------------------- Cholesky/lsq
def test_cholesky_matches_numpy_and_flags_singular():
    rng = np.random.default_rng(5)
    A = rng.normal(size=(7, 9, 9))
    Q = A @ np.transpose(A, (0, 2, 1)) + 0.1 * np.eye(9)
    L, ok = O.cholesky_checked(Q)
    assert ok.all()
    assert np.allclose(L, np.linalg.cholesky(Q), rtol=1e-12, atol=1e-12)
    B = rng.normal(size=(9, 4))
    S = B @ B.T                        # rank 4
    _, ok = O.cholesky_checked(S)
    assert not ok


@pytest.mark.parametrize("seed,n", [(1, 0), (2, 1), (3, 2), (4, 3), (5, 5)])
def test_lsq_matches_lstsq(seed, n):
    s = _series(seed, 50)
    rng = np.random.default_rng(seed)
    freqs = rng.uniform(0.01, 0.8, size=n)
    nrm = O.normalize(s.t, s.x, s.w)
    fit = O.lsq(nrm, freqs)
    assert fit.ok
    assert abs(fit.l - lstsq_l(s.t, s.x, s.w, freqs)) < 1e-12
    # theta* reproduces the residual l = <(x - Phi theta)^2>
    r = nrm.xt - O.design(nrm.tau, freqs) @ fit.theta
    assert abs(np.sum(nrm.wt * r * r) - fit.l) < 1e-13


# -------------------------------------------------------- scan, m = 0 pins
def zk09_power(t, y, w, f):
    """Generalised Lomb-Scargle power with floating mean (Zechmeister &
    Kuerster 2009, eqs. 5-20), normalised weights."""
    w = w / w.sum()
    om = 2 * np.pi * f
    c, s = np.cos(om * t), np.sin(om * t)
    Y, C, S = w @ y, w @ c, w @ s
    YY = w @ (y * y) - Y * Y
    YC = w @ (y * c) - Y * C
    YS = w @ (y * s) - Y * S
    CC = w @ (c * c) - C * C
    SS = w @ (s * s) - S * S
    CS = w @ (c * s) - C * S
    D = CC * SS - CS * CS
    return (SS * YC * YC + CC * YS * YS - 2 * CS * YC * YS) / (YY * D)


def test_scan_m0_matches_scipy_lombscargle_plain_workload():
    s = synth.plain()
    r = O.scan(s.t, s.x, s.w, [], s.df, s.F)
    p = scipy.signal.lombscargle(s.t, s.x, 2 * np.pi * r.freqs, normalize=True, weights=s.w,
                                 floating_mean=True)
    z_ref = -(s.N - 4) / 2 * np.log1p(-p)
    err = np.abs(z_ref - r.z) / np.maximum(np.abs(z_ref), 1)
    assert err.max() < 1e-10
    assert not r.flags.any()


def test_scan_m0_matches_zk09_closed_form():
    s = _series(11, 40)
    fidx = np.arange(0, 3000, 37)
    r = O.scan(s.t, s.x, s.w, [], 2e-4, 3000, idx=fidx)
    p = np.array([zk09_power(s.t, s.x, s.w, f) for f in r.freqs])
    z_ref = -(s.N - 4) / 2 * np.log1p(-p)
    assert np.max(np.abs(z_ref - r.z) / np.maximum(z_ref, 1)) < 1e-10


@pytest.mark.parametrize("m", [1, 2, 4])
def test_scan_base_matches_lstsq(m):
    s = _series(20 + m, 70, n_sin=3)
    rng = np.random.default_rng(m)
    base = rng.uniform(0.02, 0.9, size=m)
    idx = rng.integers(0, 4000, size=25)
    r = O.scan(s.t, s.x, s.w, base, 2.5e-4, 4000, idx=idx)
    lm = lstsq_l(s.t, s.x, s.w, base)
    assert abs(r.l_base - lm) < 1e-12
    for f, z, fl in zip(r.freqs, r.z, r.flags):
        if fl:
            continue
        l1 = lstsq_l(s.t, s.x, s.w, list(base) + [f])
        zr = (s.N - 3 * m - 4) / 2 * math.log(lm / l1)
        assert abs(z - zr) <= 1e-9 * max(zr, 1)


def test_scan_fft_special_case():
    """Evenly sampled, equal weights, Fourier frequencies: Q is diagonal and
    l_{m+1} = l_m - 2|X_k|^2 / (N^2 <x~^2>), X = FFT of the centred data."""
    N = 64
    rng = np.random.default_rng(9)
    t = np.arange(N, dtype=float)
    x = rng.normal(size=N) + 2 * np.cos(2 * np.pi * 5 * t / N + 0.4)
    w = np.ones(N)
    X = np.fft.fft(x - x.mean())
    var = np.mean((x - x.mean()) ** 2)
    P = 2 * np.abs(X) ** 2 / (N * N * var)             # explained fraction per k
    r0 = O.scan(t, x, w, [], 1.0 / N, N // 2 - 1)
    k = np.arange(1, N // 2)
    assert np.allclose(r0.z, (N - 4) / 2 * np.log(1 / (1 - P[k])), rtol=1e-10, atol=1e-11)
    r1 = O.scan(t, x, w, [5.0 / N], 1.0 / N, N // 2 - 1)
    lm = 1 - P[5]
    keep = r1.flags == 0
    exp = (N - 7) / 2 * np.log(lm / (lm - P[k][keep]))
    assert r1.flags[4] == O.FLAG_MASKED and keep.sum() == N // 2 - 2
    assert np.allclose(r1.z[keep], exp, rtol=1e-10, atol=1e-11)
    assert abs(r1.l_base - lm) < 1e-13


def _golden_val(expr):
    return float(eval(expr, {"ln": math.log}))


def test_golden_dft_worked_example():
    with open(os.path.join(GOLDEN, "dft_worked.json")) as fh:
        g = json.load(fh)
    t = np.asarray(g["t"], float)
    w = np.asarray(g["w"], float)
    x = np.zeros_like(t)
    for amp, kind, k in g["components"]:
        ph = 2 * np.pi * k * t / g["N"]
        x += amp * (np.cos(ph) if kind == "cos" else np.sin(ph))
    r0 = O.scan(t, x, w, [], g["df"], g["F"])
    for z, e in zip(r0.z, g["scan_m0"]["z"]):
        assert abs(z - _golden_val(e)) < 1e-12
    r1 = O.scan(t, x, w, [2.0 / 12.0], g["df"], g["F"])
    for z, fl, e in zip(r1.z, r1.flags, g["scan_m1_base_2"]["z"]):
        if e == "masked":
            assert fl == O.FLAG_MASKED and z == 0
        else:
            assert fl == 0 and abs(z - _golden_val(e)) < 1e-12
    nrm = O.normalize(t, x, w)
    for ks, e in g["tuples"]["cases"]:
        z, l, th, flag = O.tuple_fit(nrm, np.asarray(ks) / 12.0)
        assert flag == 0 and abs(z - _golden_val(e)) < 1e-12


def test_goodness_golden():
    """G of Sect. 6 (item 2) at the hand-derived l values of the worked DFT
    example, and the same G from the oracle's own least-squares fit."""
    with open(os.path.join(GOLDEN, "dft_worked.json")) as fh:
        g = json.load(fh)
    N = g["N"]
    t = np.asarray(g["t"], float)
    x = np.zeros_like(t)
    for amp, kind, k in g["components"]:
        ph = 2 * np.pi * k * t / N
        x += amp * (np.cos(ph) if kind == "cos" else np.sin(ph))
    nrm = O.normalize(t, x, np.asarray(g["w"], float))
    for ks, l_expr, G_expr in g["goodness"]["cases"]:
        m = len(ks)
        G = _golden_val(G_expr)
        assert abs(O.goodness(_golden_val(l_expr), N, m) - G) < 1e-15
        assert abs(O.goodness(O.lsq(nrm, np.asarray(ks) / N).l, N, m) - G) < 1e-13


@pytest.mark.parametrize("seed,freqs", [(5, [0.013]), (6, [0.021, 0.047]), (7, [0.011, 0.03, 0.071])])
def test_goodness_is_ratio_of_reduced_chi2(seed, freqs):
    """Sect. 6: G is the ratio of the reduced chi^2 of the best fit of H_m to
    the reduced chi^2 of H_0 (the weighted variance of the raw x with N - 1
    degrees of freedom) - computed here on the raw data by an SVD solver."""
    s = _series(seed, 90, span=300.0, n_sin=2)
    sw = np.sqrt(s.w)

    def chi2(fs):
        cols = [np.ones_like(s.t)]
        for f in fs:
            cols += [np.cos(2 * np.pi * f * s.t), np.sin(2 * np.pi * f * s.t)]
        A = np.stack(cols, 1) * sw[:, None]
        th, *_ = np.linalg.lstsq(A, s.x * sw, rcond=None)
        r = s.x * sw - A @ th
        return float(r @ r)

    m = len(freqs)
    G_ref = (chi2(freqs) / (s.N - 3 * m - 1)) / (chi2([]) / (s.N - 1))
    l = O.lsq(O.normalize(s.t, s.x, s.w), freqs).l
    assert abs(O.goodness(l, s.N, m) - G_ref) < 1e-12 * G_ref


def test_local_maxima_golden():
    """The peak rule of Phase 1 on a hand-made array with plateaus, a flagged
    point and maxima at both ends."""
    with open(os.path.join(GOLDEN, "local_maxima.json")) as fh:
        g = json.load(fh)
    z = np.asarray(g["z"], float)
    fl = np.asarray(g["flags"], np.uint8)
    assert list(O.local_maxima(z, fl)) == g["peaks"]
    # without the flag the flagged maximum is a peak too
    assert list(O.local_maxima(z, np.zeros_like(fl))) == sorted(g["peaks"] + [9])


# ------------------------------------------------------------- invariants
def _scan_small(t, x, w, base=(), df=3e-4, F=2500, idx=None):
    return O.scan(t, x, w, list(base), df, F, idx=idx)


def test_scan_invariances():
    s = _series(31, 90, n_sin=3)
    base = [s.true_f[0]]
    idx = np.arange(0, 2500, 7)
    ref = _scan_small(s.t, s.x, s.w, base, idx=idx)
    keep = ref.flags == 0
    assert (ref.z[keep] >= 0).all()

    def close(r):
        assert np.array_equal(r.flags, ref.flags)
        assert np.allclose(r.z[keep], ref.z[keep], rtol=1e-9, atol=1e-9)

    close(_scan_small(s.t + 1234.5, s.x, s.w, base, idx=idx))          # time shift
    close(_scan_small(s.t, -3.0 * s.x + 17.0, s.w, base, idx=idx))     # affine x
    close(_scan_small(s.t, s.x, 7.5 * s.w, base, idx=idx))             # weight scale
    p = np.random.default_rng(1).permutation(s.N)
    close(_scan_small(s.t[p], s.x[p], s.w[p], base, idx=idx))          # permutation
    close(_scan_small(s.t, s.x, s.w, [-base[0]], df=-3e-4, idx=idx))   # f -> -f
    lam = 3.7
    close(_scan_small(s.t * lam, s.x, s.w, [base[0] / lam], df=3e-4 / lam, idx=idx))


def test_scan_nesting_monotone_and_single_freq_consistency():
    s = _series(41, 70)
    nrm = O.normalize(s.t, s.x, s.w)
    r = O.scan(s.t, s.x, s.w, [], 3e-4, 2000, idx=np.arange(0, 2000, 50))
    for f, z in zip(r.freqs, r.z):
        zt, l, _, flag = O.tuple_fit(nrm, [f])
        assert flag == 0 and abs(zt - z) < 1e-10 * max(z, 1)
        assert z >= 0


def test_noiseless_recovery():
    s = synth.random_series(51, 300, span=500.0, n_sin=2, noise=0.0)
    df, F = 1e-4, 6000
    r = O.scan(s.t, s.x, s.w, [], df, F)
    strongest = s.true_f[np.argmax(s.true_A)]
    j = int(np.argmax(r.z))
    assert abs(r.freqs[j] - strongest) <= df * 1.0001
    r2 = O.scan(s.t, s.x, s.w, [r.freqs[j]], df, F)
    other = s.true_f[np.argmin(s.true_A)]
    j2 = int(np.argmax(r2.z))
    assert abs(r2.freqs[j2] - other) <= df * 1.0001


# ---------------------------------------------------------------- tuples
def test_tuple_permutation_and_lstsq():
    s = _series(61, 80, n_sin=3)
    nrm = O.normalize(s.t, s.x, s.w)
    f = np.array([0.05, 0.31, 0.47])
    z1, l1, _, _ = O.tuple_fit(nrm, f)
    z2, l2, _, _ = O.tuple_fit(nrm, f[::-1])
    assert abs(z1 - z2) < 1e-10 * z1
    assert abs(l1 - lstsq_l(s.t, s.x, s.w, f)) < 1e-12
    assert z1 == pytest.approx((s.N - 10) / 2 * math.log(1 / l1), rel=1e-14)


def test_tuple_degenerate_merged_frequencies():
    s = _series(62, 80)
    nrm = O.normalize(s.t, s.x, s.w)
    z, l, th, flag = O.tuple_fit(nrm, [0.2, 0.2 + 0.01 / nrm.T_eff])
    assert flag == O.FLAG_DEGENERATE and z == -np.inf


@pytest.mark.parametrize("n", [1, 2, 4])
def test_gradient_matches_central_differences(n):
    s = _series(70 + n, 120, n_sin=3)
    nrm = O.normalize(s.t, s.x, s.w)
    rng = np.random.default_rng(n)
    f = np.sort(rng.uniform(0.02, 0.9, size=n))
    z, l, g, h = O.tuple_grad(nrm, f)
    hstep = 1e-5 / nrm.T_eff
    for k in range(n):
        fp, fm = f.copy(), f.copy()
        fp[k] += hstep
        fm[k] -= hstep
        fd = (O.tuple_fit(nrm, fp)[0] - O.tuple_fit(nrm, fm)[0]) / (2 * hstep)
        assert abs(fd - g[k]) <= 1e-7 * max(abs(g[k]), 1.0 * nrm.T_eff)
    assert np.all(h > 0)


def test_gn_converges_to_truth_on_noiseless_data():
    s = synth.random_series(81, 200, span=300.0, n_sin=3, noise=0.0)
    nrm = O.normalize(s.t, s.x, s.w)
    f0 = s.true_f + np.array([0.15, -0.1, 0.05]) / nrm.T_eff
    r = O.gn_refine(nrm, f0, steps=30)
    assert r.converged and r.flag == 0
    assert np.max(np.abs(np.sort(r.f) - np.sort(s.true_f))) * nrm.T_eff < 1e-8
    assert r.l < 1e-12                      # rounding floor of l = D - a.a


def test_gn_fixed_point_is_stationary_and_matches_ascent():
    s = _series(82, 150, span=200.0, n_sin=2)
    nrm = O.normalize(s.t, s.x, s.w)
    f0 = s.true_f + np.array([0.1, -0.12]) / nrm.T_eff
    r = O.gn_refine(nrm, f0, steps=40)
    assert r.converged
    z, l, g, h = O.tuple_grad(nrm, r.f)
    assert np.max(np.abs(g / h)) * nrm.T_eff < 1e-8          # grad z = 0
    assert r.l <= O.tuple_fit(nrm, f0)[1]
    fa, za, la = O.ascent(nrm, f0, steps=400, clamp=0.1)
    assert np.max(np.abs(fa - r.f)) * nrm.T_eff < 1e-6
    assert abs(za - r.z) < 1e-8 * r.z


# ---------------------------------------------------------- FAP, Phase 3
def test_zcrit_solves_fap_equation():
    W = 1000.0
    for d in (1, 2, 3, 6):
        z = O.zcrit(d, W, 0.05)
        assert z > 1.5 * d - 1
        fap = W ** d * math.exp(-z) * z ** (1.5 * d - 1)
        assert fap == pytest.approx(0.05, rel=1e-12)
    assert O.zcrit(1, W, 0.05) > O.zcrit(1, W, 0.1)


@pytest.mark.parametrize("n", [1, 3, 5, 7])
def test_phase3_counts_and_no_nesting(n):
    rng = np.random.default_rng(n)
    ltab = np.concatenate([[1.0], rng.uniform(0.05, 1.0, size=(1 << n) - 1)])
    surv, maximal, tests = O.phase3(ltab, n, 500, O.zcrit_table(n, 100.0, 0.05))
    assert tests == 3 ** n - 2 ** n
    for a in maximal:
        assert surv[a]
        for b in maximal:
            if a != b:
                assert (a & b) != a and (a & b) != b


def test_phase3_multiplicative_table():
    """l(S) = prod_{k in S} q_k: strong components (q = 0.5) and weak ones
    (q = 0.999) with N = 1000: z_{S|S'} = N_H/2 * sum_{S\\S'} -ln q_k, so the
    survivors are exactly the non-empty subsets of the strong set, and the
    only maximal one is the strong set itself."""
    n = 6
    q = np.array([0.5, 0.999, 0.5, 0.999, 0.5, 0.999])
    ltab = np.array([np.prod(q[[k for k in range(n) if S >> k & 1]]) for S in range(1 << n)])
    surv, maximal, _ = O.phase3(ltab, n, 1000, O.zcrit_table(n, 300.0, 0.05))
    strong = 0b010101
    for S in range(1, 1 << n):
        assert surv[S] == ((S & ~strong) == 0)
    assert list(maximal) == [strong]


@pytest.mark.parametrize("n", [1, 2, 4, 6])
def test_survive_table_equals_per_subset_rule(n):
    """The whole-table form of the Phase 3 rule gives, subset by subset, what
    the per-subset rule gives (random tables with some non-finite entries and
    thresholds large enough that both outcomes occur)."""
    rng = np.random.default_rng(40 + n)
    ltab = np.concatenate([[1.0], rng.uniform(0.2, 1.0, size=(1 << n) - 1)])
    ltab[rng.integers(1, 1 << n, size=max(1, n // 2))] = np.nan
    zc = O.zcrit_table(n, 50.0, 0.05)
    tab = O.survive_table(ltab, n, 80, zc)
    for S in range(1, 1 << n):
        assert bool(tab[S]) == O.survives(ltab, S, 80, zc), S
    assert not tab[0]
    surv, maximal, _ = O.phase3(ltab, n, 80, zc)
    assert np.array_equal(surv, tab)
    assert sorted(int(S) for S in maximal) == O.maximal_sets(tab, n)


def test_survive_table_multiplicative():
    """Multiplicative table of the strong/weak components (see above) through
    the whole-table rule: survivors = non-empty subsets of the strong set."""
    n = 8
    q = np.where(np.arange(n) % 3 == 0, 0.5, 0.999)
    ltab = np.array([np.prod(q[[k for k in range(n) if S >> k & 1]]) for S in range(1 << n)])
    tab = O.survive_table(ltab, n, 1000, O.zcrit_table(n, 300.0, 0.05))
    strong = sum(1 << k for k in range(n) if k % 3 == 0)
    for S in range(1 << n):
        assert tab[S] == (S != 0 and (S & ~strong) == 0)
    assert O.maximal_sets(tab, n) == [strong]


def test_supersets_enumeration():
    n = 7
    for R in [0, 1, 0b1010, 0b1111111]:
        sup = O.supersets(R, n)
        assert sup.size == 1 << (n - O.popcount(R))
        assert len(set(sup.tolist())) == sup.size
        assert all((int(S) & R) == R and 0 <= S < (1 << n) for S in sup)


def test_phase1_noiseless_pool_contains_injected():
    s = synth.random_series(91, 400, span=400.0, n_sin=3, noise=0.05)
    df, F = 1e-4, 5000
    res = O.phase1(s.t, s.x, s.w, df, F)
    T = O.normalize(s.t, s.x, s.w).T_eff
    for f in s.true_f:                 # within the frequency resolution 1/T_eff
        assert np.min(np.abs(res.pool - f)) * T <= 0.5
    assert np.all(np.diff(res.pool) > 0)
    capped = O.phase1(s.t, s.x, s.w, df, F, pool_cap=2)
    assert capped.pool.size == 2 and capped.truncated == res.pool.size - 2


def test_phase1_rejects_inconsistent_thresholds():
    s = _series(92, 50)
    with pytest.raises(ValueError):
        O.phase1(s.t, s.x, s.w, 1e-3, 100, fap0=0.2, fap1=0.1)


def test_scan_trial_pivot_matches_schur_complement():
    """The per-frequency conditioning reported by the scan (smaller relative
    Cholesky pivot of the two trial columns) equals the Schur complements
    1 / (Q_jj (Q^-1)_jj) of those columns computed by matrix inversion, and
    collapses as f T_eff -> 0 where cos(2 pi f t) approaches the constant."""
    s = synth.random_series(811, 120, span=300.0, n_sin=2)
    base = np.array([0.07, 0.31])
    idx = np.array([0, 3, 40, 200])
    df = 2e-4
    r = O.scan(s.t, s.x, s.w, base, df, 1000, idx=idx)
    nrm = O.normalize(s.t, s.x, s.w)
    for k, j in enumerate(idx):
        Phi = O.design(nrm.tau, np.concatenate([base, [(j + 1) * df]]))
        Q = (Phi * nrm.wt[:, None]).T @ Phi
        n = Q.shape[0]
        last = 1.0 / (np.linalg.inv(Q)[n - 1, n - 1] * Q[n - 1, n - 1])
        Q2 = Q[:n - 1, :n - 1]
        second = 1.0 / (np.linalg.inv(Q2)[n - 2, n - 2] * Q2[n - 2, n - 2])
        assert abs(r.rho[k] - min(last, second)) <= 1e-6 * min(last, second) + 1e-14
    assert r.rho[0] < 1e-3 * r.rho[-1]
