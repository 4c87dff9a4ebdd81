"""Pins of the oracle's Phase 4 and per-solution report (Sect. 4 "Phase 4",
Sect. 6): the per-sample log-likelihoods against scipy's normal log-density
on the raw data fitted by numpy's least squares, the identities of the Vuong
statistic, and the residual single-frequency FAP on series whose residual
content is known.  The Vuong formula is not printed in the paper, so the
statistic itself is "parity unpinned" against it; these pins fix the
mathematics of the reading taken (plain Vuong statistic, no correction for
the numbers of parameters)."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
from paper_1309_0100_amd import synth


def _raw_loglik(s, freqs):
    """Per-sample Gaussian log-likelihood of the weighted least-squares fit of
    the raw data (x_i ~ N(mu_i, kappa / w_i), kappa by maximum likelihood),
    from numpy.linalg.lstsq and scipy.stats.norm.logpdf."""
    cols = [np.ones_like(s.t)]
    for f in freqs:
        cols += [np.cos(2 * np.pi * f * s.t), np.sin(2 * np.pi * f * s.t)]
    A = np.stack(cols, axis=1)
    sw = np.sqrt(s.w)
    theta, *_ = np.linalg.lstsq(A * sw[:, None], s.x * sw, rcond=None)
    mu = A @ theta
    kappa = np.sum(s.w * (s.x - mu) ** 2) / s.N
    return stats.norm.logpdf(s.x, loc=mu, scale=np.sqrt(kappa / s.w))


@pytest.mark.parametrize("seed", [1, 2])
def test_loglik_differences_match_scipy(seed):
    """The normalised-data log-likelihood differs from the raw-data one by a
    constant per sample (the Jacobian of the x scaling), which cancels in the
    difference of two fits: d_i must agree."""
    s = synth.random_series(300 + seed, 80, span=50.0, n_sin=3, noise=0.5)
    nrm = O.normalize(s.t, s.x, s.w)
    fa, fb = s.true_f[:2], s.true_f[1:]
    d_oracle = O.loglik_terms(nrm, fa) - O.loglik_terms(nrm, fb)
    d_raw = _raw_loglik(s, fa) - _raw_loglik(s, fb)
    assert np.allclose(d_oracle, d_raw, rtol=0, atol=1e-9 * np.max(np.abs(d_raw)))


def test_vuong_identities():
    s = synth.random_series(311, 120, span=60.0, n_sin=3, noise=0.7)
    nrm = O.normalize(s.t, s.x, s.w)
    fa, fb = s.true_f[:2], s.true_f[[0, 2]]
    # sum of d_i = N/2 ln(l_alt / l_ref): the log-likelihood ratio of the two fits
    d = O.loglik_terms(nrm, fa) - O.loglik_terms(nrm, fb)
    la, lb = O.lsq(nrm, fa).l, O.lsq(nrm, fb).l
    assert math.isclose(np.sum(d), 0.5 * nrm.N * math.log(lb / la), rel_tol=1e-9)
    # V from the scipy log-likelihoods
    draw = _raw_loglik(s, fa) - _raw_loglik(s, fb)
    v_ref = np.sum(draw) / (math.sqrt(draw.size) * np.std(draw))
    assert math.isclose(O.vuong(nrm, fa, fb), v_ref, rel_tol=1e-9)
    assert math.isclose(O.vuong(nrm, fb, fa), -v_ref, rel_tol=1e-9)
    assert O.vuong(nrm, fa, fa) == 0.0


def test_phase4_orders_and_filters():
    """Three alternatives on a series with two strong sinusoids: the true pair,
    the true pair plus a spurious frequency, and a pair missing the strongest
    component.  The output is grouped by size and chi^2-ordered, the best
    (smallest G) has V = 0, and the bad fit is filtered (V >= 5)."""
    s = synth.random_series(321, 200, span=100.0, n_sin=2, noise=0.3)
    nrm = O.normalize(s.t, s.x, s.w)
    strong = int(np.argmax(s.true_A))
    weak = 1 - strong
    good = list(s.true_f)
    extra = list(s.true_f) + [0.37]
    bad = [s.true_f[weak], 0.211]
    rows = O.phase4(nrm, [bad, extra, good])
    keys = [(r["m"], r["l"]) for r in rows]
    assert keys == sorted(keys)
    best = min(rows, key=lambda r: r["G"])
    assert best["vuong"] == 0.0 and best["keep"]
    by_index = {r["index"]: r for r in rows}
    assert by_index[0]["vuong"] > 5.0 and not by_index[0]["keep"]
    assert by_index[2]["keep"]
    for r in rows:
        assert math.isclose(r["G"], O.goodness(O.lsq(nrm, r["freqs"]).l, nrm.N, r["m"]), rel_tol=1e-14)


def test_residual_fap_known_content():
    """Residual FAP (Sect. 6): after subtracting both injected sinusoids of a
    low-noise series nothing significant is left (FAP near 1); after
    subtracting only one, the other dominates the residual periodogram (tiny
    FAP, peak at the missing frequency within one resolution element); the
    FAP scales with A~_1 as eq. zFAP says."""
    s = synth.random_series(331, 300, span=200.0, n_sin=2, noise=0.05)
    df, F = 2e-3, 2000
    fap_all, z_all, j_all = O.residual_fap(s.t, s.x, s.w, s.true_f, df, F)
    assert fap_all > 0.01
    fap_one, z_one, j_one = O.residual_fap(s.t, s.x, s.w, s.true_f[:1], df, F)
    assert fap_one < 1e-6 and z_one > z_all
    T = O.normalize(s.t, s.x, s.w).T_eff
    assert abs((j_one + 1) * df - s.true_f[1]) * T < 1.0
    r = O.scan(s.t, s.x, s.w, s.true_f[:1], df, F)
    pk = O.local_maxima(r.z, r.flags)
    assert z_one == r.z[pk].max()
    fap2, _, _ = O.residual_fap(s.t, s.x, s.w, s.true_f[:1], df, F, A1=2.0)
    assert math.isclose(fap2, 2.0 * fap_one, rel_tol=1e-12)
    W = F * df * T
    assert math.isclose(fap_one, W * math.exp(-z_one) * math.sqrt(z_one), rel_tol=1e-12)


# ------------------------------------------- global-local residual periodogram
def test_global_local_without_base_is_the_plain_periodogram():
    """With no base model there is nothing to re-optimise: z*_{1|0,loc} = z_1."""
    s = synth.random_series(341, 120, span=60.0, n_sin=2, noise=0.5)
    df, F = 5e-3, 300
    g = O.global_local_scan(s.t, s.x, s.w, [], df, F)
    r = O.scan(s.t, s.x, s.w, [], df, F)
    assert np.array_equal(g.flags, r.flags)
    assert np.allclose(g.z, r.z, rtol=1e-12, atol=1e-12)


def test_global_local_dominates_fixed_base_scan():
    """Re-optimising the base frequencies can only lower chi^2: z* is at least
    the residual periodogram on the refined base held fixed."""
    s = synth.random_series(342, 150, span=80.0, n_sin=3, noise=0.6)
    df, F = 4e-3, 200
    base = s.true_f[:2] * (1.0 + 1e-3)
    g = O.global_local_scan(s.t, s.x, s.w, base, df, F, refine_steps=6)
    r = O.scan(s.t, s.x, s.w, g.base, df, F)
    ok = (g.flags == 0) & (r.flags == 0)
    assert ok.sum() > 0.9 * F
    assert np.all(g.z[ok] >= r.z[ok] - 1e-9 * np.maximum(r.z[ok], 1.0))
    assert np.max(g.z[ok] - r.z[ok]) > 1e-3      # the re-optimisation does something


def test_global_local_matches_brute_force_minimisation():
    """m = 1: l_{1|1,loc}(f_j) is the minimum over the base frequency f' near
    the refined base of l_2({f', f_j}); a bounded scalar minimiser (scipy) on a
    dense bracket finds the same minimum."""
    from scipy.optimize import minimize_scalar
    s = synth.random_series(343, 100, span=50.0, n_sin=2, noise=0.4)
    nrm = O.normalize(s.t, s.x, s.w)
    T = nrm.T_eff
    base = np.array([s.true_f[0] + 0.05 / T])
    df, F = 6e-3, 120
    idx = np.array([7, 31, 55, 90], np.int64)
    g = O.global_local_scan(s.t, s.x, s.w, base, df, F, refine_steps=30, idx=idx)
    fb = float(g.base[0])
    checked = 0
    for q, j in enumerate(idx):
        fj = (j + 1) * df
        if g.flags[q] or abs(fj - fb) * T < 1.0:
            continue
        grid = np.linspace(fb - 0.3 / T, fb + 0.3 / T, 601)
        ls = [O.lsq(nrm, [u, fj]).l for u in grid]
        u0 = grid[int(np.argmin(ls))]
        res = minimize_scalar(lambda u: O.lsq(nrm, [u, fj]).l, bounds=(u0 - 1e-3 / T, u0 + 1e-3 / T),
                              method="bounded", options={"xatol": 1e-13 / T})
        l_loc = g.l_base * math.exp(-2.0 * g.z[q] / O.n_dof(nrm.N, 2))
        assert abs(l_loc - res.fun) <= 1e-9 * res.fun, (j, l_loc, res.fun)
        checked += 1
    assert checked >= 3
