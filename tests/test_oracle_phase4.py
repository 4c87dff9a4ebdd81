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
