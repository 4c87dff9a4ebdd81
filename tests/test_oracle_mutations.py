"""Planted mistakes in the oracle (on the CPU): each plausible slip - a
dropped term, a wrong sign, index or factor, a transposed operand - must make
at least one of the independent pins fail."""
import numpy as np
import pytest

import oracle
import oracle.fredec_ref as R
import tests.test_oracle as P
import tests.test_oracle_phase4 as P4

PINS = [
    P.test_scan_m0_matches_scipy_lombscargle_plain_workload,
    P.test_scan_fft_special_case,
    P.test_golden_dft_worked_example,
    lambda: P.test_lsq_matches_lstsq(3, 2),
    lambda: P.test_scan_base_matches_lstsq(2),
    P.test_scan_invariances,
    lambda: P.test_gradient_matches_central_differences(2),
    P.test_gn_converges_to_truth_on_noiseless_data,
    P.test_phase3_multiplicative_table,
    P.test_tuple_permutation_and_lstsq,
    P.test_goodness_golden,
    lambda: P.test_goodness_is_ratio_of_reduced_chi2(6, [0.021, 0.047]),
    P.test_local_maxima_golden,
    lambda: P4.test_loglik_differences_match_scipy(1),
    P4.test_vuong_identities,
    P4.test_phase4_orders_and_filters,
    P4.test_residual_fap_known_content,
    P4.test_global_local_dominates_fixed_base_scan,
    P4.test_global_local_matches_brute_force_minimisation,
]


def _design_no_2pi(tau, freqs):
    freqs = np.atleast_1d(np.asarray(freqs, np.float64))
    cols = [np.ones_like(tau)]
    for f in freqs:
        cols += [np.cos(f * tau), np.sin(f * tau)]
    return np.stack(cols, axis=1)


def _design_no_constant(tau, freqs):
    freqs = np.atleast_1d(np.asarray(freqs, np.float64))
    cols = [np.zeros_like(tau) + 1e-3 * tau]   # constant column replaced by a slope
    for f in freqs:
        ph = R.TWO_PI * f * tau
        cols += [np.cos(ph), np.sin(ph)]
    return np.stack(cols, axis=1)


def _forward_transposed(L, g):
    n = L.shape[-1]
    a = np.zeros(np.broadcast_shapes(L.shape[:-1], np.shape(g)))
    for i in range(n):
        a[..., i] = (g[..., i] - np.sum(L[..., :i, i] * a[..., :i], axis=-1)) / L[..., i, i]
    return a


def _jacobian_sign(nrm, freqs, theta):
    freqs = np.atleast_1d(np.asarray(freqs, np.float64))
    J = np.empty((nrm.N, freqs.size))
    for k, f in enumerate(freqs):
        ph = R.TWO_PI * f * nrm.tau
        a, b = theta[1 + 2 * k], theta[2 + 2 * k]
        J[:, k] = R.TWO_PI * nrm.tau * (a * np.sin(ph) + b * np.cos(ph))
    return J


_orig_normalize = R.normalize


def _normalize_unweighted_mean(t, x, w):
    n = _orig_normalize(t, x, w)
    xbar = float(np.mean(x))
    d = np.asarray(x) - xbar
    sx = float(np.sqrt(np.sum(n.wt * d * d)))
    return R.Normalized(n.tau, d / sx, n.wt, n.tbar, xbar, sx, n.var_t, n.T_eff)


def _local_maxima_nonstrict_left(z, flags):
    j = np.arange(1, z.size - 1)
    ok = (z[j] >= z[j - 1]) & (z[j] >= z[j + 1]) & (flags[j] == 0)
    return j[ok]


def _local_maxima_no_flags(z, flags):
    j = np.arange(1, z.size - 1)
    ok = (z[j] > z[j - 1]) & (z[j] >= z[j + 1])
    return j[ok]


def _local_maxima_with_ends(z, flags):
    zp = np.concatenate([[-np.inf], z, [-np.inf]])
    j = np.arange(1, zp.size - 1)
    ok = (zp[j] > zp[j - 1]) & (zp[j] >= zp[j + 1]) & (flags[j - 1] == 0)
    return j[ok] - 1


def _loglik_no_scale_term(nrm, freqs):
    fit = R.lsq(nrm, freqs)
    r = nrm.xt - R.design(nrm.tau, freqs) @ fit.theta
    l = float(np.sum(nrm.wt * r * r))
    return -nrm.N * nrm.wt * r * r / (2.0 * l)


def _vuong_no_sqrt_n(nrm, f_ref, f_alt):
    d = R.loglik_terms(nrm, f_ref) - R.loglik_terms(nrm, f_alt)
    om2 = float(np.mean(d * d) - np.mean(d) ** 2)
    return 0.0 if om2 <= 0 else float(np.sum(d) / np.sqrt(om2))


_orig_scan = R.scan


def _residual_scan_without_base(t, x, w, base_f, df, F, idx=None, block=256):
    return _orig_scan(t, x, w, np.zeros(0), df, F, idx=idx, block=block)


_orig_gn_step = R.gn_step


def _gn_step_ignoring_frozen(nrm, freqs, theta, frozen=()):
    return _orig_gn_step(nrm, freqs, theta)


def _gn_step_zero(nrm, freqs, theta, frozen=()):
    return np.zeros(np.atleast_1d(freqs).size), True


MUTATIONS = {
    "global-local periodogram moving the trial frequency": ("gn_step", _gn_step_ignoring_frozen),
    "global-local periodogram without re-optimised base": ("gn_step", _gn_step_zero),
    "log-likelihood without the fitted-scale term": ("loglik_terms", _loglik_no_scale_term),
    "Vuong statistic without sqrt(N)": ("vuong", _vuong_no_sqrt_n),
    "residual periodogram without the solution as base": ("scan", _residual_scan_without_base),
    "phase without 2 pi": ("design", _design_no_2pi),
    "dropped constant column": ("design", _design_no_constant),
    "N_H off by one": ("n_dof", lambda N, n: N - 3 * n),
    "N_H without the 3 per frequency": ("n_dof", lambda N, n: N - 2 * n - 1),
    "transposed L in forward substitution": ("forward_subst", _forward_transposed),
    "wrong sign in the frequency derivative": ("model_jacobian", _jacobian_sign),
    "unweighted mean of x": ("normalize", _normalize_unweighted_mean),
    "popcount off by one": ("popcount", lambda m: bin(m).count("1") + (1 if m > 2 else 0)),
    "goodness with N instead of N - 1": ("goodness", lambda l, N, m: l * N / R.n_dof(N, m)),
    "goodness with m instead of 3m": ("goodness", lambda l, N, m: l * (N - 1) / (N - m - 1)),
    "goodness inverted": ("goodness", lambda l, N, m: l * R.n_dof(N, m) / (N - 1)),
    "peaks non-strict on the left": ("local_maxima", _local_maxima_nonstrict_left),
    "peaks ignoring flags": ("local_maxima", _local_maxima_no_flags),
    "peaks at the grid ends": ("local_maxima", _local_maxima_with_ends),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(R, attr, fn)
    if hasattr(oracle, attr):   # the package re-exports the functions the pins call directly
        monkeypatch.setattr(oracle, attr, fn)
    failures = 0
    for pin in PINS:
        try:
            with np.errstate(all="ignore"):
                pin()
        except Exception:
            failures += 1
    assert failures > 0, f"no pin caught the planted mistake: {name}"
