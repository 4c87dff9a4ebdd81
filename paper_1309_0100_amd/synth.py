"""Seeded synthetic inputs shaped like the paper's workloads.

The paper analyses radial-velocity and variable-star series (Sect. 7); none of
those datasets is used here.  Every generator below draws an unevenly sampled,
weighted series  x_i = sum_k A_k cos(2 pi f_k t_i + phi_k) + eps_i  with
eps_i ~ N(0, sigma_i^2) and w_i = 1/sigma_i^2, which is the data model of
Sect. 2 (multiplicative noise model with known relative weights).

This module holds no arithmetic of the method itself (no normalisation, no
least squares, no statistics): it only produces inputs, so that the oracle and
the GPU path can be fed identical bytes.  Random numbers come from
``numpy.random.Generator(PCG64(SeedSequence(13090100 + c)))`` for workload c.

Workloads (sizes follow the benchmark configurations of this project):

1. ``plain``    N=200 over [0,1000] d with three 50 d gaps, periods 7.3 d and
                41 d, amplitudes 5 and 3, sigma ~ U[1,3]; grid f_j = j*1e-4,
                F = 10^4, base = constant.
2. ``residual`` N=2000 over [0,4000] d, each 365.25 d year observed during its
                first 8 months; 4 sinusoids (P log-U[2,1000] d, A ~ U[1,10]);
                base = constant + the 4 injected frequencies; f_j = 2j/10^6,
                F = 10^6.
3. ``batched``  4096 series, N log-U[50,5000], span log-U[100,10^4] d, 1..5
                injected sinusoids, m ~ U{0..6} base sinusoids, F = 65536 with
                f_j = 2j/65536.
4. ``tuples``   N=1000 over [0,3000] d, 6 sinusoids; 65536 tuples of 1..6
                distinct peaks of the m=0 scan on f_j = j/65536, each offset by
                U[-0.2/T, 0.2/T] with T = 3000 d.
5. ``full``     N=10^4 over 20000 d with nightly (t mod 1 < 1/3) and seasonal
                (8 months on, 4 off) windows; 12 sinusoids, P log-U[1,5000] d,
                sigma ~ U[0.5,5]; f_j = 5j/(4*10^6), F = 4*10^6.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 13090100
YEAR = 365.25


def rng_for(config: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED_BASE + config)))


@dataclass
class Series:
    """One series: times t [d], values x, weights w > 0 (all float64)."""

    t: np.ndarray
    x: np.ndarray
    w: np.ndarray
    true_f: np.ndarray = field(default_factory=lambda: np.zeros(0))
    true_A: np.ndarray = field(default_factory=lambda: np.zeros(0))
    base_f: np.ndarray = field(default_factory=lambda: np.zeros(0))
    df: float = 0.0
    F: int = 0

    @property
    def N(self) -> int:
        return int(self.t.shape[0])


def _signal(rng, t, freqs, amps, sigma):
    phases = rng.uniform(0.0, 2.0 * np.pi, size=len(freqs))
    x = np.zeros_like(t)
    for f, a, p in zip(freqs, amps, phases):
        x += a * np.cos(2.0 * np.pi * f * t + p)
    x += rng.normal(0.0, 1.0, size=t.shape) * sigma
    return x


def _log_uniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))


# --------------------------------------------------------------------------- 1
def plain(N: int = 200, F: int = 10_000, df: float = 1e-4, seed_offset: int = 0) -> Series:
    """Workload 1: N times in [0,1000] d minus three non-overlapping 50 d gaps."""
    rng = rng_for(1 + seed_offset)
    while True:
        starts = np.sort(rng.uniform(0.0, 950.0, size=3))
        if np.all(np.diff(starts) > 50.0):
            break
    t = []
    while len(t) < N:
        c = rng.uniform(0.0, 1000.0)
        if np.any((c >= starts) & (c < starts + 50.0)):
            continue
        t.append(c)
    t = np.sort(np.asarray(t))
    sigma = rng.uniform(1.0, 3.0, size=N)
    freqs = np.array([1.0 / 7.3, 1.0 / 41.0])
    amps = np.array([5.0, 3.0])
    x = _signal(rng, t, freqs, amps, sigma)
    return Series(t, x, 1.0 / sigma**2, freqs, amps, np.zeros(0), df, F)


# --------------------------------------------------------------------------- 2
def _seasonal_times(rng, n, span, on_frac=8.0 / 12.0):
    """n times uniform over the 'on' part of [0, span]: each year observed for
    its first on_frac of the year."""
    out = np.empty(0)
    while out.size < n:
        c = rng.uniform(0.0, span, size=2 * n)
        keep = np.mod(c, YEAR) < on_frac * YEAR
        out = np.concatenate([out, c[keep]])
    return np.sort(out[:n])


def residual(N: int = 2000, F: int = 1_000_000, fmax: float = 2.0, n_sin: int = 4) -> Series:
    """Workload 2: seasonal gaps, 4 sinusoids, base = the 4 injected frequencies."""
    rng = rng_for(2)
    t = _seasonal_times(rng, N, 4000.0)
    sigma = rng.uniform(1.0, 3.0, size=N)
    periods = _log_uniform(rng, 2.0, 1000.0, size=n_sin)
    amps = rng.uniform(1.0, 10.0, size=n_sin)
    freqs = 1.0 / periods
    x = _signal(rng, t, freqs, amps, sigma)
    return Series(t, x, 1.0 / sigma**2, freqs, amps, freqs.copy(), fmax / F, F)


# --------------------------------------------------------------------------- 3
@dataclass
class Batch:
    """CSR batch of series: series s owns samples [soff[s], soff[s+1]) and base
    frequencies [boff[s], boff[s+1])."""

    t: np.ndarray
    x: np.ndarray
    w: np.ndarray
    soff: np.ndarray
    base_f: np.ndarray
    boff: np.ndarray
    df: np.ndarray
    F: np.ndarray

    @property
    def n_series(self) -> int:
        return int(self.soff.shape[0] - 1)

    def series(self, s: int) -> Series:
        a, b = int(self.soff[s]), int(self.soff[s + 1])
        c, d = int(self.boff[s]), int(self.boff[s + 1])
        return Series(self.t[a:b], self.x[a:b], self.w[a:b], base_f=self.base_f[c:d],
                      df=float(self.df[s]), F=int(self.F[s]))


def _resolved_base(rng, injected, m, res):
    """m base frequencies as the method would have detected them: resolved
    from zero and from each other (f >= res, |f - f'| >= res, res = 1.5 / T):
    the injected frequencies that qualify, in order, then log-uniform draws
    in [res, 0.5] c/d (periods of 2 d and longer), rejecting unresolved ones."""
    base = []
    for f in injected:
        if len(base) < m and f >= res and all(abs(f - g) >= res for g in base):
            base.append(f)
    while len(base) < m:
        f = _log_uniform(rng, res, 0.5)
        if all(abs(f - g) >= res for g in base):
            base.append(f)
    return np.asarray(base, np.float64)


def batched(n_series: int = 4096, F: int = 65536, fmax: float = 2.0,
            n_lo: int = 50, n_hi: int = 5000, m_max: int = 6, resolved: bool = True) -> Batch:
    """Workload 3: many independent series of uneven length and base size.
    resolved=True (the benchmark): base frequencies resolved, see
    _resolved_base.  resolved=False: the plain draw, the first min(m, n_inj)
    injected frequencies then log-uniform periods in [2, 1000] d, which can
    put two base frequencies (or one and zero) closer than the series
    resolves, i.e. a singular or nearly singular base."""
    root = np.random.SeedSequence(SEED_BASE + 3)
    ts, xs, ws, bfs = [], [], [], []
    soff = [0]
    boff = [0]
    for child in root.spawn(n_series):
        rng = np.random.Generator(np.random.PCG64(child))
        N = int(round(_log_uniform(rng, n_lo, n_hi)))
        T = _log_uniform(rng, 100.0, 1e4)
        t = np.sort(rng.uniform(0.0, T, size=N))
        n_inj = int(rng.integers(1, 6))
        periods = _log_uniform(rng, 2.0, min(1000.0, T), size=n_inj)
        amps = rng.uniform(1.0, 10.0, size=n_inj)
        sigma = rng.uniform(1.0, 3.0, size=N)
        x = _signal(rng, t, 1.0 / periods, amps, sigma)
        m = int(rng.integers(0, m_max + 1))
        if resolved:
            base = _resolved_base(rng, 1.0 / periods, m, 1.5 / T)
        else:
            base = np.concatenate([1.0 / periods[:min(m, n_inj)],
                                   1.0 / _log_uniform(rng, 2.0, 1000.0, size=max(0, m - n_inj))])
        ts.append(t)
        xs.append(x)
        ws.append(1.0 / sigma**2)
        bfs.append(base)
        soff.append(soff[-1] + N)
        boff.append(boff[-1] + m)
    return Batch(np.concatenate(ts), np.concatenate(xs), np.concatenate(ws),
                 np.asarray(soff, np.int64), np.concatenate(bfs) if bfs else np.zeros(0),
                 np.asarray(boff, np.int64), np.full(n_series, fmax / F), np.full(n_series, F, np.int64))


# --------------------------------------------------------------------------- 4
def tuples_series(N: int = 1000, span: float = 3000.0, F: int = 65536, df: float = 1.0 / 65536) -> Series:
    """Workload 4 series: N times U[0,3000] d, 6 sinusoids."""
    rng = rng_for(4)
    t = np.sort(rng.uniform(0.0, span, size=N))
    periods = _log_uniform(rng, 2.0, 1000.0, size=6)
    amps = rng.uniform(1.0, 10.0, size=6)
    sigma = rng.uniform(1.0, 3.0, size=N)
    x = _signal(rng, t, 1.0 / periods, amps, sigma)
    return Series(t, x, 1.0 / sigma**2, 1.0 / periods, amps, np.zeros(0), df, F)


def tuples_draw(peaks: np.ndarray, n_tuples: int = 65536, n_max: int = 6, span: float = 3000.0,
                rel: float = 0.2):
    """Workload 4 tuples: each tuple takes n ~ U{1..n_max} distinct entries of
    ``peaks`` (frequencies found by a periodogram scan, supplied by the caller)
    and offsets each by U[-rel/span, rel/span].  Returns (freqs, toff) in ragged
    CSR form: tuple k owns freqs[toff[k]:toff[k+1]], sorted ascending."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(SEED_BASE + 40)))
    peaks = np.asarray(peaks, np.float64)
    n_max = min(n_max, peaks.size)
    sizes = rng.integers(1, n_max + 1, size=n_tuples)
    toff = np.zeros(n_tuples + 1, np.int64)
    toff[1:] = np.cumsum(sizes)
    out = np.empty(int(toff[-1]))
    for k in range(n_tuples):
        pick = np.sort(rng.choice(peaks.size, size=int(sizes[k]), replace=False))
        out[toff[k]:toff[k + 1]] = peaks[pick] + rng.uniform(-rel / span, rel / span, size=int(sizes[k]))
    return out, toff


# --------------------------------------------------------------------------- 5
def full(N: int = 10_000, span: float = 20000.0, F: int = 4_000_000, fmax: float = 5.0) -> Series:
    """Workload 5: nightly + seasonal windows, 12 sinusoids."""
    rng = rng_for(5)
    days = np.arange(int(span))
    eligible = days[np.mod(days, YEAR) < (8.0 / 12.0) * YEAR]
    d = rng.choice(eligible, size=N, replace=True).astype(np.float64)
    t = np.sort(d + rng.uniform(0.0, 1.0 / 3.0, size=N))
    periods = _log_uniform(rng, 1.0, 5000.0, size=12)
    amps = rng.uniform(1.0, 10.0, size=12)
    sigma = rng.uniform(0.5, 5.0, size=N)
    x = _signal(rng, t, 1.0 / periods, amps, sigma)
    return Series(t, x, 1.0 / sigma**2, 1.0 / periods, amps, np.zeros(0), fmax / F, F)


# ------------------------------------------------------------------ small cases
def random_series(seed: int, N: int, span: float = 100.0, n_sin: int = 2, noise: float = 1.0) -> Series:
    """Small generic weighted series for unit tests (seeded).  With noise=0
    the values are noiseless sinusoids but the weights stay random."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, seed])))
    t = np.sort(rng.uniform(0.0, span, size=N))
    periods = _log_uniform(rng, 2.0, span / 2.0, size=n_sin)
    amps = rng.uniform(1.0, 5.0, size=n_sin)
    sigma = rng.uniform(0.5, 1.5, size=N)
    x = _signal(rng, t, 1.0 / periods, amps, sigma * noise)
    return Series(t, x, 1.0 / sigma**2, 1.0 / periods, amps)


def two_frequency_alias(N: int = 400, seed: int = 7, noise: float = 0.1) -> Series:
    """Two-frequency alias example in the manner of Sect. 7.1: sinusoids at
    0.9 and 1.1 (cycles per unit time) of equal amplitude, sampled with a
    periodic on/off pattern of period 10 time units (alias frequency 0.1), plus
    Gaussian noise of `noise` times the amplitude.  The exact series of the
    paper is not available; this one only reproduces its structure."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE, 71, seed])))
    t = []
    while len(t) < N:
        c = rng.uniform(0.0, 200.0)
        if np.mod(c, 10.0) < 3.0:
            t.append(c)
    t = np.sort(np.asarray(t))
    freqs = np.array([0.9, 1.1])
    amps = np.array([1.0, 1.0])
    sigma = np.full(N, noise)
    x = _signal(rng, t, freqs, amps, sigma)
    return Series(t, x, 1.0 / sigma**2, freqs, amps)
