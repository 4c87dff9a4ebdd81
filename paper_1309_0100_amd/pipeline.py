"""The FREDEC pipeline (Sect. 4) composed from libfredec calls:

Phase 1  fredec_phase1   residual scans building the candidate pool
Phase 2  fredec_tuples   l_{m,loc} of every subset of the pool (Gauss-Newton refined)
Phase 3  fredec_cascade  relative tests, surviving inclusion-maximal subsets, G
Phase 4  fredec_grad + fredec_vuong   chi^2 order and Vuong statistics against
         the best fit (Sect. 4, Sect. 6)
Report   fredec_residual_fap  residual single-frequency FAP of each solution (Sect. 6)

Marshalling only: every statistic is computed by the library.  The result
lists the alternative solutions sorted by size and goodness of fit G, as
in Sect. 6.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fredec


@dataclass
class Solution:
    mask: int
    freqs: np.ndarray       # refined frequencies, ascending
    G: float                # l (N - 1) / (N - 3m - 1)
    z: float                # absolute statistic of the tuple
    l: float


@dataclass
class Result:
    pool: np.ndarray
    pool_z: np.ndarray
    base: np.ndarray
    W: float
    n_scans: int
    truncated: int
    solutions: list = field(default_factory=list)
    survive: np.ndarray | None = None
    ltab: np.ndarray | None = None


def run(ctx: "fredec.Context", t, x, w, df: float, F: int, fap0: float = 0.05, fap1: float = 0.1,
        fap2: float = 0.05, A=None, pool_cap: int = 0, refine_steps: int = 8, max_scans: int = 25,
        precision: int = fredec.FP64) -> Result:
    import torch
    if not (fap1 >= fap0 >= fap2 > 0):
        raise ValueError("FAP_1 >= FAP_0 >= FAP_2 > 0 required (Sect. 4.4)")
    A1 = 1.0 if A is None else float(A[1])
    p1 = ctx.phase1(t, x, w, df, F, fap0=fap0, fap1=fap1, A1=A1, pool_cap=pool_cap, max_scans=max_scans,
                    precision=precision)
    res = Result(p1["pool"], p1["pool_z"], p1["base"], p1["W"], p1["n_scans"], p1["truncated"])
    n = res.pool.size
    if n == 0:
        return res
    if n > fredec.MAX_POOL:
        raise ValueError(f"Phase 1 kept {n} candidates, more than the {fredec.MAX_POOL} frequencies a pool can hold "
                         f"(Sect. 5: 25-27 is the method's practical limit); pass pool_cap <= {fredec.MAX_POOL}")
    N = len(t) if not hasattr(t, "numel") else t.numel()
    dev = torch.device("cuda", ctx.device)
    ltab = torch.empty(1 << n, dtype=torch.float64, device=dev)
    l, z, f, fl = ctx.tuples(t, x, w, res.pool, refine_steps=refine_steps, precision=precision,
                             l_out=ltab[1:], l0_out=ltab[0:1])
    zc = fredec.zcrit(res.W, n, fap2, A)
    surv, maxi, G = ctx.cascade(ltab, n, N, zc)
    maxi = maxi.cpu().numpy()
    G = G.cpu().numpy()
    z = z.cpu().numpy()
    f = f.cpu().numpy()
    lt = ltab.cpu().numpy()
    sols = []
    for S in np.flatnonzero(maxi):
        mem = [k for k in range(n) if S >> k & 1]
        sols.append(Solution(int(S), np.sort(f[S - 1][mem]), float(G[S]), float(z[S - 1]), float(lt[S])))
    sols.sort(key=lambda s: (bin(s.mask).count("1"), s.G, s.mask))
    res.solutions = sols
    res.survive = surv.cpu().numpy()
    res.ltab = lt
    return res


@dataclass
class Alternative:
    """One row of the Phase 4 / Sect. 6 output."""
    index: int              # position in the input list
    freqs: np.ndarray       # ascending
    m: int
    l: float                # chi^2 minimum of the normalised data at freqs
    G: float                # l (N - 1) / (N - 3m - 1)
    vuong: float            # Vuong statistic of the smallest-G solution against this one
    keep: bool              # vuong < vuong_max
    fap_residual: float = float("nan")   # FAP of the highest peak left in the residual periodogram
    z_residual: float = float("nan")
    f_residual: float = float("nan")


def phase4(ctx: "fredec.Context", t, x, w, solutions, vuong_max: float = 5.0) -> list:
    """Phase 4 (Sect. 4): the solutions (frequency lists) in chi^2 order within
    each number of frequencies, G (Sect. 6), and the Vuong statistic of the
    smallest-G solution against each, kept while it is below vuong_max."""
    sols = [np.sort(np.atleast_1d(np.asarray(f, np.float64))) for f in solutions]
    if not sols:
        return []
    N = len(t) if not hasattr(t, "numel") else t.numel()
    V, l = ctx.vuong(t, x, w, sols, 0)
    l = l.cpu().numpy()
    G = l * (N - 1) / np.array([N - 3 * f.size - 1 for f in sols], np.float64)
    ref = int(min(range(len(sols)), key=lambda k: (G[k], k)))
    if ref != 0:
        V, l2 = ctx.vuong(t, x, w, sols, ref)
    V = V.cpu().numpy()
    rows = [Alternative(k, f, f.size, float(l[k]), float(G[k]), float(V[k]), bool(V[k] < vuong_max))
            for k, f in enumerate(sols)]
    rows.sort(key=lambda r: (r.m, r.l, r.index))
    return rows


def report(ctx: "fredec.Context", t, x, w, res: Result, df: float, F: int, vuong_max: float = 5.0, A1: float = 1.0,
           precision: int = fredec.FP64) -> list:
    """The per-solution output of Sect. 6 for the solutions of a pipeline run:
    Phase 4 rows with the residual single-frequency FAP of each solution."""
    rows = phase4(ctx, t, x, w, [s.freqs for s in res.solutions], vuong_max)
    if not rows:
        return rows
    fap, zr, jr = ctx.residual_fap(t, x, w, [r.freqs for r in rows], df, F, A1, precision)
    for r, a, b, j in zip(rows, fap, zr, jr):
        r.fap_residual, r.z_residual = float(a), float(b)
        r.f_residual = float((j + 1) * df) if j >= 0 else float("nan")
    return rows

