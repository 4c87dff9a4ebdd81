"""Parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times: the GPU computes everything, the float64 oracle
checks a sample of the outputs (point by point), and whole-output properties
are checked where the oracle cannot follow at that size."""
import numpy as np
import pytest

import oracle as O
from paper_1309_0100_amd import synth

pytestmark = pytest.mark.gpu

TOL = {0: 1e-9, 1: 1e-6}


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1309_0100_amd import fredec as F
    return F.Context(0)


def _rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1.0)


def _tol(prec, rho):
    """Parity bound per grid point: TOL where the two trial columns are well
    conditioned against the base model (smaller relative Cholesky pivot
    rho >= 1e-5); below that, rounding in any float64 evaluation of the
    statistic (the oracle's included) grows like eps / rho, and so does the
    bound: TOL * 1e-5 / rho.  The case is f T_eff << 1, where the trial
    cosine is nearly the constant column."""
    return TOL[prec] * np.maximum(1.0, 1e-5 / np.maximum(rho, 1e-300))


def _sample_idx(rng, F, z, n_rand=200, n_top=20):
    idx = set(rng.integers(0, F, size=n_rand).tolist())
    idx.update(range(5))
    idx.update(range(F - 5, F))
    finite = np.where(np.isfinite(z), z, -np.inf)
    idx.update(np.argpartition(-finite, n_top)[:n_top].tolist())
    return np.array(sorted(idx), np.int64)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_residual_scan_full_size(ctx, prec):
    """N = 2000, m = 4 base sinusoids, F = 10^6: random grid points, both
    ends, and the 20 highest points (where float32 re-scoring acts)."""
    s = synth.residual()
    print(f"case: residual full size prec={prec}", flush=True)
    z, fl, lb, st = (a.cpu().numpy() for a in ctx.scan_series(s.t, s.x, s.w, s.base_f, s.df, s.F, precision=prec))
    assert st[0] == 0
    idx = _sample_idx(np.random.default_rng(11 + prec), s.F, z)
    r = O.scan(s.t, s.x, s.w, s.base_f, s.df, s.F, idx=idx)
    assert np.array_equal(fl[idx] & ~np.uint8(64), r.flags)
    good = r.flags == 0
    assert good.sum() > 0.9 * idx.size
    err = _rel(z[idx][good], r.z[good])
    bound = _tol(prec, r.rho[good])
    assert np.all(err <= bound), (err.max(), idx[good][np.argmax(err / bound)])
    assert abs(lb[0] - r.l_base) <= 1e-12


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_batched_scan_full_size(ctx, prec):
    """4096 series of uneven N and m, F = 65536 each (2.7e8 outputs): 48
    series checked at 12 grid points each plus their highest point."""
    import torch
    b = synth.batched()
    print(f"case: batched full size prec={prec}", flush=True)
    from paper_1309_0100_amd import fredec as F
    z, fl, lb, st = ctx.scan(b.t, b.x, b.w, b.soff, b.base_f, b.boff, b.df, b.F, precision=prec)
    st = st.cpu().numpy()
    # series whose base model is singular (e.g. a repeated base frequency)
    # must be exactly those the oracle cannot fit
    singular = [s for s in range(b.n_series) if not O.lsq(O.normalize(b.series(s).t, b.series(s).x, b.series(s).w),
                                                           b.series(s).base_f).ok]
    assert np.flatnonzero(st != 0).tolist() == singular
    assert np.all(st[singular] == F.ESINGULAR)
    goff = np.concatenate([[0], np.cumsum(b.F)])
    rng = np.random.default_rng(21 + prec)
    ok_series = np.setdiff1d(np.arange(b.n_series), singular)
    for sidx in np.sort(rng.choice(ok_series, size=48, replace=False)):
        ser = b.series(int(sidx))
        zs = z[goff[sidx]:goff[sidx + 1]]
        top = int(torch.argmax(torch.nan_to_num(zs, nan=-1.0)).item())
        idx = np.unique(np.concatenate([rng.integers(0, ser.F, size=12), [0, ser.F - 1, top]])).astype(np.int64)
        sel = torch.as_tensor(idx, device=zs.device)
        zg = zs.index_select(0, sel).cpu().numpy()
        fg = fl[goff[sidx]:goff[sidx + 1]].index_select(0, sel).cpu().numpy()
        r = O.scan(ser.t, ser.x, ser.w, ser.base_f, ser.df, ser.F, idx=idx)
        assert np.array_equal(fg & ~np.uint8(64), r.flags), sidx
        good = r.flags == 0
        if good.any():
            err = _rel(zg[good], r.z[good])
            bound = _tol(prec, r.rho[good])
            assert np.all(err <= bound), (sidx, idx[good][np.argmax(err / bound)], err.max())


def test_tuple_ascent_full_size(ctx):
    """65536 tuples of 1..6 perturbed peaks, N = 1000, 20 ascent steps, as in
    the benchmark; 64 tuples spread over the batch follow the oracle's
    ascent."""
    s = synth.tuples_series()
    z, fl, _, _ = ctx.scan_series(s.t, s.x, s.w, [], s.df, s.F)
    idx, zp = ctx.peaks(z, fl, 0.0)
    top = idx[np.lexsort((idx, -zp))[:12]]
    peaks = (top + 1).astype(np.float64) * s.df
    f0, toff = synth.tuples_draw(peaks, n_tuples=65536)
    print("case: tuple ascent full size", flush=True)
    fa, za, la, fla = (a.cpu().numpy() for a in ctx.ascent(s.t, s.x, s.w, f0, toff, steps=20, clamp=0.1))
    nrm = O.normalize(s.t, s.x, s.w)
    for k in np.linspace(0, toff.size - 2, 64).astype(int):
        fr, zr, lr = O.ascent(nrm, f0[toff[k]:toff[k + 1]], steps=20, clamp=0.1)
        if not np.isfinite(zr):
            assert fla[k] & 8
            continue
        assert np.max(np.abs(fa[toff[k]:toff[k + 1]] - fr)) * nrm.T_eff < 1e-8
        assert _rel(za[k], zr) <= 1e-8


@pytest.fixture(scope="module")
def full_runs(ctx):
    """The full pass (N = 10^4 over 20000 d, F = 4e6, pool cap 16, 65535 subsets
    refined by 8 Gauss-Newton steps, Phase 3) in both precisions."""
    from paper_1309_0100_amd import pipeline
    s = synth.full()
    runs = {}
    for prec in (0, 1):
        print(f"case: full pipeline prec={prec}", flush=True)
        runs[prec] = pipeline.run(ctx, s.t, s.x, s.w, s.df, s.F, pool_cap=16, refine_steps=8, precision=prec)
    return s, runs


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_full_pipeline_full_size(ctx, full_runs, prec):
    """Refined l of sampled subsets against the oracle's Gauss-Newton
    refinement; Phase 3 on the returned l-table against the oracle's survival
    rule and inclusion-maximal sets; solutions ordered by size, then G."""
    from paper_1309_0100_amd import fredec as F
    s, runs = full_runs
    res = runs[prec]
    n = res.pool.size
    assert 1 <= n <= 16 and res.n_scans >= 1
    assert np.all(np.diff(res.pool) > 0) or n == 1
    nrm = O.normalize(s.t, s.x, s.w)
    lt = res.ltab
    assert abs(lt[0] - O.lsq(nrm, []).l) <= 1e-12
    rng = np.random.default_rng(5)
    masks = [1 << k for k in range(min(n, 4))] + [(1 << n) - 1] + rng.integers(1, 1 << n, size=8).tolist()
    for S in masks:
        mem = [k for k in range(n) if S >> k & 1]
        r = O.gn_refine(nrm, res.pool[mem], 8)
        if r.flag:
            assert not np.isfinite(lt[S]) or lt[S] <= 0
            continue
        assert abs(lt[S] - r.l) <= 1e-9 * r.l, (S, lt[S], r.l)
    zc = F.zcrit(res.W, n, 0.05)
    assert np.allclose(zc[1:], O.zcrit_table(n, res.W, 0.05)[1:], rtol=1e-12, atol=0)
    surv_ref = O.survive_table(lt, n, s.N, zc)
    assert np.array_equal(res.survive.astype(bool), surv_ref)
    maximal = O.maximal_sets(surv_ref, n)
    assert sorted(sol.mask for sol in res.solutions) == maximal
    keys = [(bin(sol.mask).count("1"), sol.G, sol.mask) for sol in res.solutions]
    assert keys == sorted(keys)
    for sol in res.solutions:
        assert abs(sol.G - O.goodness(lt[sol.mask], s.N, bin(sol.mask).count("1"))) <= 1e-14 * sol.G


def test_full_pipeline_forms_agree(full_runs):
    """The float32 form takes every decision of the float64 form: same scans,
    base, pool, l-table (Phase 2 is float64 in both), survivors and
    solutions."""
    _, runs = full_runs
    a, b = runs[0], runs[1]
    assert a.n_scans == b.n_scans and a.truncated == b.truncated
    assert np.array_equal(a.base, b.base)
    assert np.array_equal(a.pool, b.pool)
    assert np.allclose(a.pool_z, b.pool_z, rtol=1e-12, atol=0)
    assert np.array_equal(a.ltab, b.ltab, equal_nan=True)
    assert np.array_equal(a.survive, b.survive)
    assert [s.mask for s in a.solutions] == [s.mask for s in b.solutions]


def test_full_pass_fp32_scans_within_bound(ctx, full_runs):
    """Every Phase 1 scan of the full pass (base m = 0 .. 17: the float32
    VALU kernel, the split-float16 kernel at one, two and three column tiles,
    float64 re-scoring) in the float32 form against the float64 form at every
    grid point that neither flags: within the float32 bound 1e-6 (relative to
    max(1, z)); flags other than the re-scoring mark equal."""
    import torch
    from paper_1309_0100_amd import fredec as F
    s, runs = full_runs
    res = runs[0]
    t, x, w = (torch.as_tensor(a, device="cuda") for a in (s.t, s.x, s.w))
    for k in range(res.n_scans):
        base = res.base[:k]
        print(f"case: full pass scan {k} fp32 vs fp64", flush=True)
        z32, f32, _, st32 = ctx.scan_series(t, x, w, base, s.df, s.F, precision=F.FP32)
        z64, f64, _, st64 = ctx.scan_series(t, x, w, base, s.df, s.F, precision=F.FP64)
        assert int(st32.item()) == 0 and int(st64.item()) == 0
        assert torch.equal(f32 & ~64, f64), k
        good = (f64 == 0) & torch.isfinite(z64)
        rel = (z32 - z64).abs() / torch.clamp(z64.abs(), min=1.0)
        assert float(rel[good].max().item()) <= TOL[1], (k, float(rel[good].max().item()))


def test_full_phase1_decisions(ctx, full_runs):
    """Every Phase 1 decision of the full pass checked against the oracle at
    the grid points it rests on: in each scan (base = the SLICK frequencies
    chosen before it) the oracle's z at the GPU's 12 highest peaks and their
    neighbours (values to 1e-9, the peak property, the argmax among them,
    which must be the next SLICK frequency while its z exceeds the FAP_0
    threshold and end the phase otherwise); every pool member is a peak of
    some scan with the recorded z and passes the FAP_1 and half-height rules
    by the oracle's values."""
    import torch
    from paper_1309_0100_amd import fredec as F
    s, runs = full_runs
    res = runs[0]
    nrm = O.normalize(s.t, s.x, s.w)
    W = s.F * s.df * nrm.T_eff
    assert abs(res.W - W) <= 1e-9 * W
    zc0, zc1 = O.zcrit(1, W, 0.05), O.zcrit(1, W, 0.1)
    pool_idx = np.rint(res.pool / s.df).astype(np.int64) - 1
    assert np.array_equal((pool_idx + 1) * s.df, res.pool)
    found = np.zeros(res.pool.size, bool)
    for k in range(res.n_scans):
        base = res.base[:k]
        print(f"case: full phase 1 scan {k}", flush=True)
        z, fl, _, st = ctx.scan_series(s.t, s.x, s.w, base, s.df, s.F, precision=F.FP64)
        assert int(st.item()) == 0
        idx, zp = ctx.peaks(z, fl, 0.0, cap=s.F)
        top = idx[np.lexsort((idx, -zp))[:12]]
        idxset = set(idx.tolist())
        pts = np.unique(np.concatenate([top - 1, top, top + 1, pool_idx]))
        pts = pts[(pts >= 0) & (pts < s.F)]
        sel = torch.as_tensor(pts, device=z.device)
        zg = z.index_select(0, sel).cpu().numpy()
        fg = fl.index_select(0, sel).cpu().numpy()
        r = O.scan(s.t, s.x, s.w, base, s.df, s.F, idx=pts)
        assert np.array_equal(fg, r.flags), k
        good = r.flags == 0
        assert np.all(_rel(zg[good], r.z[good]) <= _tol(0, r.rho[good])), k
        zo = dict(zip(pts.tolist(), r.z.tolist()))
        for j in top:
            assert zo[j] > zo[j - 1] and zo[j] >= zo[j + 1], (k, j)
        jmax = int(top[0])
        assert all(zo[jmax] > zo[int(j)] or (zo[jmax] == zo[int(j)] and jmax < j) for j in top[1:]), k
        if k < res.base.size:
            assert res.base[k] == (jmax + 1) * s.df, k
            assert zo[jmax] > zc0
        else:
            assert zo[jmax] <= zc0
        zg_at = dict(zip(pts.tolist(), zg.tolist()))
        for q, j in enumerate(pool_idx.tolist()):
            if found[q] or j not in idxset:
                continue
            if abs(zg_at[j] - res.pool_z[q]) <= 1e-12 * max(1.0, res.pool_z[q]):
                found[q] = True
                assert _rel(zo[j], res.pool_z[q]) <= 1e-9
                assert zo[j] > zc1 and zo[j] >= 0.5 * zo[jmax] * (1 - 1e-12)
    assert found.all(), res.pool[~found]


def test_phase1_reduced_full_shape_matches_oracle(ctx):
    """Phase 1 and Phase 3 of a reduced series of the full-pass shape (N =
    2000 over 4000 d, F = 2e5 to 5 c/d) against the oracle's own run of both
    phases (tests/golden/phase1_full_reduced.json, written by
    make_phase1_golden.py): the SLICK base, the pool and the number of scans
    bit-exact in both precisions; pool z to 1e-9; the Phase 3 survivors and
    maximal sets on the GPU's fixed-frequency l-table bit-exact."""
    import json
    import os
    from paper_1309_0100_amd import fredec as F
    path = os.path.join(os.path.dirname(__file__), "golden", "phase1_full_reduced.json")
    with open(path) as fh:
        g = json.load(fh)
    c = g["case"]
    s = synth.full(N=c["N"], span=c["span"], F=c["F"], fmax=c["fmax"])
    for prec in (F.FP64, F.FP32):
        print(f"case: reduced full-shape phase 1 prec={prec}", flush=True)
        p1 = ctx.phase1(s.t, s.x, s.w, s.df, s.F, pool_cap=16, precision=prec)
        assert p1["n_scans"] == g["n_scans"] and p1["truncated"] == g["truncated"]
        assert np.array_equal(p1["base"], (np.asarray(g["base_index"]) + 1) * s.df)
        assert np.array_equal(p1["pool"], (np.asarray(g["pool_index"]) + 1) * s.df)
        assert np.all(_rel(p1["pool_z"], np.asarray(g["pool_z"])) <= 1e-9)
        assert abs(p1["W"] - g["W"]) <= 1e-12 * g["W"]
    import torch
    n = len(g["pool"])
    l0 = torch.empty(1, dtype=torch.float64, device="cuda:0")
    l, _, _, fl = ctx.tuples(s.t, s.x, s.w, np.asarray(g["pool"]), refine_steps=0, l0_out=l0)
    lt = np.concatenate([l0.cpu().numpy(), l.cpu().numpy()])
    degenerate = np.concatenate([[False], (fl.cpu().numpy() & F.FLAG_DEGENERATE) != 0])
    for key, ref in g["ltab_sample"].items():
        S = int(key)
        if not np.isfinite(ref):
            assert degenerate[S]
            continue
        assert not degenerate[S] and abs(lt[S] - ref) <= 1e-9 * ref, (S, lt[S], ref)
    zc = F.zcrit(g["W"], n, 0.05)
    surv, maxi, _ = (a.cpu().numpy() for a in ctx.cascade(lt, n, s.N, zc))
    bits = np.unpackbits(np.frombuffer(bytes.fromhex(g["survive_bits"]), np.uint8), bitorder="little")
    assert np.array_equal(surv.astype(np.uint8), bits[:1 << n])
    assert sorted(np.flatnonzero(maxi).tolist()) == g["maximal"]


def test_residual_scan_fp32_peaks(ctx):
    """The float32 form's 50 highest periodogram peaks of the residual scan
    (N = 2000, m = 4, F = 10^6) are the float64 form's, each a peak of the
    oracle's values with z to 1e-6."""
    import torch
    from paper_1309_0100_amd import fredec as F
    s = synth.residual()
    print("case: residual full size fp32 peaks", flush=True)
    tops = {}
    for prec in (F.FP64, F.FP32):
        z, fl, _, _ = ctx.scan_series(s.t, s.x, s.w, s.base_f, s.df, s.F, precision=prec)
        idx, zp = ctx.peaks(z, fl, 0.0, cap=s.F)
        o = np.lexsort((idx, -zp))[:50]
        tops[prec] = (idx[o], zp[o])
    assert np.array_equal(np.sort(tops[F.FP64][0]), np.sort(tops[F.FP32][0]))
    j, z32 = tops[F.FP32]
    pts = np.unique(np.concatenate([j - 1, j, j + 1]))
    r = O.scan(s.t, s.x, s.w, s.base_f, s.df, s.F, idx=pts)
    zo = dict(zip(pts.tolist(), r.z.tolist()))
    for jj, zz in zip(j.tolist(), z32.tolist()):
        assert zo[jj] > zo[jj - 1] and zo[jj] >= zo[jj + 1]
        assert abs(zz - zo[jj]) / max(1.0, zo[jj]) <= 1e-6
