"""GPU parity of the reduced-precision residual scan (float32 sums against
the base columns, float64 phase reduction, phasors, data column and solves)
against the float64 oracle, for each kernel family of that form: float32
VALU sums (m <= 12), float16 matrix cores on split operands, and the
automatic choice between them (the default).

Bound (relative error err = |z - z_ref| / max(z_ref, 1)): 1e-6 on every grid
frequency that the oracle does not flag.  Grid points whose trial columns lie
nearly in the span of the base model (relative Schur pivot < 0.6: next to a
base frequency, or f T_eff of order 1 and below) and the tops of strong peaks
(l_{m+1} < l_m / 2) are re-scored in float64 by the library and carry flag
bit 6; the rest come from the float32 MFMA sums.
The masking decision uses float64 frequencies only and must match exactly."""
import numpy as np
import pytest

import oracle as O
from paper_1309_0100_amd import synth

pytestmark = pytest.mark.gpu

TOL32 = 1e-6


FORMS = {0: "valu", 2: "f16x3", 3: "auto"}


@pytest.fixture(scope="module", params=list(FORMS), ids=list(FORMS.values()))
def ctx(request):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1309_0100_amd import fredec as F
    c = F.Context(0)
    c.set_tile(F.TILE_SCAN_F32_FORM, 0, request.param)
    c.form = request.param
    print(f"float32 form: {FORMS[request.param]}", flush=True)
    return c


def compare(z, fl, ref, tol=TOL32, label=""):
    z = z.cpu().numpy() if hasattr(z, "cpu") else z
    fl = fl.cpu().numpy() if hasattr(fl, "cpu") else fl
    T = ref.T_eff
    assert np.array_equal(fl & 1, ref.flags & 1), "masking differs"
    base_fl = fl & ~np.uint8(64)
    good = (ref.flags == 0) & (base_fl == 0)
    assert np.array_equal(base_fl, ref.flags), "flags differ"
    e = np.abs(z - ref.z) / np.maximum(np.abs(ref.z), 1.0)
    resc = (fl & 64) != 0
    low = np.abs(ref.freqs) * T < 1.0
    print(f"{label}: max err {e[good].max(initial=0):.3e} over {good.sum()} points; "
          f"float32 points {e[good & ~resc].max(initial=0):.3e} ({(good & ~resc).sum()}), "
          f"re-scored {e[good & resc].max(initial=0):.3e} ({(good & resc).sum()}), "
          f"f*T_eff<1 {e[good & low].max(initial=0):.3e} ({(good & low).sum()})", flush=True)
    assert e[good].max(initial=0.0) <= tol
    return e[good].max(initial=0.0)


def test_fp32_residual_workload_sampled(ctx):
    from paper_1309_0100_amd import fredec as F
    s = synth.residual()
    print("case: fp32 residual N=2000 F=1e6 m=4", flush=True)
    z, fl, lb, st = ctx.scan_series(s.t, s.x, s.w, s.base_f, s.df, s.F, precision=F.FP32)
    z, fl = z.cpu().numpy(), fl.cpu().numpy()
    rng = np.random.default_rng(3)
    idx = [rng.choice(s.F, size=1500, replace=False), np.arange(0, 600, 7)]
    for f in s.base_f:
        j = int(round(f / s.df)) - 1
        idx.append(np.arange(max(0, j - 60), min(s.F, j + 61)))
    idx = np.unique(np.concatenate(idx))
    ref = O.scan(s.t, s.x, s.w, s.base_f, s.df, s.F, idx=idx)
    compare(z[idx], fl[idx], ref, label="residual fp32")


@pytest.mark.parametrize("m,N,F", [(0, 500, 3001), (3, 400, 2500), (7, 600, 2049), (8, 700, 1500),
                                   (12, 500, 1300), (20, 900, 700), (24, 400, 600)])
def test_fp32_base_models(ctx, m, N, F):
    from paper_1309_0100_amd import fredec as Fr
    s = synth.random_series(400 + m, N, span=500.0, n_sin=3)
    rng = np.random.default_rng(m)
    base = np.concatenate([s.true_f, rng.uniform(0.01, 0.7, size=max(0, m - 3))])[:m]
    df = 0.8 / F
    print(f"case: fp32 m={m} N={N} F={F}", flush=True)
    z, fl, lb, st = ctx.scan_series(s.t, s.x, s.w, base, df, F, precision=Fr.FP32)
    ref = O.scan(s.t, s.x, s.w, base, df, F)
    assert int(st.item()) == 0
    assert abs(float(lb.item()) - ref.l_base) < 1e-13
    compare(z, fl, ref, label=f"m={m}")


@pytest.mark.parametrize("m,N,F", [(0, 3000, 700), (3, 17000, 1500), (9, 9001, 2500), (17, 4100, 600)])
def test_fp32_split_scan_few_tiles(ctx, m, N, F):
    """A single scan whose grid gives the split-float16 kernel few
    workgroups is split over sample chunks (raw sums per chunk, added in chunk
    order by a reduction that finishes the points): 2 chunks with a ragged
    last one, 16 chunks of which the last is empty, 8 chunks at two column
    tiles, 4 chunks at three; every grid point against the oracle."""
    from paper_1309_0100_amd import fredec as Fr
    s = synth.random_series(500 + m, N, span=800.0, n_sin=3)
    rng = np.random.default_rng(50 + m)
    base = np.concatenate([s.true_f, rng.uniform(0.01, 0.7, size=max(0, m - 3))])[:m]
    df = 1.5 / F
    print(f"case: fp32 split scan m={m} N={N} F={F}", flush=True)
    z, fl, lb, st = ctx.scan_series(s.t, s.x, s.w, base, df, F, precision=Fr.FP32)
    ref = O.scan(s.t, s.x, s.w, base, df, F)
    assert int(st.item()) == 0
    assert abs(float(lb.item()) - ref.l_base) < 1e-13
    compare(z, fl, ref, label=f"split m={m}")


def test_fp32_batched_uneven(ctx):
    from paper_1309_0100_amd import fredec as Fr
    specs = [(80, 0, 100), (300, 3, 4097), (120, 1, 513), (640, 9, 1000), (90, 2, 1), (1000, 0, 3000)]
    ts, xs, ws, bs, soff, boff, dfs, Fs = [], [], [], [], [0], [0], [], []
    for k, (N, m, F) in enumerate(specs):
        s = synth.random_series(500 + k, N, span=80.0 + 40 * k, n_sin=2)
        base = np.random.default_rng(k).uniform(0.02, 0.5, size=m)
        ts.append(s.t); xs.append(s.x); ws.append(s.w); bs.append(base)
        soff.append(soff[-1] + N); boff.append(boff[-1] + m)
        dfs.append(1.1 / F); Fs.append(F)
    print("case: fp32 batched", specs, flush=True)
    z, fl, lb, st = ctx.scan(np.concatenate(ts), np.concatenate(xs), np.concatenate(ws), soff,
                             np.concatenate(bs), boff, dfs, Fs, precision=Fr.FP32)
    z, fl = z.cpu().numpy(), fl.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    g = 0
    for k in range(len(specs)):
        ref = O.scan(ts[k], xs[k], ws[k], bs[k], dfs[k], Fs[k])
        compare(z[g:g + Fs[k]], fl[g:g + Fs[k]], ref, label=f"series {k}")
        g += Fs[k]


def test_fp32_tile_settings_and_determinism(ctx):
    """Every frequency-tile setting of the split-float16 kernel gives the
    oracle's statistic within the float32 bound (the float32 phasor tables
    depend on the tile, so settings differ by rounding only), and a repeated
    call gives identical bytes.  Unsupported settings are rejected."""
    from paper_1309_0100_amd import fredec as Fr
    s = synth.random_series(600, 700, n_sin=2)
    base = [0.05, 0.3]
    ref = O.scan(s.t, s.x, s.w, base, 2e-4, 5000)
    ctx.set_tile(Fr.TILE_SCAN_F32_FORM, 0, Fr.F32_FORM_F16X3)
    try:
        outs = []
        for ft in (1, 2, 4, 0):
            print(f"case: split-float16 scan, FT={ft}", flush=True)
            ctx.set_tile(Fr.TILE_SCAN_F16X3, 1, ft)
            z, fl, _, _ = ctx.scan_series(s.t, s.x, s.w, base, 2e-4, 5000, precision=Fr.FP32)
            outs.append(z.cpu().numpy())
            compare(outs[-1], fl.cpu().numpy(), ref, label=f"FT={ft}")
        again = ctx.scan_series(s.t, s.x, s.w, base, 2e-4, 5000, precision=Fr.FP32)[0].cpu().numpy()
        assert again.tobytes() == outs[-1].tobytes()
        for nt, ft in ((1, 3), (2, 4), (3, 2), (5, 1)):
            with pytest.raises(Fr.FredecError):
                ctx.set_tile(Fr.TILE_SCAN_F16X3, nt, ft)
        with pytest.raises(Fr.FredecError):
            ctx.set_tile(Fr.TILE_SCAN_F32_FORM, 0, 1)
    finally:
        ctx.set_tile(Fr.TILE_SCAN_F16X3, 1, 0)
        ctx.set_tile(Fr.TILE_SCAN_F32_FORM, 0, ctx.form)
