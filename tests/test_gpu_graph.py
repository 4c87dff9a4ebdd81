"""The batching form under HIP-graph capture: prepared calls (fredec_*_plan)
whose launches enqueue kernels only, captured with torch.cuda.graph and
replayed several times with eager work in between.  Every replay must equal
the unplanned call bit for bit, and a replay after new data were copied into
the captured input buffers must equal the unplanned call on the new data."""
import numpy as np
import pytest

import oracle as O
from paper_1309_0100_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1309_0100_amd import fredec as F
    return F.Context(0)


def _dev(*arrays):
    import torch
    return [torch.as_tensor(np.ascontiguousarray(a), device="cuda:0") for a in arrays]


def _small_batch(seed, n_series=24):
    """A CSR batch of uneven series (N in [60, 700], m in 0..5, F in [300, 2000])."""
    rng = np.random.default_rng(seed)
    ts, xs, ws, soff, bf, boff, dfs, Fs = [], [], [], [0], [], [0], [], []
    for s in range(n_series):
        N = int(rng.integers(60, 700))
        ser = synth.random_series(seed * 100 + s, N, span=float(rng.uniform(50, 800)), n_sin=3)
        m = int(rng.integers(0, 6))
        base = np.sort(rng.uniform(0.02, 1.5, size=m))
        ts.append(ser.t), xs.append(ser.x), ws.append(ser.w)
        soff.append(soff[-1] + N)
        bf.extend(base)
        boff.append(boff[-1] + m)
        dfs.append(2.0 / 4096)
        Fs.append(int(rng.integers(300, 2000)))
    return (np.concatenate(ts), np.concatenate(xs), np.concatenate(ws), np.array(soff, np.int64),
            np.array(bf, np.float64), np.array(boff, np.int64), np.array(dfs), np.array(Fs, np.int64))


def _same(a, b):
    a, b = a.cpu().numpy(), b.cpu().numpy()
    return np.array_equal(a, b, equal_nan=True) if a.dtype.kind == "f" else np.array_equal(a, b)


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_scan_plan_graph_replays(ctx, prec):
    import torch
    t, x, w, soff, bf, boff, df, F = _small_batch(31 + prec)
    print(f"case: scan plan graph prec={prec} series={soff.size - 1}", flush=True)
    td, xd, wd = _dev(t, x, w)
    ref = ctx.scan(td, xd, wd, soff, bf, boff, df, F, prec)
    plan, out = ctx.scan_plan(soff, bf, boff, df, F, prec)
    plan.run(td, xd, wd, out)
    torch.cuda.synchronize()
    for a, b in zip(out, ref):
        assert _same(a, b)
    # capture (after a warm launch on the capture stream)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run(td, xd, wd, out)
    torch.cuda.current_stream().wait_stream(s)
    with torch.cuda.graph(g):
        plan.run(td, xd, wd, out)
    for rep in range(3):
        for o in out:
            o.fill_(0)
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, ref):
            assert _same(a, b), rep
        # eager work between replays
        other = ctx.scan(td, xd, wd, soff, bf, boff, df, F, 1 - prec)
        torch.cuda.synchronize()
        assert torch.isfinite(other[0]).any()
    # new data into the captured buffers
    t2, x2, w2 = t.copy(), x.copy(), w.copy()
    rng = np.random.default_rng(5)
    x2 = x2 + rng.normal(0, 0.5, size=x2.size)
    w2 = w2 * rng.uniform(0.5, 2.0, size=w2.size)
    td.copy_(torch.as_tensor(t2)), xd.copy_(torch.as_tensor(x2)), wd.copy_(torch.as_tensor(w2))
    g.replay()
    torch.cuda.synchronize()
    ref2 = ctx.scan(td, xd, wd, soff, bf, boff, df, F, prec)
    torch.cuda.synchronize()
    for a, b in zip(out, ref2):
        assert _same(a, b)
    # and against the oracle on one series of the new data
    k = 3
    a, b = soff[k], soff[k + 1]
    r = O.scan(t2[a:b], x2[a:b], w2[a:b], bf[boff[k]:boff[k + 1]], df[k], F[k])
    z = out[0].cpu().numpy()[F[:k].sum():F[:k + 1].sum()]
    good = r.flags == 0
    tol = 1e-9 if prec == 0 else 1e-6
    assert np.max(np.abs(z[good] - r.z[good]) / np.maximum(np.abs(r.z[good]), 1.0)) <= tol
    plan.close()


def test_tuples_plan_graph_replays(ctx):
    import torch
    s = synth.random_series(790, 500, span=400.0, n_sin=3, noise=0.5)
    nrm = O.normalize(s.t, s.x, s.w)
    pool = np.sort(np.concatenate([s.true_f + np.array([0.1, -0.1, 0.05]) / nrm.T_eff, [0.37, 0.61]]))
    print("case: tuples plan graph n=5 R=6", flush=True)
    td, xd, wd = _dev(s.t, s.x, s.w)
    l0 = torch.empty(1, dtype=torch.float64, device="cuda:0")
    ref = ctx.tuples(td, xd, wd, pool, refine_steps=6, l0_out=l0)
    plan, out = ctx.tuples_plan(s.N, pool, refine_steps=6)
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        plan.run(td, xd, wd, out)
    torch.cuda.current_stream().wait_stream(st)
    with torch.cuda.graph(g):
        plan.run(td, xd, wd, out)
    for rep in range(3):
        for o in out:
            o.fill_(0)
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(out[:4], ref):
            assert _same(a, b), rep
        assert _same(out[4], l0)
        ctx.tuples(td, xd, wd, pool[:3])
        torch.cuda.synchronize()
    plan.close()


def test_ascent_plan_graph_replays(ctx):
    import torch
    s = synth.tuples_series()
    r = O.scan(s.t, s.x, s.w, [], s.df, 4096)
    pk = O.local_maxima(r.z, r.flags)
    peaks = r.freqs[pk[np.lexsort((pk, -r.z[pk]))[:12]]]
    f0, toff = synth.tuples_draw(peaks, n_tuples=512)
    print("case: ascent plan graph 512 tuples x 20 steps", flush=True)
    td, xd, wd, f0d = _dev(s.t, s.x, s.w, f0)
    fr, zr, lr, flr = ctx.ascent(td, xd, wd, f0d, toff, steps=20, clamp=0.1)
    plan, out = ctx.ascent_plan(s.N, toff, steps=20, clamp=0.1)
    f = f0d.clone()
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        plan.run(td, xd, wd, f, out)
    torch.cuda.current_stream().wait_stream(st)
    with torch.cuda.graph(g):
        plan.run(td, xd, wd, f, out)
    for rep in range(3):
        f.copy_(f0d)
        g.replay()
        torch.cuda.synchronize()
        assert _same(f, fr), rep
        for a, b in zip(out, (zr, lr, flr)):
            assert _same(a, b), rep
        ctx.grad(td, xd, wd, f0d[:toff[4]], toff[:5])
        torch.cuda.synchronize()
    plan.close()
