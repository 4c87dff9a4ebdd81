"""The differentiation form: z(f) of ragged tuples as a torch.autograd
function whose backward pass is the library's adjoint gradient, checked
against the float64 oracle's analytic gradient, central differences of the
GPU's own z, and the library's fixed-step ascent."""
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


def _case(seed=760, N=800, n_tuples=48):
    s = synth.random_series(seed, N, span=400.0, n_sin=4)
    nrm = O.normalize(s.t, s.x, s.w)
    rng = np.random.default_rng(seed)
    pool = np.concatenate([s.true_f, rng.uniform(0.05, 0.9, size=4)])
    sizes = rng.integers(1, 6, size=n_tuples)
    toff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    f = np.concatenate([np.sort(rng.choice(pool, size=k, replace=False)) + rng.uniform(-0.2, 0.2, size=k) / nrm.T_eff
                        for k in sizes])
    return s, nrm, f, toff


def test_backward_is_adjoint_gradient(ctx):
    import torch
    from paper_1309_0100_amd.autograd import tuple_z
    s, nrm, f, toff = _case()
    dev = torch.device("cuda", 0)
    print("case: autograd backward vs oracle gradient, 48 tuples", flush=True)
    fd = torch.tensor(f, device=dev, requires_grad=True)
    z, l, h, fl = tuple_z(ctx, s.t, s.x, s.w, fd, toff, want_h=True)
    rng = np.random.default_rng(1)
    up = torch.tensor(rng.uniform(0.5, 2.0, size=toff.size - 1), device=dev)
    (z * up).sum().backward()
    gf = fd.grad.cpu().numpy()
    zc, flc, upc = z.detach().cpu().numpy(), fl.cpu().numpy(), up.cpu().numpy()
    hc = h.cpu().numpy()
    checked = 0
    for k in range(toff.size - 1):
        a, b = toff[k], toff[k + 1]
        zr, lr, gr, hr = O.tuple_grad(nrm, f[a:b])
        if not np.isfinite(zr):
            assert flc[k] & 8
            continue
        checked += 1
        assert abs(zc[k] - zr) <= 1e-9 * max(abs(zr), 1.0)
        scale = np.maximum(np.abs(gr), 1e-3 * nrm.T_eff * max(zr, 1.0))
        assert np.max(np.abs(gf[a:b] - upc[k] * gr) / (upc[k] * scale)) < 1e-8
        assert np.max(np.abs(hc[a:b] - hr) / np.abs(hr)) < 1e-9
    assert checked >= 40


def test_autograd_matches_central_differences(ctx):
    import torch
    from paper_1309_0100_amd.autograd import tuple_z
    s, nrm, f, toff = _case(seed=761, N=600, n_tuples=8)
    dev = torch.device("cuda", 0)
    print("case: autograd vs central differences, 8 tuples", flush=True)
    fd = torch.tensor(f, device=dev, requires_grad=True)
    z, _, _, fl = tuple_z(ctx, s.t, s.x, s.w, fd, toff)
    z.sum().backward()
    g = fd.grad.cpu().numpy()
    hstep = 1e-5 / nrm.T_eff
    with torch.no_grad():
        for j in range(f.size):
            fp, fm = f.copy(), f.copy()
            fp[j] += hstep
            fm[j] -= hstep
            zp = tuple_z(ctx, s.t, s.x, s.w, torch.tensor(fp, device=dev), toff)[0].cpu().numpy()
            zm = tuple_z(ctx, s.t, s.x, s.w, torch.tensor(fm, device=dev), toff)[0].cpu().numpy()
            k = int(np.searchsorted(toff, j, side="right") - 1)
            if not np.isfinite(zp[k]) or not np.isfinite(zm[k]):
                continue
            fdv = (zp[k] - zm[k]) / (2 * hstep)
            assert abs(fdv - g[j]) <= 1e-6 * max(abs(g[j]), nrm.T_eff), (j, fdv, g[j])


def test_forward_only_has_no_curvature_and_backward_matches_grad(ctx):
    """Without want_h the forward pass makes no adjoint pass (h is NaN); the
    backward pass (fredec_adjoint on the saved theta* and l) gives the
    gradient that one fredec_grad call computes with its own adjoint pass."""
    import torch
    from paper_1309_0100_amd.autograd import tuple_z
    s, nrm, f, toff = _case(seed=733, N=500, n_tuples=32)
    dev = torch.device("cuda", 0)
    print("case: forward-only autograd and backward vs fredec_grad, 32 tuples", flush=True)
    fd = torch.tensor(f, device=dev, requires_grad=True)
    z, l, h, fl = tuple_z(ctx, s.t, s.x, s.w, fd, toff)
    assert torch.isnan(h).all()
    z.sum().backward()
    zg, lg, thg, gg, hg, flg = ctx.grad(s.t, s.x, s.w, f, toff, want_grad=True)
    a, b = fd.grad.cpu().numpy(), gg.cpu().numpy()
    assert np.array_equal(np.isnan(a), np.isnan(b))
    ok = ~np.isnan(b)
    assert np.array_equal(a[ok], b[ok])
    assert np.array_equal(z.detach().cpu().numpy(), zg.cpu().numpy())


def test_autograd_loop_reproduces_library_ascent(ctx):
    """Twenty preconditioned steps f += clamp(g / h, +-0.1 / T_eff) driven
    through autograd give the library's fixed-step ascent."""
    import torch
    from paper_1309_0100_amd.autograd import segments, tuple_z
    s = synth.tuples_series()
    nrm = O.normalize(s.t, s.x, s.w)
    r = O.scan(s.t, s.x, s.w, [], s.df, 4096)
    pk = O.local_maxima(r.z, r.flags)
    peaks = r.freqs[pk[np.lexsort((pk, -r.z[pk]))[:12]]]
    f0, toff = synth.tuples_draw(peaks, n_tuples=256)
    dev = torch.device("cuda", 0)
    print("case: autograd-driven ascent, 256 tuples x 20 steps", flush=True)
    seg = segments(toff, dev)
    f = torch.tensor(f0, device=dev)
    lim = 0.1 / nrm.T_eff
    for _ in range(20):
        fv = f.clone().requires_grad_(True)
        z, l, h, fl = tuple_z(ctx, s.t, s.x, s.w, fv, toff, seg=seg, want_h=True)
        z.sum().backward()
        with torch.no_grad():
            g = fv.grad
            ok = (fl.index_select(0, seg) == 0) & torch.isfinite(g) & torch.isfinite(h) & (h > 0)
            stp = torch.clamp(g / torch.where(ok, h, torch.ones_like(h)), -lim, lim)
            f = torch.where(ok, f + stp, f)
    fa, za, la, fla = ctx.ascent(s.t, s.x, s.w, f0, toff, steps=20, clamp=0.1)
    assert np.max(np.abs(f.cpu().numpy() - fa.cpu().numpy())) * nrm.T_eff < 1e-9
    z, _, _, _ = tuple_z(ctx, s.t, s.x, s.w, f, toff, seg=seg)
    zc, zac = z.cpu().numpy(), za.cpu().numpy()
    good = np.isfinite(zac)
    assert np.array_equal(good, np.isfinite(zc))
    assert np.max(np.abs(zc[good] - zac[good]) / np.maximum(np.abs(zac[good]), 1.0)) < 1e-9
