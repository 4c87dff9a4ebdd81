"""torch.autograd binding of the tuple statistic z(f) (eq. zpow) and its
adjoint gradient.

`tuple_z(ctx, t, x, w, f, toff)` returns z of every ragged tuple (tuple k owns
f[toff[k]:toff[k+1]]) as a differentiable function of the frequencies f.  The
forward pass is one fredec_grad call without the adjoint (z, l and theta*);
the backward pass launches the adjoint kernels alone (fredec_adjoint on the
saved theta* and l): by the envelope theorem on l = min over theta of chi^2
(Sect. 3, eq. lsqf) the derivative dz/df_k = (N_H / l) <r J_k> needs no
differentiation through the least-squares solve, and it is scaled by the
upstream gradient of the tuple that owns it.  Forward-only evaluations
therefore pay for no adjoint.  With want_h=True the forward pass also
returns the diagonal Gauss-Newton curvature h_k = (N_H / l) <J_k^2> (not
differentiable; it needs the adjoint pass) for preconditioned steps such as
f += clamp(g / h).

Only argument marshalling happens here; z, dz/df and h are computed by the
library's kernels.
"""
from __future__ import annotations

import numpy as np

from . import fredec


class _TupleZ:
    """Holder of the torch.autograd.Function (built lazily so that importing
    this module does not import torch)."""

    fn = None


def _function():
    if _TupleZ.fn is not None:
        return _TupleZ.fn
    import torch

    class TupleZ(torch.autograd.Function):
        @staticmethod
        def forward(actx, f, t, x, w, toff, seg, lib_ctx, precision, want_h):
            fd = f.detach()
            z, l, theta, g, h, flags = lib_ctx.grad(t, x, w, fd, toff, want_grad=want_h, precision=precision)
            actx.save_for_backward(fd, t, x, w, theta, l, seg)
            actx.toff, actx.lib_ctx, actx.precision = toff, lib_ctx, precision
            if h is None:
                h = torch.full_like(fd, float("nan"))
            actx.mark_non_differentiable(l, h, flags)
            return z, l, h, flags

        @staticmethod
        def backward(actx, gz, gl, gh, gflags):
            gf = None
            if actx.needs_input_grad[0]:
                fd, t, x, w, theta, l, seg = actx.saved_tensors
                g, _ = actx.lib_ctx.adjoint(t, x, w, fd, actx.toff, theta, l, precision=actx.precision)
                gf = g * gz.index_select(0, seg)
            return gf, None, None, None, None, None, None, None, None

    _TupleZ.fn = TupleZ
    return TupleZ


def segments(toff, device):
    """Owner tuple of every frequency, as a device int64 tensor."""
    import torch
    toff = np.ascontiguousarray(toff, np.int64)
    seg = np.repeat(np.arange(toff.size - 1, dtype=np.int64), np.diff(toff))
    return torch.as_tensor(seg, device=device)


def tuple_z(ctx: "fredec.Context", t, x, w, f, toff, precision: int = fredec.FP64, seg=None, want_h=False):
    """Differentiable z of ragged tuples.  f: device float64 tensor (may require
    grad); toff: host int64 offsets.  Returns (z, l, h, flags); only z carries
    a gradient (dz/df from the adjoint kernel, launched by backward).  h is
    NaN unless want_h."""
    toff = np.ascontiguousarray(toff, np.int64)
    if seg is None:
        seg = segments(toff, f.device)
    t, x, w = ctx._f64(t), ctx._f64(x), ctx._f64(w)
    return _function().apply(f, t, x, w, toff, seg, ctx, precision, want_h)
