"""torch.autograd binding of the tuple statistic z(f) (eq. zpow) and its
adjoint gradient.

`tuple_z(ctx, t, x, w, f, toff)` returns z of every ragged tuple (tuple k owns
f[toff[k]:toff[k+1]]) as a differentiable function of the frequencies f.  The
forward pass and the gradient both come from one fredec_grad call: by the
envelope theorem on l = min over theta of chi^2 (Sect. 3, eq. lsqf) the
derivative dz/df_k = (N_H / l) <r J_k> needs no differentiation through the
least-squares solve, so the backward pass only scales the stored per-frequency
gradient by the upstream gradient of the tuple that owns it.  The diagonal
Gauss-Newton curvature h_k = (N_H / l) <J_k^2> is returned beside z (not
differentiable) for preconditioned steps such as f += clamp(g / h).

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
        def forward(actx, f, t, x, w, toff, seg, lib_ctx, precision):
            z, l, theta, g, h, flags = lib_ctx.grad(t, x, w, f.detach(), toff, want_grad=True,
                                                    precision=precision)
            actx.save_for_backward(g, seg)
            actx.mark_non_differentiable(l, h, flags)
            return z, l, h, flags

        @staticmethod
        def backward(actx, gz, gl, gh, gflags):
            g, seg = actx.saved_tensors
            gf = None
            if actx.needs_input_grad[0]:
                gf = g * gz.index_select(0, seg)
            return gf, None, None, None, None, None, None, None

    _TupleZ.fn = TupleZ
    return TupleZ


def segments(toff, device):
    """Owner tuple of every frequency, as a device int64 tensor."""
    import torch
    toff = np.ascontiguousarray(toff, np.int64)
    seg = np.repeat(np.arange(toff.size - 1, dtype=np.int64), np.diff(toff))
    return torch.as_tensor(seg, device=device)


def tuple_z(ctx: "fredec.Context", t, x, w, f, toff, precision: int = fredec.FP64, seg=None):
    """Differentiable z of ragged tuples.  f: device float64 tensor (may require
    grad); toff: host int64 offsets.  Returns (z, l, h, flags); only z carries
    a gradient (dz/df from the adjoint kernel)."""
    toff = np.ascontiguousarray(toff, np.int64)
    if seg is None:
        seg = segments(toff, f.device)
    t, x, w = ctx._f64(t), ctx._f64(x), ctx._f64(w)
    return _function().apply(f, t, x, w, toff, seg, ctx, precision)
