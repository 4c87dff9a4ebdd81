"""Thin Python binding of libfredec (ctypes).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libfredec.so.  torch provides device memory (tensors, workspaces)
and streams; no torch type crosses the C ABI.  If the library is not built,
every call raises: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfredec.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "fredec.h")

FP64 = 0
FP32 = 1

OK, EINVAL, EDOF, EWEIGHT, EDEGEN, ESINGULAR, ENOMEM, EDEVICE, ENOTSUP = 0, -1, -2, -3, -4, -5, -6, -7, -8
TILE_SCAN_F16X3 = 1
TILE_SCAN_F32_FORM = 2
TILE_TUPLE_LANES = 3
F32_FORM_VALU, F32_FORM_F16X3, F32_FORM_AUTO = 0, 2, 3
MAX_BASE = 24
MAX_POOL = 27
STATIC_SCRATCH_BYTES = 32 * 1024 * 1024
FLAG_MASKED, FLAG_SINGULAR, FLAG_PERFECT, FLAG_DEGENERATE, FLAG_BADSERIES = 1, 2, 4, 8, 128
FLAG_CONVERGED, FLAG_RESCORED = 16, 64
PROF_KINDS = ("scan", "gram", "solve", "prep", "rescore", "adjoint")

c_i32, c_i64, c_sz, c_p, c_d = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_double
c_pp = ctypes.POINTER(ctypes.c_void_p)
c_szp = ctypes.POINTER(ctypes.c_size_t)

_SIGS = {
    "fredec_create": (c_i32, [c_pp, ctypes.c_int]),
    "fredec_destroy": (None, [c_p]),
    "fredec_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "fredec_version": (ctypes.c_int, []),
    "fredec_set_tile": (c_i32, [c_p, c_i32, c_i32, c_i32]),
    "fredec_profile": (c_i32, [c_p, c_i32]),
    "fredec_profile_read": (c_i32, [c_p, ctypes.POINTER(c_d), ctypes.POINTER(c_i64)]),
    "fredec_profile_read_kinds": (c_i32, [c_p, c_i32, c_p, c_p]),
    "fredec_normalize_workspace": (c_i32, [c_i32, c_szp]),
    "fredec_normalize": (c_i32, [c_p, c_p, c_i32, c_p, c_p, c_p, c_p, c_p, c_sz, c_p, c_p, c_p, c_p, c_p]),
    "fredec_scan_workspace": (c_i32, [c_i32, c_p, c_p, c_p, c_i32, c_szp]),
    "fredec_scan": (c_i32, [c_p, c_p, c_i32, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_i32, c_p, c_sz,
                            c_p, c_p, c_p, c_p]),
    "fredec_tuples_workspace": (c_i32, [c_i64, c_i32, c_p, c_i64, c_i32, c_szp]),
    "fredec_tuples": (c_i32, [c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_i32, c_p, c_i64, c_i32, c_i32, c_p, c_sz,
                              c_p, c_p, c_p, c_p, c_p]),
    "fredec_grad_workspace": (c_i32, [c_i64, c_p, c_i64, c_szp]),
    "fredec_grad": (c_i32, [c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_p, c_i64, c_i32, c_p, c_sz, c_p, c_p, c_p, c_p,
                            c_p, c_p]),
    "fredec_adjoint": (c_i32, [c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_p, c_i64, c_p, c_p, c_i32, c_p, c_sz, c_p,
                               c_p]),
    "fredec_ascent": (c_i32, [c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_p, c_i64, c_i32, c_d, c_i32, c_p, c_sz, c_p,
                              c_p, c_p]),
    "fredec_vuong_workspace": (c_i32, [c_i64, c_p, c_i64, c_szp]),
    "fredec_vuong": (c_i32, [c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_p, c_i64, c_p, c_i64, c_p, c_sz, c_p, c_p]),
    "fredec_global_local_workspace": (c_i32, [c_i64, c_i32, c_i64, c_szp]),
    "fredec_global_local": (c_i32, [c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_i32, c_d, c_i64, c_i32, c_p, c_sz, c_p, c_p,
                                    c_p, c_p]),
    "fredec_zcrit": (c_i32, [c_d, c_i32, c_d, c_p, c_p]),
    "fredec_peaks_workspace": (c_i32, [c_i64, c_szp]),
    "fredec_peaks": (c_i32, [c_p, c_p, c_p, c_p, c_i64, c_d, c_p, c_sz, c_i64, c_p, c_p, c_p]),
    "fredec_cascade_workspace": (c_i32, [c_i32, c_szp]),
    "fredec_cascade": (c_i32, [c_p, c_p, c_p, c_i32, c_i64, c_p, c_p, c_sz, c_p, c_p, c_p]),
    "fredec_phase1_workspace": (c_i32, [c_i64, c_i64, c_i32, c_i32, c_szp]),
    "fredec_phase1": (c_i32, [c_p, c_p, c_p, c_p, c_p, c_i64, c_d, c_i64, c_d, c_d, c_d, c_i32, c_i32, c_i32, c_p,
                              c_sz, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p]),
    "fredec_scan_static": (c_i32, [c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_i32, c_d, c_i64, c_i32, c_p, c_p, c_p,
                                   c_p]),
    "fredec_residual_fap_workspace": (c_i32, [c_i64, c_i64, c_i32, c_i32, c_szp]),
    "fredec_residual_fap": (c_i32, [c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_p, c_i32, c_d, c_i64, c_d, c_i32, c_p,
                                    c_sz, c_p, c_p, c_p]),
    "fredec_scan_at_workspace": (c_i32, [c_i64, c_i32, c_szp]),
    "fredec_scan_at": (c_i32, [c_p, c_p, c_p, c_p, c_p, c_i64, c_p, c_i32, c_d, c_p, c_i64, c_p, c_sz, c_p, c_p]),
    "fredec_plan_destroy": (None, [c_p]),
    "fredec_scan_plan": (c_i32, [c_p, c_p, c_i32, c_p, c_p, c_p, c_p, c_p, c_i32, c_p, c_sz, c_pp]),
    "fredec_plan_scan": (c_i32, [c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p]),
    "fredec_tuples_plan": (c_i32, [c_p, c_p, c_i64, c_p, c_i32, c_p, c_i64, c_i32, c_i32, c_p, c_sz, c_pp]),
    "fredec_plan_tuples": (c_i32, [c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p]),
    "fredec_ascent_plan": (c_i32, [c_p, c_p, c_i64, c_p, c_i64, c_i32, c_d, c_i32, c_p, c_sz, c_pp]),
    "fredec_plan_ascent": (c_i32, [c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p]),
}

_lib = None


class FredecError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = load().fredec_strerror(code).decode() if _lib is not None else str(code)
        super().__init__(f"{where}: {msg} ({code})")


def header_functions() -> list[str]:
    """Names of every function declared in include/fredec.h."""
    with open(HEADER) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(fredec_[a-z0-9_]+)\s*\(", text)))


def load():
    """Load libfredec.so (built in-tree) and declare its signatures."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname as the system
        # one; loading torch first makes libfredec bind to that single runtime
        # (two runtimes in one process would not share devices or streams).
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_1309_0100_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(code: int, where: str):
    if code != OK:
        raise FredecError(code, where)


def _ptr(a) -> int | None:
    """Device pointer of a tensor, host pointer of a numpy array, or None."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        assert a.flags["C_CONTIGUOUS"]
        return a.ctypes.data
    assert a.is_contiguous()
    return a.data_ptr()


def _torch():
    import torch
    return torch


def _stream(device):
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


class Plan:
    """A prepared libfredec call (fredec_*_plan).  Its launches enqueue
    kernels only, so they may be captured into a HIP graph
    (torch.cuda.graph) and replayed.  The plan owns its workspace tensor and
    keeps the output tensors it was given; every launch reads the series from
    the tensors passed to `run`, so new data copied into those tensors are
    picked up by a replay."""

    def __init__(self, ctx: "Context", handle, kind: str, ws, meta: dict):
        self.ctx, self.handle, self.kind, self.ws, self.meta = ctx, handle, kind, ws, meta

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.fredec_plan_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # pragma: no cover - interpreter shutdown
            pass

    def run(self, *args, **kw):
        return getattr(self, "_run_" + self.kind)(*args, **kw)

    def _run_scan(self, t, x, w, out):
        """out = (z, flags, l_base, status) preallocated device tensors."""
        z, fl, lb, st = out
        _check(load().fredec_plan_scan(self.ctx.handle, self.handle, _stream(self.ctx.device), _ptr(t), _ptr(x),
                                       _ptr(w), _ptr(z), _ptr(fl), _ptr(lb), _ptr(st)), "fredec_plan_scan")
        return out

    def _run_tuples(self, t, x, w, out):
        """out = (l, z, f[n_tuples, n_pool], flags, l0) preallocated device tensors."""
        l, z, f, fl, l0 = out
        _check(load().fredec_plan_tuples(self.ctx.handle, self.handle, _stream(self.ctx.device), _ptr(t), _ptr(x),
                                         _ptr(w), _ptr(l), _ptr(z), _ptr(f), _ptr(fl), _ptr(l0)),
               "fredec_plan_tuples")
        return out

    def _run_ascent(self, t, x, w, f, out):
        """f: device float64 frequencies, updated in place; out = (z, l, flags)."""
        z, l, fl = out
        _check(load().fredec_plan_ascent(self.ctx.handle, self.handle, _stream(self.ctx.device), _ptr(t), _ptr(x),
                                         _ptr(w), _ptr(f), _ptr(z), _ptr(l), _ptr(fl)), "fredec_plan_ascent")
        return f, z, l, fl


class Context:
    """A libfredec context bound to one GPU."""

    def __init__(self, device: int = 0, tuning: bool = True):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.fredec_create(ctypes.byref(h), device), "fredec_create")
        self.handle = h
        self.device = device
        if tuning:
            from . import autotune
            autotune.apply(self)

    def close(self):
        if getattr(self, "handle", None):
            load().fredec_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tile(self, kernel: int, key: int, value: int):
        _check(load().fredec_set_tile(self.handle, kernel, key, value), "fredec_set_tile")

    def profile(self, enable: bool = True):
        _check(load().fredec_profile(self.handle, int(enable)), "fredec_profile")

    def profile_read_kinds(self):
        """{kind: (ms, timed groups)} for every kind of kernel group since the last read."""
        n = len(PROF_KINDS)
        ms = np.zeros(n, np.float64)
        cnt = np.zeros(n, np.int64)
        _check(load().fredec_profile_read_kinds(self.handle, n, _ptr(ms), _ptr(cnt)), "fredec_profile_read_kinds")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(PROF_KINDS)}

    def profile_read(self):
        """(total ms, event pairs) of the dominant kernels since the last read."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(load().fredec_profile_read(self.handle, ctypes.byref(ms), ctypes.byref(n)), "fredec_profile_read")
        return ms.value, n.value

    # ------------------------------------------------------------ helpers
    def _dev(self):
        return _torch().device("cuda", self.device)

    def _empty(self, n, dtype):
        return _torch().empty(int(n), dtype=dtype, device=self._dev())

    def _workspace(self, nbytes: int):
        return _torch().empty(max(int(nbytes), 1), dtype=_torch().uint8, device=self._dev())

    def _f64(self, a):
        torch = _torch()
        if isinstance(a, torch.Tensor):
            assert a.dtype == torch.float64 and a.device.type == "cuda"
            return a.contiguous()
        return torch.as_tensor(np.ascontiguousarray(a, np.float64), device=self._dev())

    # ------------------------------------------------------------ API
    def normalize(self, t, x, w, soff=None):
        """Normalised series (tau, xt, wt), per-series stats and status."""
        torch = _torch()
        t, x, w = self._f64(t), self._f64(x), self._f64(w)
        soff = np.asarray([0, t.numel()] if soff is None else soff, np.int64)
        ns = soff.size - 1
        need = ctypes.c_size_t()
        _check(load().fredec_normalize_workspace(ns, ctypes.byref(need)), "fredec_normalize_workspace")
        ws = self._workspace(need.value)
        tau, xt, wt = (torch.empty_like(t) for _ in range(3))
        stats = self._empty(6 * ns, torch.float64)
        status = self._empty(ns, torch.int32)
        _check(load().fredec_normalize(self.handle, _stream(self.device), ns, _ptr(soff), _ptr(t), _ptr(x), _ptr(w),
                                       _ptr(ws), need.value, _ptr(tau), _ptr(xt), _ptr(wt), _ptr(stats),
                                       _ptr(status)), "fredec_normalize")
        return tau, xt, wt, stats.view(ns, 6), status

    def scan_workspace(self, soff, boff, F, precision=FP64) -> int:
        soff = np.ascontiguousarray(soff, np.int64)
        boff = np.ascontiguousarray(boff, np.int64)
        F = np.ascontiguousarray(F, np.int64)
        need = ctypes.c_size_t()
        _check(load().fredec_scan_workspace(soff.size - 1, _ptr(soff), _ptr(boff), _ptr(F), precision,
                                            ctypes.byref(need)), "fredec_scan_workspace")
        return need.value

    def scan(self, t, x, w, soff, base_f, boff, df, F, precision=FP64, workspace=None, out=None):
        """Residual periodogram of a CSR batch of series.  Returns
        (z, flags, l_base, status) as device tensors; z of series s occupies
        [sum(F[:s]), sum(F[:s+1]))."""
        torch = _torch()
        t, x, w = self._f64(t), self._f64(x), self._f64(w)
        soff = np.ascontiguousarray(soff, np.int64)
        boff = np.ascontiguousarray(boff, np.int64)
        base_f = np.ascontiguousarray(base_f, np.float64)
        df = np.ascontiguousarray(np.broadcast_to(df, (soff.size - 1,)), np.float64)
        F = np.ascontiguousarray(np.broadcast_to(F, (soff.size - 1,)), np.int64)
        ns = soff.size - 1
        need = self.scan_workspace(soff, boff, F, precision)
        ws = workspace if workspace is not None and workspace.numel() >= need else self._workspace(need)
        total = int(F.sum())
        if out is None:
            out = (self._empty(total, torch.float64), self._empty(total, torch.uint8),
                   self._empty(ns, torch.float64), self._empty(ns, torch.int32))
        z, flags, lbase, status = out
        _check(load().fredec_scan(self.handle, _stream(self.device), ns, _ptr(t), _ptr(x), _ptr(w), _ptr(soff),
                                  _ptr(base_f) if base_f.size else None, _ptr(boff), _ptr(df), _ptr(F), precision,
                                  _ptr(ws), ws.numel(), _ptr(z), _ptr(flags), _ptr(lbase), _ptr(status)),
               "fredec_scan")
        return z, flags, lbase, status

    def scan_series(self, t, x, w, base_f, df, F, precision=FP64):
        """One series: returns (z, flags, l_base, status)."""
        n = len(t) if not hasattr(t, "numel") else t.numel()
        base_f = np.atleast_1d(np.asarray(base_f, np.float64))
        return self.scan(t, x, w, [0, n], base_f, [0, base_f.size], [df], [F], precision)

    def scan_static(self, t, x, w, base_f, df, F, precision=FP64, out=None):
        """One series through the allocation-free entry point
        (fredec_scan_static: scratch in the library's static device array;
        `out` = preallocated (z, flags, l_base, status) tensors, else they are
        allocated here, outside the call).  Returns (z, flags, l_base, status)."""
        torch = _torch()
        t, x, w = self._f64(t), self._f64(x), self._f64(w)
        base_f = np.ascontiguousarray(np.atleast_1d(np.asarray(base_f, np.float64)))
        if out is None:
            out = (self._empty(F, torch.float64), self._empty(F, torch.uint8), self._empty(1, torch.float64),
                   self._empty(1, torch.int32))
        z, flags, lbase, status = out
        _check(load().fredec_scan_static(self.handle, _stream(self.device), _ptr(t), _ptr(x), _ptr(w), t.numel(),
                                         _ptr(base_f) if base_f.size else None, base_f.size, float(df), int(F),
                                         precision, _ptr(z), _ptr(flags), _ptr(lbase), _ptr(status)),
               "fredec_scan_static")
        return z, flags, lbase, status

    def scan_at(self, t, x, w, base_f, df, idx):
        """float64 statistic of one series at grid indices idx (device int64)."""
        torch = _torch()
        t, x, w = self._f64(t), self._f64(x), self._f64(w)
        base_f = np.ascontiguousarray(np.atleast_1d(base_f), np.float64)
        idx = idx if isinstance(idx, torch.Tensor) else torch.as_tensor(np.asarray(idx, np.int64), device=self._dev())
        n_idx = idx.numel()
        need = ctypes.c_size_t()
        _check(load().fredec_scan_at_workspace(t.numel(), base_f.size, ctypes.byref(need)), "fredec_scan_at_workspace")
        ws = self._workspace(need.value)
        z = self._empty(n_idx, torch.float64)
        fl = self._empty(n_idx, torch.uint8)
        _check(load().fredec_scan_at(self.handle, _stream(self.device), _ptr(t), _ptr(x), _ptr(w), t.numel(),
                                     _ptr(base_f) if base_f.size else None, base_f.size, float(df), _ptr(idx), n_idx,
                                     _ptr(ws), need.value, _ptr(z), _ptr(fl)), "fredec_scan_at")
        return z, fl


    # ------------------------------------------------------------ tuples
    def tuples(self, t, x, w, pool, masks=None, refine_steps=0, precision=FP64, l_out=None, l0_out=None):
        """Statistics of subsets of a frequency pool.  Returns device tensors
        (l, z, f[n_tuples, n_pool], flags); l may be written into a caller
        tensor l_out, and l_0 of the constant model into l0_out."""
        torch = _torch()
        t, x, w = self._f64(t), self._f64(x), self._f64(w)
        pool = np.ascontiguousarray(pool, np.float64)
        npool = pool.size
        mk = None if masks is None else np.ascontiguousarray(masks, np.uint64)
        nt = (1 << npool) - 1 if mk is None else mk.size
        need = ctypes.c_size_t()
        _check(load().fredec_tuples_workspace(t.numel(), npool, _ptr(mk), nt, refine_steps, ctypes.byref(need)),
               "fredec_tuples_workspace")
        ws = self._workspace(need.value)
        l = self._empty(nt, torch.float64) if l_out is None else l_out
        z = self._empty(nt, torch.float64)
        f = self._empty(nt * npool, torch.float64)
        fl = self._empty(nt, torch.uint8)
        _check(load().fredec_tuples(self.handle, _stream(self.device), _ptr(t), _ptr(x), _ptr(w), t.numel(),
                                    _ptr(pool), npool, _ptr(mk), nt, refine_steps, precision, _ptr(ws), need.value,
                                    _ptr(l), _ptr(z), _ptr(f), _ptr(fl), _ptr(l0_out)), "fredec_tuples")
        return l, z, f.view(nt, npool), fl

    def grad(self, t, x, w, f, toff, want_grad=True, precision=FP64):
        """z, l, theta, dz/df, h, flags of ragged tuples (f device float64)."""
        torch = _torch()
        t, x, w, f = self._f64(t), self._f64(x), self._f64(w), self._f64(f)
        toff = np.ascontiguousarray(toff, np.int64)
        nt = toff.size - 1
        need = ctypes.c_size_t()
        _check(load().fredec_grad_workspace(t.numel(), _ptr(toff), nt, ctypes.byref(need)), "fredec_grad_workspace")
        ws = self._workspace(need.value)
        z, l = self._empty(nt, torch.float64), self._empty(nt, torch.float64)
        th = self._empty(2 * int(toff[-1]) + nt, torch.float64)
        g = self._empty(int(toff[-1]), torch.float64) if want_grad else None
        h = self._empty(int(toff[-1]), torch.float64) if want_grad else None
        fl = self._empty(nt, torch.uint8)
        _check(load().fredec_grad(self.handle, _stream(self.device), _ptr(t), _ptr(x), _ptr(w), t.numel(), _ptr(f),
                                  _ptr(toff), nt, precision, _ptr(ws), need.value, _ptr(z), _ptr(l), _ptr(th),
                                  _ptr(g), _ptr(h), _ptr(fl)), "fredec_grad")
        return z, l, th, g, h, fl

    def adjoint(self, t, x, w, f, toff, theta, l, want_h=False, precision=FP64):
        """dz/df (and h) of ragged tuples from an earlier forward evaluation's
        theta and l (device tensors, as returned by grad)."""
        torch = _torch()
        t, x, w, f = self._f64(t), self._f64(x), self._f64(w), self._f64(f)
        theta, l = self._f64(theta), self._f64(l)
        toff = np.ascontiguousarray(toff, np.int64)
        nt = toff.size - 1
        need = ctypes.c_size_t()
        _check(load().fredec_grad_workspace(t.numel(), _ptr(toff), nt, ctypes.byref(need)), "fredec_grad_workspace")
        ws = self._workspace(need.value)
        g = self._empty(int(toff[-1]), torch.float64)
        h = self._empty(int(toff[-1]), torch.float64) if want_h else None
        _check(load().fredec_adjoint(self.handle, _stream(self.device), _ptr(t), _ptr(x), _ptr(w), t.numel(), _ptr(f),
                                     _ptr(toff), nt, _ptr(theta), _ptr(l), precision, _ptr(ws), need.value, _ptr(g),
                                     _ptr(h)), "fredec_adjoint")
        return g, h

    def ascent(self, t, x, w, f, toff, steps=20, clamp=0.1, precision=FP64):
        """Preconditioned ascent; returns (f, z, l, flags) with f a new device tensor."""
        torch = _torch()
        t, x, w = self._f64(t), self._f64(x), self._f64(w)
        f = self._f64(f).clone()
        toff = np.ascontiguousarray(toff, np.int64)
        nt = toff.size - 1
        need = ctypes.c_size_t()
        _check(load().fredec_grad_workspace(t.numel(), _ptr(toff), nt, ctypes.byref(need)), "fredec_grad_workspace")
        ws = self._workspace(need.value)
        z, l = self._empty(nt, torch.float64), self._empty(nt, torch.float64)
        fl = self._empty(nt, torch.uint8)
        _check(load().fredec_ascent(self.handle, _stream(self.device), _ptr(t), _ptr(x), _ptr(w), t.numel(), _ptr(f),
                                    _ptr(toff), nt, steps, float(clamp), precision, _ptr(ws), need.value, _ptr(z),
                                    _ptr(l), _ptr(fl)), "fredec_ascent")
        return f, z, l, fl


    # ------------------------------------------------------------ plans
    def scan_plan(self, soff, base_f, boff, df, F, precision=FP64):
        """Plan of fredec_scan for a fixed batch; returns (plan, out) with out
        the preallocated (z, flags, l_base, status) for plan.run(t, x, w, out)."""
        torch = _torch()
        soff = np.ascontiguousarray(soff, np.int64)
        boff = np.ascontiguousarray(boff, np.int64)
        base_f = np.ascontiguousarray(base_f, np.float64)
        ns = soff.size - 1
        df = np.ascontiguousarray(np.broadcast_to(df, (ns,)), np.float64)
        F = np.ascontiguousarray(np.broadcast_to(F, (ns,)), np.int64)
        ws = self._workspace(self.scan_workspace(soff, boff, F, precision))
        h = ctypes.c_void_p()
        _check(load().fredec_scan_plan(self.handle, _stream(self.device), ns, _ptr(soff),
                                       _ptr(base_f) if base_f.size else None, _ptr(boff), _ptr(df), _ptr(F),
                                       precision, _ptr(ws), ws.numel(), ctypes.byref(h)), "fredec_scan_plan")
        total = int(F.sum())
        out = (self._empty(total, torch.float64), self._empty(total, torch.uint8), self._empty(ns, torch.float64),
               self._empty(ns, torch.int32))
        return Plan(self, h, "scan", ws, {"n_series": ns, "F": F}), out

    def tuples_plan(self, N, pool, masks=None, refine_steps=0, precision=FP64):
        """Plan of fredec_tuples; returns (plan, out) with out = (l, z, f, flags, l0)."""
        torch = _torch()
        pool = np.ascontiguousarray(pool, np.float64)
        npool = pool.size
        mk = None if masks is None else np.ascontiguousarray(masks, np.uint64)
        nt = (1 << npool) - 1 if mk is None else mk.size
        need = ctypes.c_size_t()
        _check(load().fredec_tuples_workspace(int(N), npool, _ptr(mk), nt, refine_steps, ctypes.byref(need)),
               "fredec_tuples_workspace")
        ws = self._workspace(need.value)
        h = ctypes.c_void_p()
        _check(load().fredec_tuples_plan(self.handle, _stream(self.device), int(N), _ptr(pool), npool, _ptr(mk), nt,
                                         refine_steps, precision, _ptr(ws), need.value, ctypes.byref(h)),
               "fredec_tuples_plan")
        out = (self._empty(nt, torch.float64), self._empty(nt, torch.float64),
               self._empty(nt * npool, torch.float64).view(nt, npool), self._empty(nt, torch.uint8),
               self._empty(1, torch.float64))
        return Plan(self, h, "tuples", ws, {"n_tuples": nt}), out

    def ascent_plan(self, N, toff, steps=20, clamp=0.1, precision=FP64):
        """Plan of fredec_ascent; returns (plan, out) with out = (z, l, flags)."""
        torch = _torch()
        toff = np.ascontiguousarray(toff, np.int64)
        nt = toff.size - 1
        need = ctypes.c_size_t()
        _check(load().fredec_grad_workspace(int(N), _ptr(toff), nt, ctypes.byref(need)), "fredec_grad_workspace")
        ws = self._workspace(need.value)
        h = ctypes.c_void_p()
        _check(load().fredec_ascent_plan(self.handle, _stream(self.device), int(N), _ptr(toff), nt, steps,
                                         float(clamp), precision, _ptr(ws), need.value, ctypes.byref(h)),
               "fredec_ascent_plan")
        out = (self._empty(nt, torch.float64), self._empty(nt, torch.float64), self._empty(nt, torch.uint8))
        return Plan(self, h, "ascent", ws, {"n_tuples": nt}), out


    # ------------------------------------------------------------ selection
    def peaks(self, z, flags, zmin, cap=1 << 16):
        """Local maxima of z above zmin: (idx, z) host arrays sorted by index."""
        F = z.numel()
        need = ctypes.c_size_t()
        _check(load().fredec_peaks_workspace(cap, ctypes.byref(need)), "fredec_peaks_workspace")
        ws = self._workspace(need.value)
        idx = np.zeros(cap, np.int64)
        zp = np.zeros(cap, np.float64)
        nf = ctypes.c_int64()
        _check(load().fredec_peaks(self.handle, _stream(self.device), _ptr(z), _ptr(flags), F, float(zmin), _ptr(ws),
                                   need.value, cap, _ptr(idx), _ptr(zp), ctypes.byref(nf)), "fredec_peaks")
        n = min(nf.value, cap)
        return idx[:n].copy(), zp[:n].copy()

    def global_local(self, t, x, w, base_f, df, F, refine_steps=8):
        """Global-local residual periodogram: device tensors (z, flags, l_b,
        refined base frequencies)."""
        torch = _torch()
        t, x, w = self._f64(t), self._f64(x), self._f64(w)
        base_f = np.ascontiguousarray(np.atleast_1d(np.asarray(base_f, np.float64)))
        m = base_f.size
        need = ctypes.c_size_t()
        _check(load().fredec_global_local_workspace(t.numel(), m, int(F), ctypes.byref(need)),
               "fredec_global_local_workspace")
        ws = self._workspace(need.value)
        z, fl = self._empty(F, torch.float64), self._empty(F, torch.uint8)
        lb, fb = self._empty(1, torch.float64), self._empty(max(m, 1), torch.float64)
        _check(load().fredec_global_local(self.handle, _stream(self.device), _ptr(t), _ptr(x), _ptr(w), t.numel(),
                                          _ptr(base_f) if m else None, m, float(df), int(F), int(refine_steps),
                                          _ptr(ws), need.value, _ptr(z), _ptr(fl), _ptr(lb), _ptr(fb) if m else None),
               "fredec_global_local")
        return z, fl, lb, fb[:m]

    def vuong(self, t, x, w, solutions, ref):
        """Vuong's statistic of solution `ref` against every solution (a list
        of frequency lists), at the least-squares fits of their frequencies:
        device tensors (V, l)."""
        torch = _torch()
        t, x, w = self._f64(t), self._f64(x), self._f64(w)
        flat, toff = _ragged(solutions)
        nt = toff.size - 1
        f = self._f64(flat[:toff[-1]])
        _, _, theta, _, _, _ = self.grad(t, x, w, f, toff, want_grad=False)
        need = ctypes.c_size_t()
        _check(load().fredec_vuong_workspace(t.numel(), _ptr(toff), nt, ctypes.byref(need)), "fredec_vuong_workspace")
        ws = self._workspace(need.value)
        V = self._empty(nt, torch.float64)
        l = self._empty(nt, torch.float64)
        _check(load().fredec_vuong(self.handle, _stream(self.device), _ptr(t), _ptr(x), _ptr(w), t.numel(), _ptr(f),
                                   _ptr(toff), nt, _ptr(theta), int(ref), _ptr(ws), need.value, _ptr(l), _ptr(V)),
               "fredec_vuong")
        return V, l

    def residual_fap(self, t, x, w, solutions, df, F, A1=1.0, precision=FP64):
        """Residual single-frequency FAP of each solution (a list of frequency
        lists): host arrays (fap, z_max, j_max)."""
        t, x, w = self._f64(t), self._f64(x), self._f64(w)
        flat, off = _ragged(solutions)
        n_sol = off.size - 1
        m_max = int(np.max(np.diff(off))) if n_sol else 0
        need = ctypes.c_size_t()
        _check(load().fredec_residual_fap_workspace(t.numel(), int(F), m_max, precision, ctypes.byref(need)),
               "fredec_residual_fap_workspace")
        ws = self._workspace(need.value)
        fap, zmax = np.zeros(n_sol), np.zeros(n_sol)
        jmax = np.zeros(n_sol, np.int64)
        _check(load().fredec_residual_fap(self.handle, _stream(self.device), _ptr(t), _ptr(x), _ptr(w), t.numel(),
                                          _ptr(flat), _ptr(off), n_sol, float(df), int(F), float(A1), precision,
                                          _ptr(ws), need.value, _ptr(fap), _ptr(zmax), _ptr(jmax)),
               "fredec_residual_fap")
        return fap, zmax, jmax

    def cascade(self, ltab, n, N, zcrit):
        """Phase 3: (survive, maximal, G) device tensors of length 2^n."""
        torch = _torch()
        ltab = self._f64(ltab)
        zc = np.ascontiguousarray(zcrit, np.float64)
        need = ctypes.c_size_t()
        _check(load().fredec_cascade_workspace(n, ctypes.byref(need)), "fredec_cascade_workspace")
        ws = self._workspace(need.value)
        M = 1 << n
        surv, maxi = self._empty(M, torch.uint8), self._empty(M, torch.uint8)
        G = self._empty(M, torch.float64)
        _check(load().fredec_cascade(self.handle, _stream(self.device), _ptr(ltab), n, int(N), _ptr(zc), _ptr(ws),
                                     need.value, _ptr(surv), _ptr(maxi), _ptr(G)), "fredec_cascade")
        return surv, maxi, G

    def phase1(self, t, x, w, df, F, fap0=0.05, fap1=0.1, A1=1.0, pool_cap=0, max_scans=25, precision=FP64):
        """Phase 1 preliminary scan: dict with pool, pool_z, base, n_scans, truncated, W."""
        t, x, w = self._f64(t), self._f64(x), self._f64(w)
        N = t.numel()
        need = ctypes.c_size_t()
        _check(load().fredec_phase1_workspace(N, F, max_scans, precision, ctypes.byref(need)),
               "fredec_phase1_workspace")
        ws = self._workspace(need.value)
        capn = max(pool_cap, N // 10, 1)
        pool, pz = np.zeros(capn), np.zeros(capn)
        base = np.zeros(max_scans)
        n_pool, n_base, n_scans, trunc = (ctypes.c_int32() for _ in range(4))
        W = ctypes.c_double()
        _check(load().fredec_phase1(self.handle, _stream(self.device), _ptr(t), _ptr(x), _ptr(w), N, float(df),
                                    int(F), fap0, fap1, A1, pool_cap, max_scans, precision, _ptr(ws), need.value,
                                    _ptr(pool), _ptr(pz), ctypes.byref(n_pool), _ptr(base), ctypes.byref(n_base),
                                    ctypes.byref(n_scans), ctypes.byref(trunc), ctypes.byref(W)), "fredec_phase1")
        return {"pool": pool[:n_pool.value].copy(), "pool_z": pz[:n_pool.value].copy(),
                "base": base[:n_base.value].copy(), "n_scans": n_scans.value, "truncated": trunc.value,
                "W": W.value}


def _ragged(lists):
    """Concatenated float64 values and int64 offsets of a list of sequences."""
    vals = [np.atleast_1d(np.asarray(v, np.float64)) for v in lists]
    off = np.zeros(len(vals) + 1, np.int64)
    off[1:] = np.cumsum([v.size for v in vals])
    flat = np.ascontiguousarray(np.concatenate(vals) if off[-1] else np.zeros(1), np.float64)
    return flat, off


def zcrit(W, n, fap, A=None):
    """Thresholds zc[0..n] of eq. zFAP (host computation in libfredec)."""
    zc = np.zeros(n + 1)
    Aa = None if A is None else np.ascontiguousarray(A, np.float64)
    _check(load().fredec_zcrit(float(W), int(n), float(fap), _ptr(Aa), _ptr(zc)), "fredec_zcrit")
    return zc


@dataclass
class ScanOut:
    z: object
    flags: object
    l_base: object
    status: object
