"""Kernel and tile-shape autotuner of the reduced-precision residual scan.

It times, with the library's own HIP-event timing of the scan kernels, on a
synthetic series of the benchmark's shape (N samples, F grid points; by
default the full pass's scans, N = 10^4 and F = 4e6):

* for every column-tile bucket NT of the split-float16 kernel (NT = 1 for
  m <= 7, 2 for m <= 15, ...), every supported count FT of 16-frequency tiles
  per wave, and keeps the fastest;
* for m = 0 .. 6, the float32 VALU kernel against the split-float16 kernel,
  which fixes the boundary of the automatic form (the largest 2m + 2 up to
  which the VALU kernel is faster);
* every kernel family over m = 0, 2, 4, 8, keeping the fastest as the form.

The choice is written to tuning.json next to this file; Context(tuning=True)
applies it through fredec_set_tile.
Usage: python -m paper_1309_0100_amd.autotune [--N 10000 --F 4000000]
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

from . import fredec, synth

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING = os.path.join(HERE, "tuning.json")
# supported FT per column-tile bucket (FT in {1, 2, 4}, NT FT <= 4) and the base size timed for each
F16X3_FT = {1: (1, 2, 4), 2: (1, 2), 3: (1,), 4: (1,)}
BUCKET_M = {1: 4, 2: 10, 3: 18, 4: 24}


def time_scan(ctx, s, base, df, F, reps=5):
    """Mean HIP-event time (ms) of the scan kernels of one float32 scan."""
    import torch
    ctx.scan_series(s.t, s.x, s.w, base, df, F, precision=fredec.FP32)
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(reps):
        ctx.scan_series(s.t, s.x, s.w, base, df, F, precision=fredec.FP32)
    ms, n = ctx.profile_read()
    ctx.profile(False)
    return ms / max(n, 1)


def tune(N=10_000, F=4_000_000, buckets=(1, 2), reps=5, verbose=True, out_path=TUNING):
    ctx = fredec.Context(0, tuning=False)
    s = synth.random_series(7, N, span=4000.0, n_sin=4)
    df = 2.0 / F
    out = {"N": N, "F": F, "scan_f16x3": {}}
    ctx.set_tile(fredec.TILE_SCAN_F32_FORM, 0, fredec.F32_FORM_F16X3)
    for nt in buckets:
        m = BUCKET_M[nt]
        base = np.random.default_rng(nt).uniform(0.01, 1.5, size=m)
        best = None
        for ft in F16X3_FT[nt]:
            ctx.set_tile(fredec.TILE_SCAN_F16X3, nt, ft)
            ms = time_scan(ctx, s, base, df, F, reps)
            if verbose:
                print(f"split-float16 NT={nt} (m={m}) FT={ft}: {ms:.3f} ms", flush=True)
            if best is None or ms < best[1]:
                best = (ft, ms)
        out["scan_f16x3"][str(nt)] = {"FT": best[0], "ms": best[1]}
        ctx.set_tile(fredec.TILE_SCAN_F16X3, nt, best[0])
    # automatic form: the VALU kernel up to the largest 2m + 2 where it wins
    valu_max_kp = 0
    for m in range(0, 7):
        base = np.random.default_rng(100 + m).uniform(0.01, 1.5, size=m)
        t = {}
        for form in (fredec.F32_FORM_VALU, fredec.F32_FORM_F16X3):
            ctx.set_tile(fredec.TILE_SCAN_F32_FORM, 0, form)
            t[form] = time_scan(ctx, s, base, df, F, reps)
        if verbose:
            print(f"m={m}: VALU {t[fredec.F32_FORM_VALU]:.3f} ms, split-float16 {t[fredec.F32_FORM_F16X3]:.3f} ms",
                  flush=True)
        if t[fredec.F32_FORM_VALU] < t[fredec.F32_FORM_F16X3] and valu_max_kp == 2 * m:
            valu_max_kp = 2 * m + 2
    ctx.set_tile(fredec.TILE_SCAN_F32_FORM, 1, valu_max_kp)
    out["scan_f32_auto"] = {"valu_max_kp": valu_max_kp}
    ms_form = {}
    names = {fredec.F32_FORM_VALU: "VALU", fredec.F32_FORM_F16X3: "F16X3", fredec.F32_FORM_AUTO: "AUTO"}
    for form in names:
        ctx.set_tile(fredec.TILE_SCAN_F32_FORM, 0, form)
        tot = 0.0
        for m in (0, 2, 4, 8):
            base = np.random.default_rng(200 + m).uniform(0.01, 1.5, size=m)
            tot += time_scan(ctx, s, base, df, F, reps)
        ms_form[form] = tot
        if verbose:
            print(f"float32 form {names[form]}: {tot:.3f} ms over m = 0, 2, 4, 8", flush=True)
    best_form = min(ms_form, key=ms_form.get)
    out["scan_f32_form"] = {"form": best_form, "ms": ms_form[best_form]}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def apply(ctx, path=TUNING):
    """Apply a stored tuning table to a context (no-op if absent)."""
    if not os.path.exists(path):
        return False
    with open(path) as fh:
        tab = json.load(fh)
    for nt, v in tab.get("scan_f16x3", {}).items():
        ctx.set_tile(fredec.TILE_SCAN_F16X3, int(nt), int(v["FT"]))
    if "scan_f32_form" in tab:
        ctx.set_tile(fredec.TILE_SCAN_F32_FORM, 0, int(tab["scan_f32_form"]["form"]))
    if "scan_f32_auto" in tab:
        ctx.set_tile(fredec.TILE_SCAN_F32_FORM, 1, int(tab["scan_f32_auto"]["valu_max_kp"]))
    return True


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=10_000)
    ap.add_argument("--F", type=int, default=4_000_000)
    ap.add_argument("--buckets", type=int, nargs="+", default=[1, 2])
    ap.add_argument("--out", default=TUNING, help="where to write the table (default: tuning.json here)")
    a = ap.parse_args()
    print(json.dumps(tune(a.N, a.F, tuple(a.buckets), out_path=a.out)))
