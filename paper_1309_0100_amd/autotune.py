"""Kernel and tile-shape autotuner for the float32 residual scan.

For each operand width bucket NT (16-column tiles: 1 for m <= 7, 2 for
m <= 15, ...) it times every supported frequency-tile count FT of the MFMA
kernel on a synthetic series of the benchmark's shape (N samples, m base
frequencies, F grid points) and keeps the fastest; then it times the VALU
kernel of the float32 form against the tuned MFMA kernel and keeps the
faster.  The choice is written to
tuning.json next to this file; Context(tuning=True) applies it through
fredec_set_tile.  Usage: python -m paper_1309_0100_amd.autotune [--N 2000 --F 1000000]
"""
from __future__ import annotations

import argparse
import json
import os

import numpy as np

from . import fredec, synth

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING = os.path.join(HERE, "tuning.json")
CANDIDATES = {1: (2, 4, 6, 8), 2: (2, 4), 3: (2,), 4: (2,)}
BUCKET_M = {1: 4, 2: 10, 3: 18, 4: 24}


def time_scan(ctx, s, base, df, F, reps=5):
    import torch
    ctx.scan_series(s.t, s.x, s.w, base, df, F, precision=fredec.FP32)
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(reps):
        ctx.scan_series(s.t, s.x, s.w, base, df, F, precision=fredec.FP32)
    ms, n = ctx.profile_read()
    ctx.profile(False)
    return ms / max(n, 1)


def tune(N=2000, F=1_000_000, buckets=(1, 2), reps=5, verbose=True, out_path=TUNING):
    ctx = fredec.Context(0, tuning=False)
    s = synth.random_series(7, N, span=4000.0, n_sin=4)
    out = {"N": N, "F": F, "scan_mfma": {}}
    ctx.set_tile(fredec.TILE_SCAN_F32_FORM, 0, 1)  # time the MFMA kernel's tiles first
    for nt in buckets:
        m = BUCKET_M[nt]
        base = np.random.default_rng(nt).uniform(0.01, 1.5, size=m)
        best = None
        for ft in CANDIDATES[nt]:
            ctx.set_tile(fredec.TILE_SCAN_MFMA, nt, ft)
            ms = time_scan(ctx, s, base, 2.0 / F, F, reps)
            if verbose:
                print(f"NT={nt} (m={m}) FT={ft}: {ms:.3f} ms", flush=True)
            if best is None or ms < best[1]:
                best = (ft, ms)
        out["scan_mfma"][str(nt)] = {"FT": best[0], "ms": best[1]}
        ctx.set_tile(fredec.TILE_SCAN_MFMA, nt, best[0])
    # float32 form: VALU kernel against the tuned MFMA kernel, on the m of the first bucket
    m = BUCKET_M[buckets[0]]
    base = np.random.default_rng(buckets[0]).uniform(0.01, 1.5, size=m)
    t_form = {}
    for form in (1, 0):
        ctx.set_tile(fredec.TILE_SCAN_F32_FORM, 0, form)
        t_form[form] = time_scan(ctx, s, base, 2.0 / F, F, reps)
        if verbose:
            print(f"float32 form {'MFMA' if form else 'VALU'} (m={m}): {t_form[form]:.3f} ms", flush=True)
    best_form = min(t_form, key=t_form.get)
    out["scan_f32_form"] = {"form": best_form, "ms": t_form[best_form]}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    return out


def apply(ctx, path=TUNING):
    """Apply a stored tuning table to a context (no-op if absent)."""
    if not os.path.exists(path):
        return False
    with open(path) as fh:
        tab = json.load(fh)
    for nt, v in tab.get("scan_mfma", {}).items():
        ctx.set_tile(fredec.TILE_SCAN_MFMA, int(nt), int(v["FT"]))
    if "scan_f32_form" in tab:
        ctx.set_tile(fredec.TILE_SCAN_F32_FORM, 0, int(tab["scan_f32_form"]["form"]))
    return True


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--N", type=int, default=2000)
    ap.add_argument("--F", type=int, default=1_000_000)
    ap.add_argument("--buckets", type=int, nargs="+", default=[1, 2])
    ap.add_argument("--out", default=TUNING, help="where to write the table (default: tuning.json here)")
    a = ap.parse_args()
    print(json.dumps(tune(a.N, a.F, tuple(a.buckets), out_path=a.out)))
