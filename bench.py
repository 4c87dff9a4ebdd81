"""Benchmark of the FREDEC residual-periodogram hot path on one MI355X.

Workload (default): the residual scan - one series of N=2000 irregular times
over 4000 d with seasonal gaps (8 months on / 4 off), 4 injected sinusoids,
base model = constant + the 4 injected frequencies (m = 4), F = 10^6 grid
frequencies up to 2 cycles/day.  One step = normalisation, base-model
precomputation, trig sums and 2x2 Schur solves for every grid frequency
(fredec_scan).  Inputs are resident in HBM before the timed region.

Prints one JSON line: points/s = N * F per second (whole job), the roofline of
the dominant kernel (its duration measured live with HIP events on its own
stream), and the float64 CPU oracle timed on a bounded sample of the same
workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "periodogram points/s (N×F) + tuples/s at stated rel-err vs FP64 oracle"

# MI355X published peaks
PEAK_FP64_VALU = 78.6e12      # flop/s, FMA = 2 flops
PEAK_FP32_MFMA = 157.3e12     # flop/s, dense
PEAK_HBM = 8.0e12             # B/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle time of the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile", type=int, default=0, help="MFMA frequency tiles per wave (0 = tuned/default)")
    return ap.parse_args()


def cpu_baseline(s, z_gpu, seconds):
    """The float64 oracle on a bounded, strided sample of the grid, single
    thread; also the error of the GPU result on those frequencies."""
    try:
        from threadpoolctl import threadpool_limits
        limiter = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        limiter = None
    import oracle as O
    stride = 11
    idx_all = np.arange(0, s.F, stride)
    done = []
    errs = []
    t0 = time.perf_counter()
    block = 256
    for b in range(0, idx_all.size, block):
        idx = idx_all[b:b + block]
        ref = O.scan(s.t, s.x, s.w, s.base_f, s.df, s.F, idx=idx)
        good = ref.flags == 0
        zg = z_gpu[idx]
        errs.append(np.max(np.abs(zg[good] - ref.z[good]) / np.maximum(np.abs(ref.z[good]), 1.0), initial=0.0))
        done.append(idx.size)
        if time.perf_counter() - t0 > seconds:
            break
    el = time.perf_counter() - t0
    nf = int(np.sum(done))
    if limiter is not None:
        limiter.unregister() if hasattr(limiter, "unregister") else None
    return {
        "value": s.N * nf / el,
        "unit": "points/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{nf} grid frequencies (every {stride}th of F={s.F}) of the same series, N={s.N}, m={s.base_f.size}; {el:.1f} s",
    }, float(np.max(errs))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    from paper_1309_0100_amd import fredec, synth

    prec = fredec.FP64 if args.precision == "fp64" else fredec.FP32
    ctx = fredec.Context(0)
    if args.tile:
        ctx.set_tile(fredec.TILE_SCAN_MFMA, 1, args.tile)
    s = synth.residual()
    dev = torch.device("cuda", 0)
    t = torch.as_tensor(s.t, device=dev)
    x = torch.as_tensor(s.x, device=dev)
    w = torch.as_tensor(s.w, device=dev)
    soff = np.array([0, s.N], np.int64)
    boff = np.array([0, s.base_f.size], np.int64)
    need = ctx.scan_workspace(soff, boff, [s.F], prec)
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    out = (torch.empty(s.F, dtype=torch.float64, device=dev), torch.empty(s.F, dtype=torch.uint8, device=dev),
           torch.empty(1, dtype=torch.float64, device=dev), torch.empty(1, dtype=torch.int32, device=dev))

    def step():
        ctx.scan(t, x, w, soff, s.base_f, boff, [s.df], [s.F], prec, workspace=ws, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kms, nl = ctx.profile_read()
    ctx.profile(False)
    points = s.N * s.F
    value = points * args.steps / el
    m = s.base_f.size
    KP = 2 * m + 2
    kernel_s = kms / 1e3 / max(nl, 1)
    if prec == fredec.FP64:
        sums = 2 * KP + 3                  # trig sums per (frequency, sample) pair
        flops_per_pair = 2 * sums          # one multiply-add each
        roof = {"bound": "alu", "peak": PEAK_FP64_VALU, "kernel": "scan_f64_kernel",
                "algorithmic": f"{flops_per_pair} flop per (frequency, sample) pair: {sums} float64 multiply-adds"}
    else:
        flops_per_pair = 4 * KP            # (cos, sin) x KP columns, one multiply-add each, on MFMA
        roof = {"bound": "mfma", "peak": PEAK_FP32_MFMA, "kernel": "scan_mfma_kernel",
                "algorithmic": f"{flops_per_pair} flop per (frequency, sample) pair: 2 x {KP} float32 "
                               "multiply-adds on MFMA (unpadded)"}
    achieved = flops_per_pair * points / kernel_s
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == fredec.FP64 else "f32",
        "data": "synthetic",
        "config": {"workload": "residual scan: N=2000 over 4000 d, seasonal gaps, m=4 base sinusoids, "
                               "F=10^6 grid to 2 c/d", "N": s.N, "F": s.F, "m": m,
                   "precision": args.precision},
        "roofline": {"bound": roof["bound"], "achieved": achieved / 1e12, "peak": roof["peak"] / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / roof["peak"], "traffic": None,
                     "kernel": roof["kernel"], "kernel_ms": kernel_s * 1e3, "algorithmic": roof["algorithmic"]},
    }
    if not args.no_cpu:
        z_gpu = out[0].cpu().numpy()
        cb, err = cpu_baseline(s, z_gpu, args.cpu_seconds)
        res["cpu_baseline"] = cb
        res["max_rel_err_vs_oracle"] = err
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
