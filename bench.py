"""Benchmark of the FREDEC multifrequency-periodogram hot path on one MI355X.

Default workload: the whole method on one series shaped like the paper's
largest analyses - N = 10^4 irregular times over 20000 d with nightly and
seasonal gaps, 12 injected sinusoids + noise.  One step = one full pass:
Phase 1 residual scans on F = 4e6 grid frequencies up to 5 c/d (base model
grown until the FAP_0 stop), a pool capped at 16 candidates, all 65535
subsets of the pool refined (8 Gauss-Newton steps each) in Phase 2, and the
Phase 3 cascade.  Inputs are resident in HBM before the timed region.  The
headline is the float32 form (float32 trig and sums, the base-column sums on
the float16 matrix cores with split operands, float64 phase reduction,
solves and re-scoring); the float64 form is timed beside it.

value = scan points (N x F per Phase 1 scan) per second of the whole pass;
tuples/s = refined subsets per second of the same pass.

Roofline (dominant kernel group: the Phase 1 scan kernels, one launch per
scan, HIP events on the call's stream): T_roof = max(VALU model, MFMA model,
HBM bytes) per scan, summed over the scans, against the HIP-event time:
  VALU model (lane-op slots per (frequency, sample) pair; chip issue peak
  256 CU x 64 lanes x 2.4 GHz = 39.3 Tops/s):
    trig generation, one complex rotation per pair       4
    second-order terms w~c, <w~ c c>, <w~ c s>            3
    data-column sums <w~ r_b c>, <w~ r_b s>               2
    base-column sums 2(2m+1), where they run on the VALU  4m + 2
  MFMA model: the base-column sums as split-float16 products (three per sum,
  2 flops each) against the float16 dense peak of 2.5 PFLOP/s.
The sums themselves are 2 S = 8m + 12 flops per pair (S = 4m + 6 sums).

Extra keys: the residual scan (N = 2000, m = 4, F = 10^6), the tuple ascent
(65536 tuples of 1..6 frequencies, N = 1000, 20 steps) in both forms, and the
float64 oracle timed on the host cores (one process, then one per core).

--workload residual | batched | tuples: that workload alone as the headline.
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

# MI355X: issue and published peaks
PEAK_VALU_OPS = 256 * 64 * 2.4e9   # VALU lane-op slots per second (one instruction per lane and cycle)
PEAK_F16_MFMA = 2.5e15             # flop/s, dense float16 matrix cores
PEAK_F64_MFMA = 78.6e12            # flop/s, float64 matrix cores
PEAK_HBM = 8.0e12                  # B/s

# HBM traffic per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE passes (KiB per dispatch), scaled by
# what the same counters read for a plain device copy of known size (FETCH x2.0, WRITE x1.0).  A
# figure is only used while the kernel source and its compile flags still have the hash it was
# measured with (source_hash); keyed by (kernel, workload).
COUNTER_SCALE = {"fetch": 2.0, "write": 1.0}
TRAFFIC = {
    # float32 Phase 1 scans of the full pass, averaged over its 18 launches (scan_f16x3_kernel x16,
    # scan_f32_kernel x2)
    "full_fp32_phase1_scans": {"src": {"scan_f16x3.hip": "57f1b384d05695681b3cf4ebf052560541298357",
                                        "scan_f32.hip": "ce2bad490820f493b1da42222c1e35694aabec42"},
                               "fetch_kib": 20029.4, "write_kib": 35173.7},
}


def source_hash(src):
    """sha1 of a kernel source file followed by its per-file compile flags."""
    import hashlib
    from paper_1309_0100_amd import build
    with open(os.path.join(build.CSRC, src), "rb") as fh:
        h = hashlib.sha1(fh.read())
    h.update(" ".join(build.FILE_FLAGS.get(src, [])).encode())
    return h.hexdigest()


def traffic_bytes(key):
    """Measured HBM bytes per launch, or None when not measured for the current sources."""
    t = TRAFFIC.get(key)
    if not t or any(source_hash(src) != sha for src, sha in t["src"].items()):
        return None
    return 1024.0 * (COUNTER_SCALE["fetch"] * t["fetch_kib"] + COUNTER_SCALE["write"] * t["write_kib"])


def f32_auto_valu_max_kp():
    """Largest 2m + 2 that the float32 form gives to its VALU kernel (tuning table, else the default)."""
    try:
        with open(os.path.join(ROOT, "paper_1309_0100_amd", "tuning.json")) as fh:
            return int(json.load(fh).get("scan_f32_auto", {}).get("valu_max_kp", 6))
    except (OSError, ValueError):
        return 6


def scan_kernel(m, fp32):
    if not fp32:
        return "scan_f64_kernel"
    return "scan_f32_kernel" if 2 * m + 2 <= f32_auto_valu_max_kp() else "scan_f16x3_kernel"


def scan_model(m, fp32):
    """Per (frequency, sample) pair: VALU slots, MFMA flops and the MFMA peak of the kernel that scans a
    base of m frequencies (see the module docstring)."""
    kern = scan_kernel(m, fp32)
    K = 2 * m + 1
    if kern == "scan_f16x3_kernel":
        return kern, 8.0, 12.0 * K, PEAK_F16_MFMA
    return kern, 8.0 + 2.0 * K, 0.0, PEAK_F16_MFMA


def scan_roofline(ms_list, N, F, t_meas, fp32, traffic=None):
    """Roofline of a list of scans (base sizes ms_list, one launch each) measured at t_meas seconds."""
    P = float(N) * float(F)
    t_roof, t_serial, slots, mflops, kerns = 0.0, 0.0, 0.0, 0.0, {}
    for m in ms_list:
        kern, v, mf, mpk = scan_model(m, fp32)
        kerns[kern] = kerns.get(kern, 0) + 1
        tv, tm = v * P / PEAK_VALU_OPS, mf * P / mpk
        th = (traffic or 0.0) / PEAK_HBM
        t_roof += max(tv, tm, th)
        # at two waves per SIMD the VALU and MFMA times of a wave add (timing probe: 16x16x32 float16
        # MFMAs interleaved with float32 FMAs take the sum of both alone), so the bound of a kernel
        # that issues both is their sum
        t_serial += max(tv + tm, th)
        slots += v * P
        mflops += mf * P
    achieved = slots / t_meas
    extra = {}
    if fp32:
        # the slot model fixed for the float32 form before the first measurement: float64 phase (3),
        # hardware sin and cos at quarter rate (2 x 4), double angle (3) = 14 per pair, every sum on
        # the matrix cores
        extra["frac_fixed_14_slot_model"] = 14.0 * P * len(ms_list) / PEAK_VALU_OPS / t_meas
        extra["frac_serial_pipes"] = t_serial / t_meas
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_OPS / 1e12, "unit": "Tops/s",
            "frac": t_roof / t_meas, **extra, "traffic": traffic,
            "kernel": " + ".join(f"{k} x{n}" for k, n in sorted(kerns.items())),
            "kernel_ms": t_meas * 1e3, "launches": len(ms_list),
            "mfma_frac": (mflops / t_meas / PEAK_F16_MFMA) if mflops else 0.0,
            "sum_flops_per_pair": [8 * m + 12 for m in ms_list],
            "algorithmic": "VALU lane-op slots per (frequency, sample) pair: 8 (complex rotation 4 giving the "
                           "sqrt(w~)-weighted cos and sin, second-order sums <cos^2> and <cos sin> 2 (<sin^2> from "
                           "eq. idn), data-column sums 2) + 2(2m+1) base-column sums where they run on the VALU; "
                           "split-float16 kernel: base-column sums on the float16 matrix cores (12(2m+1) flops per "
                           "pair vs 2.5 PFLOP/s); T_roof = sum over scans of max(VALU, MFMA, HBM), frac = "
                           "T_roof / HIP-event time; achieved = model slots / HIP-event time"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["full", "residual", "batched", "tuples", "report"], default="full")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target oracle time of each CPU baseline leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline workload only")
    ap.add_argument("--fp64-steps", type=int, default=3,
                    help="timed passes of the float64 form beside the headline (0: not run)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes 5 times (the reference kernel "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def copy_reference(nbytes):
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / 5
    print(json.dumps({"copy_bytes": 4 * n, "seconds_per_copy": el, "GB_per_s": 2 * 4 * n / el / 1e9}), flush=True)


def timed(ctx, step, steps, warmup):
    """Wall time per step over `steps` timed steps (after `warmup`), and the
    HIP-event time (seconds per step) of the library's kernel groups by kind."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kinds = ctx.profile_read_kinds()
    ctx.profile(False)
    per = {k: (ms / 1e3 / max(steps, 1), n / max(steps, 1)) for k, (ms, n) in kinds.items()}
    return el / steps, per


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ------------------------------------------------------------------ full pass
def full_leg(ctx, s, dev, fp32, steps, warmup):
    import torch
    from paper_1309_0100_amd import fredec, pipeline
    prec = fredec.FP32 if fp32 else fredec.FP64
    t, x, w = (torch.as_tensor(a, device=dev) for a in (s.t, s.x, s.w))
    out = {}

    def step():
        out["r"] = pipeline.run(ctx, t, x, w, s.df, s.F, pool_cap=16, refine_steps=8, precision=prec)

    sec, per = timed(ctx, step, steps, warmup)
    res = out["r"]
    # one more pass with the series starting in host memory: the copies to the device (pageable
    # float64 arrays, 24 N bytes) and the pass, timed together (the pass's results come back to the
    # host inside pipeline.run, so this is the whole job as a caller with host data sees it)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th, xh, wh = (torch.as_tensor(a).to(dev) for a in (s.t, s.x, s.w))
    torch.cuda.synchronize()
    h2d = time.perf_counter() - t0
    pipeline.run(ctx, th, xh, wh, s.df, s.F, pool_cap=16, refine_steps=8, precision=prec)
    torch.cuda.synchronize()
    e2e = time.perf_counter() - t0
    n = res.pool.size
    t_scan = per["scan"][0]
    roof = scan_roofline(list(range(res.n_scans)), s.N, s.F, t_scan, fp32,
                         traffic_bytes("full_fp32_phase1_scans") if fp32 else None)
    # Phase 2 Gauss-Newton Gram passes (float64 matrix cores): C(C+1) flops per (tuple, sample) and pass,
    # C = 4n + 2 columns, over the 8 per-subset passes of the 9 (the first is gathered from the pool's
    # Gram: its two timed groups, the pool Gram and the gather, take under a millisecond)
    from math import comb
    C = np.array([4 * k + 2 for k in range(1, n + 1)], np.float64)
    cnt = np.array([comb(n, k) for k in range(1, n + 1)], np.float64)
    gram_flops = float(np.sum(cnt * C * (C + 1))) * s.N
    t_gram = per["gram"][0]
    n_gram = 8
    leg = {"seconds_per_pass": sec, "points_per_s": s.N * s.F * res.n_scans / sec,
           "tuples_per_s": ((1 << n) - 1) / sec, "n_scans": res.n_scans, "pool_size": n,
           "n_solutions": len(res.solutions), "truncated": res.truncated,
           "kernel_seconds_per_pass": {k: v[0] for k, v in per.items()},
           "launch_groups_per_pass": {k: v[1] for k, v in per.items()},
           "end_to_end_from_host": {"seconds": e2e, "h2d_ms": h2d * 1e3, "input_bytes": 24 * s.N,
                                    "points_per_s": s.N * s.F * res.n_scans / e2e},
           "roofline": roof,
           "phase2_gram_roofline": {"bound": "mfma", "kernel": "tuple_gram_kernel",
                                    "achieved": gram_flops * n_gram / t_gram / 1e12 if t_gram else None,
                                    "peak": PEAK_F64_MFMA / 1e12, "unit": "TFLOP/s",
                                    "frac": gram_flops * n_gram / t_gram / PEAK_F64_MFMA if t_gram else None,
                                    "passes": n_gram, "ms_per_gram_pass": t_gram / max(n_gram, 1) * 1e3,
                                    "algorithmic": "C(C+1) flop per (tuple, sample) per Gauss-Newton Gram pass, "
                                                   "C = 4n+2 columns, every subset of the pool, 8 passes "
                                                   "(the first of 9 gathered from the pool Gram)"}}
    return leg, res


def full_errors(ctx, s, dev, res32, res64):
    """Error of the float32 pass: its decisions against the float64 pass, its refined l-table against
    the float64 pass and against the oracle's Gauss-Newton refinement on sampled subsets, and the
    float32 statistic of the final Phase 1 scan against the float64 one at every grid point."""
    import torch
    import oracle as O
    from paper_1309_0100_amd import fredec
    e = {"pool_identical": bool(np.array_equal(res32.pool, res64.pool)),
         "n_scans_identical": res32.n_scans == res64.n_scans,
         "solutions_identical": [sl.mask for sl in res32.solutions] == [sl.mask for sl in res64.solutions]}
    if res32.ltab is not None and res64.ltab is not None and res32.ltab.size == res64.ltab.size:
        a, b = res32.ltab, res64.ltab
        ok = np.isfinite(a) & np.isfinite(b) & (b > 0)
        e["ltab_rel_err_fp32_vs_fp64"] = float(np.max(np.abs(a[ok] - b[ok]) / b[ok]))
    nrm = O.normalize(s.t, s.x, s.w)
    n = res64.pool.size
    rng = np.random.default_rng(7)
    masks = [1 << k for k in range(min(n, 3))] + [(1 << n) - 1] + rng.integers(1, 1 << n, size=4).tolist()
    err = {"fp32": 0.0, "fp64": 0.0}
    for S in masks:
        mem = [k for k in range(n) if S >> k & 1]
        r = O.gn_refine(nrm, res64.pool[mem], 8)
        if r.flag:
            continue
        for k, res in (("fp32", res32), ("fp64", res64)):
            err[k] = max(err[k], abs(res.ltab[S] - r.l) / r.l)
    e["refined_l_rel_err_vs_oracle"] = err
    e["refined_subsets_checked"] = len(masks)
    # every Phase 1 scan of the pass (scan k has the first k SLICK frequencies as its base) in both
    # forms, compared at every grid point where neither is flagged
    t, x, w = (torch.as_tensor(a, device=dev) for a in (s.t, s.x, s.w))
    per_scan = []
    for k in range(res64.n_scans):
        base = res64.base[:k]
        z32, f32_, _, _ = ctx.scan_series(t, x, w, base, s.df, s.F, precision=fredec.FP32)
        z64, f64_, _, _ = ctx.scan_series(t, x, w, base, s.df, s.F, precision=fredec.FP64)
        good = ((f32_ & ~64) == 0) & (f64_ == 0) & torch.isfinite(z64)
        rel = (z32 - z64).abs() / torch.clamp(z64.abs(), min=1.0)
        per_scan.append((float(rel[good].max().item()), int(good.sum().item()), int(((f32_ & 64) != 0).sum().item())))
    e["scans_z_rel_err_fp32_vs_fp64"] = [v[0] for v in per_scan]
    e["scans_z_rel_err_fp32_vs_fp64_max"] = max(v[0] for v in per_scan)
    e["scans_points_compared"] = sum(v[1] for v in per_scan)
    e["scans_points_rescored_fp32"] = sum(v[2] for v in per_scan)
    e["last_scan_m"] = int(res64.n_scans - 1)
    e["last_scan_z_rel_err_fp32_vs_fp64"] = per_scan[-1][0]
    return e


def convergence_leg(ctx, s, dev, res, n_masks=4096):
    """Gauss-Newton (fredec_tuples, refine_steps R) against the fixed-step
    preconditioned ascent (fredec_ascent, S steps) on pool subsets of the full
    pass, both from the pool frequencies: the share of subsets whose
    Gauss-Newton iteration stopped on the step tolerance (max |df| T_eff <
    1e-10) within R passes, and each method's largest distance (times T_eff)
    from the R = 16 Gauss-Newton frequencies over the subsets that stay in
    that basin (within 0.1 / T_eff)."""
    import torch
    from paper_1309_0100_amd import fredec
    pool = res.pool
    n = pool.size
    rng = np.random.default_rng(17)
    masks = np.unique(rng.integers(1, 1 << n, size=n_masks).astype(np.uint64))
    t, x, w = (torch.as_tensor(a, device=dev) for a in (s.t, s.x, s.w))
    T = float(ctx.normalize(t, x, w)[3][0, 4].item())
    mem = [[k for k in range(n) if int(m) >> k & 1] for m in masks]
    gn = {}
    for R in (1, 2, 4, 8, 16):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        l, z, f, fl = ctx.tuples(t, x, w, pool, masks=masks, refine_steps=R)
        torch.cuda.synchronize()
        gn[R] = (time.perf_counter() - t0, f.cpu().numpy(), fl.cpu().numpy())
    ref = gn[16][1]
    out = {"subsets": int(masks.size), "pool_size": int(n), "gauss_newton": {}, "ascent": {}}
    for R, (sec, f, fl) in gn.items():
        d = np.array([np.max(np.abs(f[k, m] - ref[k, m])) for k, m in enumerate(mem)]) * T
        ok = np.isfinite(d) & (d < 0.1)
        out["gauss_newton"][str(R)] = {"passes": R + 1, "ms": sec * 1e3,
                                       "converged_share": float(np.mean((fl & fredec.FLAG_CONVERGED) != 0)),
                                       "max_dist_to_R16_times_T_eff": float(d[ok].max(initial=0.0)),
                                       "median_dist": float(np.median(d[ok])) if ok.any() else None,
                                       "p90_dist": float(np.percentile(d[ok], 90)) if ok.any() else None,
                                       "share_within_1e-8": float(np.mean(d[ok] < 1e-8))}
    toff = np.concatenate([[0], np.cumsum([len(m) for m in mem])]).astype(np.int64)
    f0 = np.concatenate([pool[m] for m in mem])
    for S in (5, 10, 20, 40):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fa, za, la, fla = ctx.ascent(t, x, w, f0, toff, steps=S, clamp=0.1)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        fa = fa.cpu().numpy()
        d = np.array([np.max(np.abs(fa[toff[k]:toff[k + 1]] - ref[k, m])) for k, m in enumerate(mem)]) * T
        ok = np.isfinite(d) & (d < 0.1)
        out["ascent"][str(S)] = {"steps": S, "ms": sec * 1e3, "basin_share": float(np.mean(ok)),
                                 "max_dist_to_gn_times_T_eff": float(d[ok].max(initial=0.0)),
                                 "median_dist": float(np.median(d[ok])) if ok.any() else None,
                                 "p90_dist": float(np.percentile(d[ok], 90)) if ok.any() else None,
                                 "share_within_1e-8": float(np.mean(d[ok] < 1e-8))}
    return out


def report_leg(ctx, s, dev, res, gl_F=100_000, gl_steps=8):
    """The per-solution report (Sect. 6) and Phase 4 of the full pass, then
    the global-local residual periodogram (Sect. 2) of the residual-scan
    series: timings, the float64 Gram roofline of the global-local Gram
    passes, and errors against the oracle on samples."""
    import torch
    import oracle as O
    from paper_1309_0100_amd import fredec, pipeline, synth
    out = {}
    t, x, w = (torch.as_tensor(a, device=dev) for a in (s.t, s.x, s.w))
    sols = [sl.freqs for sl in res.solutions]
    for prec, name in ((fredec.FP32, "fp32"), (fredec.FP64, "fp64")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fap, zr, jr = ctx.residual_fap(t, x, w, sols, s.df, s.F, precision=prec)
        sec = time.perf_counter() - t0
        out[f"residual_fap_{name}"] = {"solutions": len(sols), "seconds": sec, "scan_points_per_s":
                                       len(sols) * s.N * s.F / sec, "median_fap": float(np.median(fap)),
                                       "highest_residual_z": float(np.nanmax(zr))}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rows = pipeline.phase4(ctx, t, x, w, sols)
    sec = time.perf_counter() - t0
    nrm = O.normalize(s.t, s.x, s.w)
    ref = O.phase4(nrm, sols)
    out["phase4"] = {"solutions": len(sols), "ms": sec * 1e3, "kept": int(sum(r.keep for r in rows)),
                     "order_equal_oracle": [r.index for r in rows] == [r["index"] for r in ref],
                     "max_abs_vuong_err_vs_oracle": float(max(abs(a.vuong - b["vuong"]) for a, b in zip(rows, ref)))}
    # global-local periodogram: residual-scan series, base = its 4 injected frequencies
    sr = synth.residual()
    df = 2.0 / gl_F
    tr, xr, wr = (torch.as_tensor(a, device=dev) for a in (sr.t, sr.x, sr.w))
    ctx.global_local(tr, xr, wr, sr.base_f, df, 4096, refine_steps=gl_steps)   # warm up
    torch.cuda.synchronize()
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    z, fl, lb, fb = ctx.global_local(tr, xr, wr, sr.base_f, df, gl_F, refine_steps=gl_steps)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    kinds = ctx.profile_read_kinds()
    ctx.profile(False)
    m = sr.base_f.size
    C = 4 * (m + 1) + 2
    n_passes = kinds["gram"][1]
    # 1 + steps Gauss-Newton Gram passes of the trial tuples at most (a tuple that stops early skips the
    # rest, so this is an upper bound of the work and of the fraction)
    gram_flops = float(C * (C + 1)) * sr.N * gl_F * (gl_steps + 1)
    t_gram = kinds["gram"][0] / 1e3
    zc, flc = z.cpu().numpy(), fl.cpu().numpy()
    idx = np.linspace(0, gl_F - 1, 12).astype(np.int64)
    r = O.global_local_scan(sr.t, sr.x, sr.w, sr.base_f, df, gl_F, refine_steps=gl_steps, idx=idx)
    good = r.flags == 0
    out["global_local"] = {"workload": f"N={sr.N}, m={m}, F={gl_F} to 2 c/d, {gl_steps} Gauss-Newton steps per point",
                           "seconds": sec, "grid_points_per_s": gl_F / sec,
                           "kernel_ms": {k: v[0] for k, v in kinds.items()}, "gram_groups": n_passes,
                           "roofline": {"bound": "mfma", "kernel": "tuple_gram_kernel", "unit": "TFLOP/s",
                                        "achieved": gram_flops / t_gram / 1e12 if t_gram else None,
                                        "peak": PEAK_F64_MFMA / 1e12,
                                        "frac": gram_flops / t_gram / PEAK_F64_MFMA if t_gram else None,
                                        "algorithmic": f"C(C+1) flop per (tuple, sample) per Gauss-Newton Gram pass, "
                                                       f"C = 4(m+1)+2 = {C}, 1 + {gl_steps} passes per grid point "
                                                       f"(an upper bound: a tuple that stops early skips the rest)"},
                           "points_checked": int(good.sum()),
                           "flags_equal_oracle": bool(np.array_equal(flc[idx], r.flags)),
                           "max_rel_err_vs_oracle": float(np.max(np.abs(zc[idx][good] - r.z[good]) /
                                                                 np.maximum(np.abs(r.z[good]), 1.0)))}
    return out


# ------------------------------------------------------------------ residual scan
def residual_leg(ctx, s, dev, fp32, steps, warmup):
    import torch
    from paper_1309_0100_amd import fredec
    prec = fredec.FP32 if fp32 else fredec.FP64
    t, x, w = (torch.as_tensor(a, device=dev) for a in (s.t, s.x, s.w))
    plan, pout = ctx.scan_plan(np.array([0, s.N], np.int64), s.base_f, np.array([0, s.base_f.size], np.int64),
                               [s.df], [s.F], prec)
    # FAP_1 listing threshold, W = f_max T_eff (Sect. 2), T_eff from the library's normalisation
    T_eff = float(ctx.normalize(t, x, w)[3][0, 4].item())
    zc1 = float(fredec.zcrit(s.F * s.df * T_eff, 1, 0.1)[1])
    peaks = {}

    def step():
        plan.run(t, x, w, pout)
        peaks["p"] = ctx.peaks(pout[0], pout[1], zc1)

    sec, per = timed(ctx, step, steps, warmup)
    t_scan = per["scan"][0]
    fl = pout[1]
    return {"value": s.N * s.F / sec, "unit": "points/s", "ms_per_step": sec * 1e3,
            "roofline": scan_roofline([s.base_f.size], s.N, s.F, t_scan, fp32),
            "kernel_ms": {k: v[0] * 1e3 for k, v in per.items()},
            "rescored_points": int(((fl & 64) != 0).sum().item()),
            "n_peaks_above_fap1": int(len(peaks["p"][0]))}, pout[0].cpu().numpy(), pout[1].cpu().numpy()


def residual_error(s, z, fl, n_idx=1500):
    import oracle as O
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([rng.integers(0, s.F, size=n_idx),
                                    np.argsort(-np.nan_to_num(z["fp64"], nan=-1.0))[:50]])).astype(np.int64)
    r = O.scan(s.t, s.x, s.w, s.base_f, s.df, s.F, idx=idx)
    good = r.flags == 0
    out = {}
    for k, v in z.items():
        e = np.abs(v[idx][good] - r.z[good]) / np.maximum(np.abs(r.z[good]), 1.0)
        out[k] = float(e.max())
        out[k + "_flags_equal"] = bool(np.array_equal(fl[k][idx] & ~np.uint8(64), r.flags))
    out["points_checked"] = int(good.sum())
    return out


# ------------------------------------------------------------------ tuples
def tuples_leg(ctx, dev, fp32, steps, n_steps=20):
    import torch
    from paper_1309_0100_amd import fredec, synth
    prec = fredec.FP32 if fp32 else fredec.FP64
    s = synth.tuples_series()
    t, x, w = (torch.as_tensor(a, device=dev) for a in (s.t, s.x, s.w))
    z, fl, _, _ = ctx.scan_series(t, x, w, [], s.df, s.F)
    idx, zp = ctx.peaks(z, fl, 0.0)
    top = idx[np.lexsort((idx, -zp))[:12]]
    peaks = (top + 1).astype(np.float64) * s.df
    f0, toff = synth.tuples_draw(peaks, n_tuples=65536)
    nt = toff.size - 1
    f0d = torch.as_tensor(f0, device=dev)
    # the one-shot call (host planning of the 65536 tuples, descriptor upload, workspace) for reference
    sec_call, _ = timed(ctx, lambda: ctx.ascent(t, x, w, f0d, toff, steps=n_steps, clamp=0.1, precision=prec),
                        steps, 1)
    # the prepared plan: eager launches give the per-kind HIP-event times; the timed value replays the
    # plan's launches captured in a HIP graph (each call starts again from the same frequencies, copied
    # in before the replay)
    plan, out = ctx.ascent_plan(s.N, toff, steps=n_steps, clamp=0.1, precision=prec)
    f = f0d.clone()

    def eager():
        f.copy_(f0d)
        plan.run(t, x, w, f, out)

    _, per = timed(ctx, eager, steps, 1)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(t, x, w, f, out)

    def replay():
        f.copy_(f0d)
        g.replay()

    sec, _ = timed(ctx, replay, steps, 1)
    torch.cuda.synchronize()
    res = {"r": (f.clone(), out[0].clone(), out[1].clone(), out[2].clone())}
    plan.close()
    nn = np.diff(toff).astype(np.float64)
    C = 2 * nn + 2
    # per (tuple, sample) and pass: the Gram lower triangle C(C+1)/2 multiply-adds less the n <w sin^2>
    # that eq. idn gives from <w> - <w cos^2>, + 12 slots of trig per member (offset rotation 8 + complex
    # product 4)
    slots = float(np.sum(C * (C + 1) / 2 - nn + 12 * nn)) * s.N * (n_steps + 1)
    t_gram = per["gram"][0]
    fa, zz, ll, ff = res["r"]
    return {"value": nt / sec, "unit": "tuples/s", "tuple_steps_per_s": nt * n_steps / sec,
            "ms_per_call": sec * 1e3, "ms_per_one_shot_call": sec_call * 1e3,
            "kernel_ms": {k: v[0] * 1e3 for k, v in per.items()},
            "roofline": {"bound": "alu", "kernel": "tuple_gram_lanes_kernel", "achieved": slots / t_gram / 1e12,
                         "peak": PEAK_VALU_OPS / 1e12, "unit": "Tops/s", "frac": slots / t_gram / PEAK_VALU_OPS,
                         "algorithmic": "VALU lane-op slots per (tuple, sample) and pass: C(C+1)/2 - n Gram "
                                        "multiply-adds (C = 2n+2; the n <w sin^2> follow from eq. idn) + 12 per member "
                                        "for its trig; 21 passes per call; the kernel also makes the forward solve"}}, \
        (s, f0, toff, fa.cpu().numpy(), zz.cpu().numpy())


def tuples_error(data, n_check=24):
    import oracle as O
    s, f0, toff, fa, zz = data
    nrm = O.normalize(s.t, s.x, s.w)
    err_f, err_z = 0.0, 0.0
    nt = toff.size - 1
    ks = range(0, nt, max(1, nt // n_check))
    for k in ks:
        fr, zr, lr = O.ascent(nrm, f0[toff[k]:toff[k + 1]], steps=20, clamp=0.1)
        if not np.isfinite(zr):
            continue
        err_f = max(err_f, float(np.max(np.abs(fa[toff[k]:toff[k + 1]] - fr)) * nrm.T_eff))
        err_z = max(err_z, float(abs(zz[k] - zr) / max(abs(zr), 1.0)))
    return {"z": err_z, "f_times_T_eff": err_f, "tuples_checked": len(ks)}


# ------------------------------------------------------------------ batched
def batched_leg(ctx, b, dev, fp32, steps, warmup):
    import torch
    from paper_1309_0100_amd import fredec
    prec = fredec.FP32 if fp32 else fredec.FP64
    t, x, w = (torch.as_tensor(a, device=dev) for a in (b.t, b.x, b.w))
    plan, out = ctx.scan_plan(b.soff, b.base_f, b.boff, b.df, b.F, prec)

    def step():
        plan.run(t, x, w, out)

    # eager launches of the prepared plan give the per-kind HIP-event times; the timed value replays
    # its launches captured in a HIP graph
    _, per = timed(ctx, step, steps, warmup)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(t, x, w, out)
    sec, _ = timed(ctx, g.replay, steps, 1)
    Ns = np.diff(b.soff).astype(np.float64)
    ms = np.diff(b.boff)
    points = float(np.sum(Ns * np.asarray(b.F)))
    t_scan = per["scan"][0]
    t_roof = 0.0
    for m in np.unique(ms):
        P = float(np.sum(Ns[ms == m] * np.asarray(b.F)[ms == m]))
        _, v, mf, mpk = scan_model(int(m), fp32)
        t_roof += max(v * P / PEAK_VALU_OPS, mf * P / mpk)
    return {"value": points / sec, "ms_per_step": sec * 1e3, "pairs": points,
            "kernel_ms": {k: v[0] * 1e3 for k, v in per.items()},
            "roofline": {"bound": "alu", "frac": t_roof / t_scan, "kernel": "all scan kernel launches",
                         "unit": "Tops/s", "peak": PEAK_VALU_OPS / 1e12, "kernel_ms": t_scan * 1e3},
            "rescored_points": int(((out[1] & 64) != 0).sum().item())}, out[0].clone(), out[1].clone()


# ------------------------------------------------------------------ CPU baseline
def _oracle_block(args):
    """One block of the oracle's scan (worker of the CPU baseline)."""
    try:
        from threadpoolctl import threadpool_limits
        lim = threadpool_limits(limits=1)
    except Exception:  # pragma: no cover
        lim = None
    import oracle as O
    t, x, w, base, df, F, idx = args
    O.scan(t, x, w, base, df, F, idx=idx)
    del lim
    return idx.size


def cpu_baseline(s, seconds):
    """The float64 oracle on a bounded sample of the full pass's scans: base models of m = 0 .. 12
    frequencies (the injected frequencies, strongest first, as stand-ins for the SLICK frequencies), 64
    random grid points per scan per block; first one process, then one process per core (at most 16).
    Runs before anything touches the GPU (the worker processes are forked)."""
    import multiprocessing as mp
    order = np.argsort(-s.true_A)
    bases = [s.true_f[order[:m]] for m in range(s.true_f.size + 1)]
    rng = np.random.default_rng(1)
    blocks = []
    for rep in range(200):
        for base in bases:
            idx = np.sort(rng.choice(s.F, size=64, replace=False)).astype(np.int64)
            blocks.append((s.t, s.x, s.w, base, s.df, s.F, idx))
    # one process
    t0 = time.perf_counter()
    done1 = 0
    for b in blocks:
        done1 += _oracle_block(b)
        if time.perf_counter() - t0 > seconds:
            break
    el1 = time.perf_counter() - t0
    # one process per core
    P = max(1, min(16, os.cpu_count() or 1))
    t0 = time.perf_counter()
    doneP = 0
    with mp.get_context("fork").Pool(P) as pool:
        for k in pool.imap_unordered(_oracle_block, blocks, chunksize=1):
            doneP += k
            if time.perf_counter() - t0 > seconds:
                pool.terminate()
                break
    elP = time.perf_counter() - t0
    return {"value": s.N * done1 / el1, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"{done1} grid points of the full-pass series (N={s.N}, F={s.F}) in blocks of 64 random "
                      f"points, cycling over base models of m = 0..{len(bases) - 1} injected frequencies; "
                      f"{el1:.1f} s in one process (BLAS threads = 1)",
            "all_cores": {"value": s.N * doneP / elP, "unit": "points/s", "cores": P,
                          "sample": f"{doneP} grid points, same blocks, {P} processes, {elP:.1f} s"}}


# ------------------------------------------------------------------ main
def main():
    args = parse()
    if args.copy_bytes:
        copy_reference(args.copy_bytes)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 "
                                   "(multi-GPU sharding is a design note, not built)"}))
        sys.exit(2)
    from paper_1309_0100_amd import synth
    cpu = None
    if args.workload == "full" and not args.no_cpu:
        progress("oracle on the host cores")
        cpu = cpu_baseline(synth.full(), args.cpu_seconds)
    import torch
    from paper_1309_0100_amd import fredec
    dev = torch.device("cuda", 0)
    ctx = fredec.Context(0)
    res = {"metric": METRIC, "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    extra = not args.no_extra

    if args.workload == "full":
        s = synth.full()
        progress("full pass, float32 form")
        leg32, r32 = full_leg(ctx, s, dev, True, args.steps, args.warmup)
        leg64 = r64 = None
        if args.fp64_steps > 0:
            progress("full pass, float64 form")
            leg64, r64 = full_leg(ctx, s, dev, False, min(args.steps, args.fp64_steps), min(args.warmup, 1))
        res.update({"value": leg32["points_per_s"], "ms_per_step": leg32["seconds_per_pass"] * 1e3,
                    "tuples_per_s": leg32["tuples_per_s"], "dtype": "f32 (f16x3 MFMA)",
                    "config": {"workload": "full FREDEC pass: N=10^4 over 20000 d (nightly + seasonal gaps), 12 "
                                           "sinusoids; Phase 1 scans on F=4e6 to 5 c/d until the FAP_0 stop, pool "
                                           "cap 16, all 65535 subsets refined (8 Gauss-Newton steps), Phase 3",
                               "N": s.N, "F": s.F, "pool_cap": 16, "form": "fp32"},
                    "roofline": leg32["roofline"], "fp32_form": leg32})
        if leg64 is not None:
            res["fp64_form"] = dict(leg64, steps=min(args.steps, args.fp64_steps))
            res["speedup_fp32_over_fp64"] = leg64["seconds_per_pass"] / leg32["seconds_per_pass"]
            progress("errors of the float32 pass")
            res["errors"] = full_errors(ctx, s, dev, r32, r64)
        if extra:
            progress("Gauss-Newton against ascent on pool subsets")
            res["gn_vs_ascent"] = convergence_leg(ctx, s, dev, r32)
            progress("report: residual FAP, Phase 4, global-local periodogram")
            res["report"] = report_leg(ctx, s, dev, r32)
            progress("residual scan (N=2000, m=4, F=1e6)")
            sr = synth.residual()
            legs, zs, fls = {}, {}, {}
            for k, fp32 in (("fp32", True), ("fp64", False)):
                legs[k], zs[k], fls[k] = residual_leg(ctx, sr, dev, fp32, 20, 5)
            legs["speedup_fp32_over_fp64"] = legs["fp64"]["ms_per_step"] / legs["fp32"]["ms_per_step"]
            legs["max_rel_err_vs_oracle"] = residual_error(sr, zs, fls)
            res["residual_scan"] = legs
            progress("tuple ascent (65536 tuples, 20 steps)")
            tl = {}
            for k, fp32 in (("fp64", False), ("fp32", True)):
                tl[k], data = tuples_leg(ctx, dev, fp32, 3)
                tl[k]["max_err_vs_oracle"] = tuples_error(data)
            tl["speedup_fp32_over_fp64"] = tl["fp64"]["ms_per_call"] / tl["fp32"]["ms_per_call"]
            res["tuples"] = tl
        if cpu is not None:
            res["cpu_baseline"] = cpu
    elif args.workload == "residual":
        sr = synth.residual()
        legs, zs, fls = {}, {}, {}
        for k, fp32 in (("fp32", True), ("fp64", False)):
            legs[k], zs[k], fls[k] = residual_leg(ctx, sr, dev, fp32, args.steps, args.warmup)
        res.update({"value": legs["fp32"]["value"], "ms_per_step": legs["fp32"]["ms_per_step"],
                    "dtype": "f32 (f16x3 MFMA)", "roofline": legs["fp32"]["roofline"],
                    "config": {"workload": "residual scan: N=2000 over 4000 d, seasonal gaps, m=4, F=10^6 to 2 c/d",
                               "N": sr.N, "F": sr.F, "m": int(sr.base_f.size), "form": "fp32"},
                    "forms": legs, "speedup_fp32_over_fp64": legs["fp64"]["ms_per_step"] / legs["fp32"]["ms_per_step"],
                    "max_rel_err_vs_oracle": residual_error(sr, zs, fls)})
    elif args.workload == "batched":
        b = synth.batched()
        runs = {k: batched_leg(ctx, b, dev, fp32, args.steps, args.warmup) for k, fp32 in (("fp32", True),
                                                                                          ("fp64", False))}
        legs = {k: r[0] for k, r in runs.items()}
        z32, f32_, z64, f64_ = runs["fp32"][1], runs["fp32"][2], runs["fp64"][1], runs["fp64"][2]
        good = (f32_ == 0) & (f64_ == 0) & torch.isfinite(z64)
        err = (z32 - z64).abs() / torch.clamp(z64.abs(), min=1.0)
        legs["fp32"]["max_rel_err_vs_fp64"] = float(err[good].max().item())
        res.update({"value": legs["fp32"]["value"], "ms_per_step": legs["fp32"]["ms_per_step"],
                    "dtype": "f32 (f16x3 MFMA)", "roofline": legs["fp32"]["roofline"],
                    "config": {"workload": "batched scan: 4096 series, N log-uniform in [50, 5000], m uniform in "
                                           "0..6, F=65536", "series": int(b.soff.size - 1),
                               "samples": int(b.soff[-1]), "form": "fp32"}, "forms": legs})
    elif args.workload == "report":
        from paper_1309_0100_amd import pipeline
        s = synth.full()
        t, x, w = (torch.as_tensor(a, device=dev) for a in (s.t, s.x, s.w))
        r32 = pipeline.run(ctx, t, x, w, s.df, s.F, pool_cap=16, refine_steps=8, precision=fredec.FP32)
        rep = report_leg(ctx, s, dev, r32)
        res.update({"value": rep["global_local"]["grid_points_per_s"], "unit": "grid points/s",
                    "ms_per_step": rep["global_local"]["seconds"] * 1e3, "dtype": "f64",
                    "roofline": rep["global_local"]["roofline"],
                    "config": {"workload": "report of the full pass (residual FAP of every solution, Phase 4) and the "
                                           "global-local periodogram of the residual-scan series (N=2000, m=4, F=1e5)",
                               "form": "fp64"}, "report": rep})
    else:
        tl = {}
        for k, fp32 in (("fp64", False), ("fp32", True)):
            tl[k], data = tuples_leg(ctx, dev, fp32, args.steps)
            tl[k]["max_err_vs_oracle"] = tuples_error(data)
        res.update({"value": tl["fp32"]["value"], "unit": "tuples/s", "ms_per_step": tl["fp32"]["ms_per_call"],
                    "speedup_fp32_over_fp64": tl["fp64"]["ms_per_call"] / tl["fp32"]["ms_per_call"],
                    "dtype": "f32", "roofline": tl["fp32"]["roofline"],
                    "config": {"workload": "tuple ascent: N=1000 over 3000 d, 65536 tuples of 1..6 perturbed peaks, "
                                           "20 steps", "form": "fp32"}, "forms": tl})
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
