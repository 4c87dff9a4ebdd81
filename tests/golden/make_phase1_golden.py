"""Writes tests/golden/phase1_full_reduced.json: the float64 oracle's Phase 1
(Sect. 4.2) and Phase 3 (Sect. 4.4) on a reduced series of the full-pass
shape (synth.full with N = 2000 over 4000 d, F = 2e5 grid points to 5 c/d).

Only the oracle computes anything here.  Each residual scan is split into
blocks of grid frequencies that worker processes hand to oracle.scan (every
grid point is an independent least-squares fit, so the blocks put together
are the oracle's scan of the whole grid); oracle.phase1 takes the decisions.
The Phase 3 table is oracle.phase2 on the pool at the pool frequencies; the
file keeps a seeded sample of it and the survivor set as packed bits.

    python tests/golden/make_phase1_golden.py [processes]
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1309_0100_amd import synth  # noqa: E402

CASE = {"N": 2000, "span": 4000.0, "F": 200_000, "fmax": 5.0}
BLOCK = 4096
_pool = None


def _block(args):
    t, x, w, base, df, F, lo, hi = args
    return lo, O.scan(t, x, w, base, df, F, idx=np.arange(lo, hi, dtype=np.int64))


def scan_parallel(t, x, w, base, df, F):
    jobs = [(t, x, w, base, df, F, lo, min(F, lo + BLOCK)) for lo in range(0, F, BLOCK)]
    parts = dict(_pool.map(_block, jobs))
    los = sorted(parts)
    cat = lambda name: np.concatenate([getattr(parts[lo], name) for lo in los])  # noqa: E731
    first = parts[los[0]]
    return O.ScanResult(cat("z"), cat("flags"), first.l_base, first.T_eff, cat("freqs"), cat("rho"))


def _sample_masks(n):
    rng = np.random.default_rng(1309)
    masks = {0, (1 << n) - 1} | {1 << k for k in range(n)}
    masks |= set(int(v) for v in rng.integers(1, 1 << n, size=1000))
    return sorted(masks)


def main():
    global _pool
    procs = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    s = synth.full(N=CASE["N"], span=CASE["span"], F=CASE["F"], fmax=CASE["fmax"])
    t0 = time.time()
    with mp.get_context("fork").Pool(procs) as pool:
        _pool = pool
        r = O.phase1(s.t, s.x, s.w, s.df, s.F, pool_cap=16, scan_fn=scan_parallel)
    nrm = O.normalize(s.t, s.x, s.w)
    n = r.pool.size
    ltab, _ = O.phase2(nrm, r.pool, refine_steps=0)
    zc = O.zcrit_table(n, r.W, 0.05)
    surv = O.survive_table(ltab, n, s.N, zc)
    maximal = O.maximal_sets(surv, n)
    out = {
        "source": "Float64 oracle (oracle.phase1 with its scans split over grid blocks, oracle.phase2 at the pool "
                  "frequencies, oracle.survive_table / maximal_sets) on synth.full(N=2000, span=4000, F=2e5, "
                  "fmax=5); Phase 1 defaults fap0 = 0.05, fap1 = 0.1, A1 = 1, pool cap 16; Phase 3 fap2 = 0.05. "
                  "Written by tests/golden/make_phase1_golden.py.",
        "case": CASE,
        "pool_index": [int(round(f / s.df)) - 1 for f in r.pool],
        "pool": [float(f) for f in r.pool],
        "pool_z": [float(z) for z in r.pool_z],
        "base_index": [int(round(f / s.df)) - 1 for f in r.base],
        "n_scans": int(r.n_scans),
        "truncated": int(r.truncated),
        "W": float(r.W),
        # l at the pool frequencies of the empty set, every single, the full
        # pool and 1000 seeded random subsets (mask -> l)
        "ltab_sample": {str(S): float(ltab[S]) for S in _sample_masks(n)},
        # survivors of Phase 3: bit S of the little-endian bit string
        "survive_bits": np.packbits(np.asarray(surv, np.uint8), bitorder="little").tobytes().hex(),
        "maximal": [int(v) for v in maximal],
        "seconds": time.time() - t0,
    }
    # grid frequencies are (j + 1) df exactly: the indices identify them
    assert all(f == (j + 1) * s.df for f, j in zip(r.pool, out["pool_index"]))
    assert all(f == (j + 1) * s.df for f, j in zip(r.base, out["base_index"]))
    with open(os.path.join(HERE, "phase1_full_reduced.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"pool {n}, scans {r.n_scans}, maximal {len(maximal)}, {out['seconds']:.0f} s")


if __name__ == "__main__":
    main()
