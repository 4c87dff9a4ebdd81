"""Whole-pipeline checks of the oracle (Phases 1-3, Sect. 4) on the
two-frequency alias structure of Sect. 7.1.  Qualitative: the paper's exact
series is not available."""
import json
import os

import numpy as np

import oracle as O
from paper_1309_0100_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_two_frequency_alias_example():
    with open(os.path.join(GOLDEN, "two_frequency_alias.json")) as fh:
        g = json.load(fh)
    s = synth.two_frequency_alias()
    nrm = O.normalize(s.t, s.x, s.w)
    r0 = O.scan(s.t, s.x, s.w, [], g["df"], g["F"])
    assert abs(r0.freqs[np.argmax(r0.z)] - g["expect"]["first_scan_argmax"]) < 2 * g["df"]
    res = O.phase1(s.t, s.x, s.w, g["df"], g["F"])
    assert np.allclose(res.pool, g["expect"]["pool_is_alias_comb"], atol=2 * g["df"])
    n = res.pool.size
    ltab, fout = O.phase2(nrm, res.pool, refine_steps=g["refine_steps"])
    surv, maximal, tests = O.phase3(ltab, n, nrm.N, O.zcrit_table(n, res.W, g["fap"]))
    assert tests == 3 ** n - 2 ** n
    sizes = [O.popcount(int(S)) for S in maximal]
    assert sizes == sorted(sizes)
    pairs = [S for S in maximal if O.popcount(int(S)) == 2]
    assert len(pairs) == 1
    members = [k for k in range(n) if pairs[0] >> k & 1]
    f = np.sort(fout[pairs[0], members])
    tol = g["expect"]["tolerance_in_1_over_Teff"] / nrm.T_eff
    assert np.allclose(f, g["expect"]["two_frequency_solution"], atol=tol)
    assert min(sizes) == 2                      # the single alias at 1.0 is not a solution
