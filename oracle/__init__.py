"""FP64 CPU oracle for the FREDEC multifrequency periodogram.

TEST INFRASTRUCTURE ONLY: used by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py.  The product path never imports it.  Every
function is pinned by tests that do not go through this package (lstsq,
scipy's Lomb-Scargle, FFT special cases, invariants, finite differences,
counts); the FAP constants of eq. zFAP and the Phase 1/3 selection rules are
"parity unpinned" against the paper (it does not print them).
"""
from .fredec_ref import *  # noqa: F401,F403
from .fredec_ref import (Normalized, normalize, design, cholesky_checked, lsq, n_dof, grid, scan,  # noqa: F401
                         tuple_fit, tuple_grad, gn_step, gn_refine, ascent, zcrit, zcrit_table, log_fap,
                         local_maxima, phase1, phase2, phase3, goodness, popcount, survive_table,
                         maximal_sets, supersets, residual_fap, loglik_terms, vuong, phase4,
                         global_local_scan)
