"""GPU diagnostics of the constraints through the C-ABI (grmhd_diagnostics)
against the oracle (oracle.diagnostics.constraint_norms): the Hamiltonian and
momentum constraints the coupled evolution monitors.

  * Michel + Kerr-Schild at 20 x 18 x 12 (odd and even sizes): the L2 and max
    norms of H and |M| equal the oracle's;
  * exact data on flat space (tests/momentum_case.py: Bowen-York curvature,
    K = k0 x, the balancing momentum density): the library's |M| is as small
    as the oracle's (both converge to 0) and equal to it;
  * the diagnostics leave the evolution alone: with the paper's damped
    recovery (warm-started from the previous one) a run that calls
    grmhd_diagnostics between its steps ends bitwise equal to one that does
    not."""

import numpy as np
import pytest
import torch

from gpu_util import log, oracle_problem, solver, workload
from momentum_case import bowen_york_state, scale

pytestmark = pytest.mark.gpu


def test_constraint_norms_match_oracle():
    from oracle import diagnostics
    for over in (dict(nr=20, nth=18, nph=12), dict(nr=16, nth=16, nph=16)):
        log(f"[constraints] Michel {over}")
        w = workload("ks_michel_16x16x16", **over)
        g, pb, U, K0 = oracle_problem(w)
        s = solver(w)
        s.set_state(U, K0)
        d = s.diagnostics()
        s.close()
        ref = diagnostics.constraint_norms(pb, U)
        log("  GPU " + " ".join(f"{k}={d[k]:.6e}" for k in ref) + "; oracle " +
            " ".join(f"{k}={v:.6e}" for k, v in ref.items()))
        for k in ("ham_l2", "ham_linf"):
            assert abs(d[k] / ref[k] - 1) < 1e-9, k
        for k in ("mom_l2", "mom_linf"):
            assert abs(d[k] / ref[k] - 1) < 1e-10, k


def test_momentum_constraint_vanishes_on_exact_flat_data():
    from oracle import diagnostics
    from paper_2508_18221_amd import Solver, make_grid, make_phys
    from momentum_case import R_IN, R_OUT, TH0, TH1
    log("[constraints] Bowen-York + K gradient + balancing momentum, flat space 32x32x8")
    g, pb, U, f, S = bowen_york_state(32, 32, 8)
    s = Solver(make_grid(32, 32, 8, r_in=R_IN, r_out=R_OUT, th_min=TH0, th_max=TH1), make_phys(M=0.0, a=0.0))
    s.set_state(U, U[13])
    d = s.diagnostics()
    s.close()
    M, Mn = diagnostics.momentum_constraint(pb, U)
    sc = scale(f, S)
    log(f"  |M| max: GPU {d['mom_linf']:.3e}, oracle {Mn.max():.3e} (scale {sc:.3e})")
    assert d["mom_linf"] < 1e-8 * sc
    assert abs(d["mom_linf"] - Mn.max()) < 1e-11 * sc


def test_diagnostics_leave_the_warm_start_alone():
    """Damped recovery (c2p = "damped"): diagnostics between steps must not
    change the trajectory (they recover into scratch memory)."""
    log("[constraints] damped recovery, 16^3: 6 steps with and without diagnostics in between")
    w = workload("ks_michel_16x16x16")
    w["phys"]["c2p"] = "damped"
    g, pb, U, K0 = oracle_problem(w)
    a, b = solver(w), solver(w)
    a.set_state(U, K0)
    b.set_state(U, K0)
    for _ in range(6):
        a.step(1)
        b.step(1)
        b.diagnostics()
    ua, ub = a.get_state(), b.get_state()
    da, db = a.diagnostics(), b.diagnostics()
    a.close()
    b.close()
    assert np.array_equal(ua, ub)
    assert da["c2p_fail"] == db["c2p_fail"]
