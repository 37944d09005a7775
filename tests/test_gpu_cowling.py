"""GPU parity of the fixed-background (Cowling) form against the oracle,
through the C-ABI: the spacetime right-hand sides are zero, the 24 spacetime
fields stay bit-identical through RK4 steps with the filter on, and the GRMHD
fields match the oracle after 10 steps.  Also: diagnostics of a state holding a
NaN report it (non-finite count, NaN extrema, a failed recovery) instead of
a finite value."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from gpu_util import workload, oracle_problem, solver, field_errors, rhs_errors, log  # noqa: E402


def cowling_workload(**grid):
    w = workload("ks_michel_16x16x16", **grid)
    w["phys"]["cowling"] = True
    return w


@pytest.mark.parametrize("size", [(16, 16, 16), (20, 18, 12)])
def test_cowling_rhs_matches_oracle(size):
    log(f"[cowling rhs] grid {size}")
    w = cowling_workload(nr=size[0], nth=size[1], nph=size[2])
    g, pb, U, K0 = oracle_problem(w)
    s = solver(w)
    s.set_state(U, K0)
    dU = torch.tensor(U, device="cuda")
    out = torch.full_like(dU, np.nan)
    s.rhs(dU, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    s.close()
    ref = pb.rhs(U, K0)
    assert np.isfinite(got).all()
    assert np.abs(got[:24]).max() == 0.0
    e = rhs_errors(got, ref, U)
    log("  e_f = " + " ".join(f"{x:.1e}" for x in e[24:]))
    assert e.max() < 1e-11


def test_cowling_ten_steps_match_oracle():
    log("[cowling evolve] 16^3, 10 RK4 steps")
    w = cowling_workload()
    g, pb, U, K0 = oracle_problem(w)
    ref = pb.evolve(U, K0, pb.dt(), 10)
    s = solver(w)
    s.set_state(U, K0)
    s.step(10)
    got = s.get_state()
    d = s.diagnostics()
    s.close()
    assert np.array_equal(got[:24], U[:24])
    assert np.abs(got[24:] - U[24:]).max() > 0
    e = field_errors(got, ref)
    log("  e_f = " + " ".join(f"{x:.1e}" for x in e[24:]))
    assert e.max() < 1e-11
    assert d["nonfinite"] == 0 and d["c2p_fail"] == 0


def test_diagnostics_report_a_nan():
    log("[diagnostics] NaN in one point of S_r, B^r, alpha and K")
    w = workload("ks_michel_16x16x16")
    g, pb, U, K0 = oracle_problem(w)
    s = solver(w)
    s.set_state(U, K0)
    d0 = s.diagnostics()
    V = U.copy()
    V[25, 3, 5, 7] = np.nan
    V[29, 3, 5, 7] = np.nan
    V[17, 9, 2, 4] = np.nan
    V[13, 1, 8, 8] = np.nan  # K enters the Hamiltonian constraint (alpha does not)
    s.set_state(V, K0)
    d1 = s.diagnostics()
    s.close()
    assert d0["nonfinite"] == 0 and np.isfinite(d0["max_abs_divB"]) and np.isfinite(d0["max_W"])
    assert d1["nonfinite"] >= 4 and d1["c2p_fail"] >= 1
    assert np.isnan(d1["max_abs_divB"])
    assert np.isnan(d1["min_alpha"])
    assert np.isnan(d1["ham_linf"]) and np.isnan(d1["ham_l2"])
