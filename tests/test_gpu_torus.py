"""GPU parity on the magnetised Fishbone-Moncrief torus (spin 0.9375,
r in [1.300, 60], Gamma = 13/9, one poloidal loop, +-4 % pressure
perturbation): the library's host initial data against the oracle's, one RHS
evaluation and 10 RK4 steps against the oracle on the same uploaded state."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from gpu_util import workload, solver, oracle_problem, field_errors, rhs_errors, log  # noqa: E402

SMALL = "ks_torus_24x20x16"


@pytest.mark.parametrize("over", [{}, dict(nr=20, nth=18, nph=12)])
def test_torus_initial_data_matches_oracle(over):
    log(f"[torus init] {over or '24x20x16'}")
    w = workload(SMALL, **over)
    g, pb, U, K0 = oracle_problem(w)
    s = solver(w)
    s.init_state()
    got, gk = s.get_state(with_k0=True)
    e = field_errors(got, U)
    log("  e_f = " + " ".join(f"{x:.1e}" for x in e))
    # metric fields: spectral derivatives of gamma_ij near an a = 0.9375 hole
    # (host full matrices vs the oracle's coefficient route); matter: closed form
    assert e[:24].max() < 1e-11
    assert e[24:].max() < 1e-12
    assert np.abs(gk - K0).max() < 1e-11 * np.abs(K0).max()
    s.close()


def test_torus_single_rhs_matches_oracle():
    log("[torus rhs] 24x20x16")
    w = workload(SMALL)
    g, pb, U, K0 = oracle_problem(w)
    s = solver(w)
    s.set_state(U, K0)
    dU = torch.tensor(U, device="cuda")
    out = torch.full_like(dU, np.nan)
    s.rhs(dU, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = pb.rhs(U, K0)
    e = rhs_errors(got, ref, U)
    log("  e_f = " + " ".join(f"{x:.1e}" for x in e))
    assert np.isfinite(got).all()
    assert e.max() < 1e-11
    assert not pb.last_fail.any()
    s.close()


def test_torus_ten_steps_match_oracle():
    log("[torus evolve] 24x20x16, 10 RK4 steps")
    w = workload(SMALL)
    g, pb, U, K0 = oracle_problem(w)
    s = solver(w)
    s.set_state(U, K0)
    s.step(10)
    got = s.get_state()
    ref = pb.evolve(U, K0, pb.dt(), 10)
    e = field_errors(got, ref)
    log("  e_f = " + " ".join(f"{x:.1e}" for x in e))
    d = s.diagnostics()
    pb.rhs(ref, K0)
    log(f"  c2p atmosphere points: GPU {d['c2p_fail']}, oracle {int(pb.last_fail.sum())}")
    assert np.isfinite(got).all()
    assert e.max() < 1e-11
    s.close()
