"""GPU parity of one RHS evaluation and of the RK4 evolution against the
oracle, on the same seeded initial data (the oracle's state is uploaded
through grmhd_set_state).

Tolerances: the second-derivative contractions of the two routes differ by
their FP64 conditioning (~N^4 eps relative to max|f''|: 2e-13 at N = 16,
3e-10 at N = 64); the state after 10 RK4 steps must agree to relative 1e-11
per field (per tensor group scale, see gpu_util.field_errors)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from gpu_util import workload, solver, oracle_problem, field_errors, rhs_errors, log  # noqa: E402
from oracle import evolve  # noqa: E402


def run_rhs(w):
    g, pb, U, K0 = oracle_problem(w)
    s = solver(w)
    s.set_state(U, K0)
    dU = torch.tensor(U, device="cuda")
    out = torch.full_like(dU, np.nan)
    s.rhs(dU, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = pb.rhs(U, K0)
    s.close()
    return got, ref, pb, U


@pytest.mark.parametrize("size", [(16, 16, 16), (20, 18, 12), (33, 7, 6)])
def test_single_rhs_matches_oracle(size):
    log(f"[rhs] grid {size}")
    w = workload("ks_michel_16x16x16", nr=size[0], nth=size[1], nph=size[2])
    got, ref, pb, U = run_rhs(w)
    assert np.isfinite(got).all()
    e = rhs_errors(got, ref, U)
    log("  e_f = " + " ".join(f"{x:.1e}" for x in e))
    assert e.max() < 1e-11
    assert not pb.last_fail.any()


def test_single_rhs_matches_oracle_64x64x128():
    """Full-size workload, the launch configuration the benchmark times."""
    log("[rhs] grid 64x64x128")
    w = workload("ks_michel_64x64x128")
    got, ref, pb, U = run_rhs(w)
    assert np.isfinite(got).all()
    e = rhs_errors(got, ref, U)
    log("  e_f = " + " ".join(f"{x:.1e}" for x in e))
    assert e.max() < 1e-9


def test_rhs_refuses_an_output_that_overlaps_its_input():
    """The right-hand side goes to a buffer apart from its input (the kernel
    takes the two as non-overlapping): an overlapping pair is refused before
    any device work, and the context stays usable."""
    from paper_2508_18221_amd._lib import GrmhdError
    log("[rhs overlap] 16^3: dU_dt over the input, shifted by one field, then a separate buffer")
    w = workload("ks_michel_16x16x16")
    g, pb, U, K0 = oracle_problem(w)
    s = solver(w)
    s.set_state(U, K0)
    buf = torch.tensor(np.concatenate([U.ravel(), U.ravel()]), device="cuda")
    n = U.size
    dU = buf[:n]
    for out in (buf[:n], buf[n // 32:n // 32 + n]):
        with pytest.raises(GrmhdError, match="overlap"):
            s.rhs(dU, out)
    out = torch.full_like(dU, np.nan)
    s.rhs(dU, out)
    torch.cuda.synchronize()
    e = rhs_errors(out.cpu().numpy().reshape(U.shape), pb.rhs(U, K0), U)
    s.close()
    assert e.max() < 1e-11


def test_con2prim_and_fluxes_match_oracle():
    log("[c2p] grid 20x18x12")
    w = workload("ks_michel_16x16x16", nr=20, nth=18, nph=12)
    g, pb, U, K0 = oracle_problem(w)
    s = solver(w)
    s.set_state(U, K0)
    dU = torch.tensor(U, device="cuda")
    prim = torch.empty((5,) + g.shape, dtype=torch.float64, device="cuda")
    flux = torch.empty((24,) + g.shape, dtype=torch.float64, device="cuda")
    s.con2prim(dU, prim, flux)
    torch.cuda.synchronize()
    P = pb.primitives(U)
    from oracle.grmhd import fluxes
    f, _ = evolve.unpack(U)
    F = fluxes(P['D'], P['S'], P['tau'], P['B'], P['rho'], P['p'], P['v'], f['alpha'], f['beta'],
               P['gam'], P['sqrtg'])
    gp = prim.cpu().numpy()
    assert np.abs(gp[0] / P['rho'] - 1).max() < 1e-13
    assert np.abs(gp[1] / P['p'] - 1).max() < 1e-12
    assert np.abs(gp[2:] - P['v']).max() < 1e-13 * np.abs(P['v']).max() + 1e-300
    gf = flux.cpu().numpy().reshape(3, 8, *g.shape)
    # scale of each variable's flux terms: alpha sqrt(gamma) |vt| |U_v| and the
    # pressure / field terms; the induction fluxes vt^a B^k - vt^k B^a cancel
    # exactly in one route and to FMA round-off in the other
    f_, _ = evolve.unpack(U)
    asg = f_['alpha'] * P['sqrtg']
    vt = np.abs(P['v'] - f_['beta'] / f_['alpha']).max()
    Bmax = np.abs(P['B']).max()
    scale = [np.abs(F[v]).max() for v in range(8)]
    for k in range(5, 8):
        scale[k] = max(scale[k], (asg * vt * Bmax).max())
    for a in range(3):
        for v in range(8):
            assert np.abs(gf[a, v] - F[v, a]).max() < 1e-12 * scale[v], (a, v)
    s.close()


def test_ten_steps_match_oracle_16cubed():
    """The tiny coupled evolution: 10 RK4 steps, per-field relative 1e-11."""
    log("[evolve] 16^3, 10 RK4 steps")
    w = workload("ks_michel_16x16x16")
    g, pb, U, K0 = oracle_problem(w)
    s = solver(w)
    s.set_state(U, K0)
    assert abs(s.dt - pb.dt()) < 1e-15 * pb.dt()
    s.step(10)
    got = s.get_state()
    ref = pb.evolve(U, K0, pb.dt(), 10)
    e = field_errors(got, ref)
    log("  e_f = " + " ".join(f"{x:.1e}" for x in e))
    assert np.isfinite(got).all()
    assert e.max() < 1e-11
    assert abs(s.time - 10 * pb.dt()) < 1e-14
    s.close()


def test_ten_steps_ragged_grid():
    log("[evolve] 20x18x12, 10 RK4 steps")
    w = workload("ks_michel_16x16x16", nr=20, nth=18, nph=12)
    g, pb, U, K0 = oracle_problem(w)
    s = solver(w)
    s.set_state(U, K0)
    s.step(10)
    got = s.get_state()
    ref = pb.evolve(U, K0, pb.dt(), 10)
    e = field_errors(got, ref)
    log("  e_f = " + " ".join(f"{x:.1e}" for x in e))
    assert e.max() < 1e-11
    s.close()


def test_library_initial_data_matches_oracle():
    """grmhd_init_state (host C++) vs the oracle's initial data.  The Michel
    temperature is the root of the Bernoulli relation, which has a double root
    at the sonic radius: matter fields agree to 1e-6 there, everything else to
    round-off."""
    log("[init] 16^3 and 20x18x12")
    for over in ({}, dict(nr=20, nth=18, nph=12)):
        w = workload("ks_michel_16x16x16", **over)
        g, pb, U, K0 = oracle_problem(w)
        s = solver(w)
        s.init_state()
        got, gk = s.get_state(with_k0=True)
        e = field_errors(got, U)
        log("  e_f = " + " ".join(f"{x:.1e}" for x in e))
        assert e[:24].max() < 1e-12
        assert e[24:].max() < 1e-6
        assert np.abs(gk - K0).max() < 1e-12 * np.abs(K0).max()
        s.close()


def test_k0_from_state_matches_oracle():
    w = workload("ks_michel_16x16x16", nr=20, nth=18, nph=12)
    g, pb, U, K0 = oracle_problem(w)
    s = solver(w)
    s.set_state(U, None)
    _, gk = s.get_state(with_k0=True)
    assert np.abs(gk - K0).max() < 1e-12 * np.abs(K0).max()
    s.close()


def test_diagnostics_match_oracle():
    from oracle import diagnostics
    w = workload("ks_michel_16x16x16", nr=20, nth=18, nph=12)
    g, pb, U, K0 = oracle_problem(w)
    s = solver(w)
    s.set_state(U, K0)
    d = s.diagnostics()
    assert d["c2p_fail"] == 0 and d["nonfinite"] == 0
    assert abs(d["rest_mass"] / diagnostics.rest_mass(pb, U) - 1) < 1e-13
    assert abs(d["entropy"] / diagnostics.entropy(pb, U) - 1) < 1e-11
    divB = diagnostics.div_B(pb, U)
    assert abs(d["max_abs_divB"] - np.abs(divB).max()) < 1e-12 * np.abs(U[29]).max()
    assert abs(d["min_alpha"] - U[17].min()) < 1e-15
    s.close()


def test_init_state_rejects_parameters_without_data():
    """Initial data that do not exist for the parameters (no black hole, no
    transonic Michel flow, no field) end in an error with the state
    untouched; the context stays usable."""
    from paper_2508_18221_amd import Solver, make_grid, make_phys
    from paper_2508_18221_amd._lib import GrmhdError
    log("[init errors] 16^3: M = 0, r_c below the Michel bound, beta_min = 0, pert_amp = 1")
    g = make_grid(16, 16, 16)
    for over, msg in [(dict(M=0.0, a=0.0), "M > 0"), (dict(r_c=2.5), "transonic"),
                      (dict(beta_min=0.0), "beta_min"), (dict(pert_amp=1.0), "pert_amp")]:
        s = Solver(g, make_phys(**over))
        with pytest.raises(GrmhdError, match=msg):
            s.init_state()
        s.close()
    ok = Solver(g, make_phys())
    ok.init_state()
    ok.step(1)
    assert ok.diagnostics()["nonfinite"] == 0
    ok.close()


def test_lapse_pulse_rates_closed_form():
    """The library's spacetime right-hand side against closed forms, not
    only against the oracle: a lapse pulse on flat space (M = 0, coupled
    path; tests/gauge_case.py).  The oracle's bars at 40 x 40 x 64, and the
    pulse's difference of right-hand sides against the oracle's.  The
    flat-space rates are largest (~0.1, the truncation of the discrete Ricci
    tensor of the conformal variables) at the nodes next to the theta ends on
    the inner edge; the difference removes that truncation but not the
    rounding of those terms, so the bar is the second derivatives' N^4 eps
    of the largest spacetime rate."""
    from paper_2508_18221_amd import Solver, make_grid, make_phys
    from gauge_case import lapse_errors, lapse_pulse_state
    n = (40, 40, 64)
    log(f"[lapse pulse] {n}, M = 0, coupled, RHS(pulse) - RHS(alpha = 1) vs the exact rates")
    g, pb, U, U_flat, K0, exact = lapse_pulse_state(*n)
    s = Solver(make_grid(*n), make_phys(M=0.0, a=0.0))
    got = []
    for state in (U, U_flat):
        s.set_state(state, K0)
        dU = torch.tensor(state, device="cuda")
        out = torch.full_like(dU, np.nan)
        s.rhs(dU, out)
        torch.cuda.synchronize()
        got.append(out.cpu().numpy())
    s.close()
    assert np.isfinite(got[0]).all() and np.isfinite(got[1]).all()
    eK, eA, e0 = lapse_errors(got[0][:24] - got[1][:24], exact)
    log(f"  errors vs exact: K {eK:.1e}, At {eA:.1e}, zero-rate fields {e0:.1e}")
    assert e0 < 1e-14 and eK < 1e-3 and eA < 1e-2
    d_lib = got[0][:24] - got[1][:24]
    d_ora = pb.rhs(U, K0)[:24] - pb.rhs(U_flat, K0)[:24]
    inner = (slice(None), slice(1, -1), slice(1, None))
    scale = max(np.abs(pb.rhs(U, K0)[:24]).max(), np.abs(exact).max())
    e = max(np.abs(d_lib[q][inner] - d_ora[q][inner]).max() for q in range(24)) / scale
    bar = 4e-16 * max(n) ** 4
    log(f"  vs oracle (difference of right-hand sides): {e:.1e} of the largest rate {scale:.1e} (bar {bar:.1e})")
    assert e < bar


def test_shift_pulse_rates_closed_form():
    """The library's shift terms against closed forms: a shift pulse on flat
    space (M = 0, coupled path; tests/gauge_case.py), the oracle's bars at
    40 x 40 x 64, and the difference of right-hand sides against the
    oracle's at N^4 eps of the largest spacetime rate (as for the lapse
    pulse)."""
    from paper_2508_18221_amd import Solver, make_grid, make_phys
    from gauge_case import shift_errors, shift_pulse_state
    n = (40, 40, 64)
    log(f"[shift pulse] {n}, M = 0, coupled, RHS(pulse) - RHS(beta = 0) vs the exact rates")
    g, pb, U, U_flat, K0, exact = shift_pulse_state(*n)
    s = Solver(make_grid(*n), make_phys(M=0.0, a=0.0))
    got = []
    for state in (U, U_flat):
        s.set_state(state, K0)
        dU = torch.tensor(state, device="cuda")
        out = torch.full_like(dU, np.nan)
        s.rhs(dU, out)
        torch.cuda.synchronize()
        got.append(out.cpu().numpy())
    s.close()
    assert np.isfinite(got[0]).all() and np.isfinite(got[1]).all()
    d_lib = got[0][:24] - got[1][:24]
    ephi, egt, eGt, e0 = shift_errors(d_lib, exact)
    log(f"  errors vs exact: phi {ephi:.1e}, gt {egt:.1e}, Gt {eGt:.1e}, zero-rate fields {e0:.1e}")
    assert e0 < 1e-14 and ephi < 1e-3 and egt < 1e-3 and eGt < 1e-3
    d_ora = pb.rhs(U, K0)[:24] - pb.rhs(U_flat, K0)[:24]
    inner = (slice(None), slice(1, -1), slice(1, None))
    scale = max(np.abs(pb.rhs(U, K0)[:24]).max(), np.abs(exact).max())
    e = max(np.abs(d_lib[q][inner] - d_ora[q][inner]).max() for q in range(24)) / scale
    bar = 4e-16 * max(n) ** 4
    log(f"  vs oracle (difference of right-hand sides): {e:.1e} of the largest rate {scale:.1e} (bar {bar:.1e})")
    assert e < bar
