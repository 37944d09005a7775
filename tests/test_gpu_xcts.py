"""XCTS initial data on the GPU (grmhd_xcts_solve through the C-ABI): the
conformal factor of the conformally flat, time-symmetric data against the
oracle's direct collocation solve (element by element, same iteration
count), against the exact Plummer-like conformal factor (tests/xcts_case.py)
on a grid the oracle's dense solve would not reach in seconds, and the
library's Hamiltonian-constraint diagnostic on the state built from it.

The library keeps grmhd_xcts_solve switched off (GRMHD_E_UNAVAILABLE): its
first hardware run ended in a device fault whose cause has not been found, so
the parity tests below are skipped until one is.  Only the refusal itself is
tested, on a 16^3 context (no XCTS kernel runs)."""

import math

import numpy as np
import pytest
import torch

from gpu_util import log
from xcts_case import boundary_guess, manufactured, matter

pytestmark = pytest.mark.gpu

OFF = pytest.mark.skip(reason="grmhd_xcts_solve is switched off: device fault on its first hardware run, "
                              "cause not found (kernel indexing checks out on the CPU)")

R_IN, R_OUT = 1.8, 20.0


def solver_for(nr, nth, nph, th0=0.05):
    from paper_2508_18221_amd import Solver, make_grid, make_phys
    return Solver(make_grid(nr, nth, nph, r_in=R_IN, r_out=R_OUT, th_min=th0, th_max=np.pi - th0),
                  make_phys(M=0.0, a=0.0))


def gpu_solve(s, E, psi_guess, **kw):
    dE = torch.tensor(E, device="cuda")
    dpsi = torch.tensor(psi_guess, device="cuda")
    it, ch = s.xcts_solve(dE, dpsi, **kw)
    return dpsi.cpu().numpy(), it, ch


@OFF
@pytest.mark.parametrize("shape,case", [((12, 10, 4), {}), ((16, 14, 8), dict(c=(2.0, 0.0, 0.0), w=4.0)),
                                        ((20, 18, 12), dict(c=(2.0, 0.0, 0.0), w=4.0)),
                                        ((15, 13, 6), dict(c=(0.0, 1.0, 3.0), w=3.0))])
def test_xcts_matches_oracle(shape, case):
    from oracle import spectral, xcts
    log(f"[xcts] {shape} {case}")
    g = spectral.Grid(*shape, R_IN, R_OUT, 0.05, np.pi - 0.05)
    psi_x, E = manufactured(g.R, g.TH, g.PH, **case)
    guess = boundary_guess(psi_x)
    ref, it_ref, _ = xcts.solve(g, E, guess)
    s = solver_for(*shape)
    got, it, ch = gpu_solve(s, E, guess)
    s.close()
    d = np.abs(got - ref).max()
    log(f"  iterations GPU {it} oracle {it_ref}; max |psi_gpu - psi_oracle| {d:.2e}; "
        f"vs exact {np.abs(got - psi_x).max():.2e}")
    assert np.isfinite(got).all() and ch <= 1e-11
    assert abs(it - it_ref) <= 1
    assert d < 1e-11 * np.abs(ref).max()
    assert np.array_equal(got[:, :, 0], guess[:, :, 0]) and np.array_equal(got[:, 0, :], guess[:, 0, :])


@OFF
def test_xcts_exact_solution_larger_grid():
    """48 x 40 x 16 (30,720 nodes): the exact conformal factor to spectral
    accuracy, off axis."""
    from oracle import spectral
    log("[xcts] 48x40x16 off-axis exact solution")
    g = spectral.Grid(48, 40, 16, R_IN, R_OUT, 0.05, np.pi - 0.05)
    psi_x, E = manufactured(g.R, g.TH, g.PH, c=(2.0, 0.0, 0.0), w=4.0)
    s = solver_for(48, 40, 16)
    got, it, ch = gpu_solve(s, E, boundary_guess(psi_x))
    s.close()
    err = np.abs(got - psi_x).max()
    log(f"  {it} iterations, error vs exact {err:.2e}")
    assert err < 1e-7


@OFF
def test_xcts_state_satisfies_hamiltonian_constraint():
    """The library's diagnostics on the BSSN state built from the GPU's
    conformal factor (matter at rest, tau + D = E; polar range kept away from
    the axis): the Hamiltonian-constraint maximum equals the oracle's on the
    same state and is small against 16 pi E."""
    from oracle import diagnostics, evolve, spectral, xcts
    G = 4.0 / 3.0
    n = 32
    log("[xcts] Hamiltonian constraint of the solved data, 32x32x4, theta in [0.4, pi - 0.4]")
    g = spectral.Grid(n, n, 4, R_IN, R_OUT, 0.4, np.pi - 0.4)
    psi_x, E = manufactured(g.R, g.TH, g.PH)
    s = solver_for(n, n, 4, th0=0.4)
    psi, it, ch = gpu_solve(s, E, boundary_guess(psi_x))
    rho, p = matter(E, G)
    U = xcts.state(g, psi, rho, p, G)
    s.set_state(U, np.zeros(g.shape))
    d = s.diagnostics()
    s.close()
    pb = evolve.Problem(g, M=0.0, a=0.0, Gamma=G)
    H = diagnostics.hamiltonian_constraint(pb, U)
    scale = 16 * np.pi * E.max()
    log(f"  max |H| GPU {d['ham_linf']:.3e} oracle {np.abs(H).max():.3e}; 16 pi E {scale:.3e}")
    assert abs(d["ham_linf"] / np.abs(H).max() - 1) < 1e-8
    assert d["ham_linf"] < 3e-4 * scale


@OFF
def test_xcts_nonfinite_source_stops():
    """A NaN in E stops the iteration and is reported as a NaN change."""
    s = solver_for(12, 10, 4)
    E = np.zeros((4, 10, 12))
    E[1, 4, 5] = np.nan
    got, it, ch = gpu_solve(s, E, np.ones((4, 10, 12)), max_iter=20)
    s.close()
    assert math.isnan(ch) and it == 1


def test_xcts_switched_off_refuses_without_device_work():
    """The switched-off entry point returns GRMHD_E_UNAVAILABLE and leaves
    psi as it was."""
    from paper_2508_18221_amd import Solver, make_grid, make_phys
    from paper_2508_18221_amd._lib import GrmhdError
    s = Solver(make_grid(16, 16, 16), make_phys(M=0.0, a=0.0))
    E = torch.zeros((16, 16, 16), dtype=torch.float64, device="cuda")
    psi = torch.ones_like(E)
    with pytest.raises(GrmhdError, match="error -6: grmhd_xcts_solve is switched off"):
        s.xcts_solve(E, psi)
    s.close()
    assert bool((psi == 1.0).all())
