"""Pins for the oracle's XCTS initial data (oracle/xcts.py; Methods, "Initial
Data: Approximate XCTS Solution"):

  * the conformal-factor equation Lap psi = -2 pi E psi^5 against an exact
    solution (tests/xcts_case.py): on-axis and off-axis Plummer-like conformal
    factors are recovered to the grid's spectral accuracy, converging
    geometrically with the resolution;
  * the Laplacian assembled from the oracle's derivative route reproduces the
    flat Laplacian of closed forms (|x|^2 -> 6, x -> 0, 1/|x - c| -> 0);
  * the BSSN state of the solved data satisfies the Hamiltonian constraint,
    computed by the oracle's BSSN code (conformal Ricci tensor from phi,
    gt_ij, Gamma-tilde^i and the matter's E = tau + D), to truncation level:
    an independent check of the conformal factor's normalisation, exponent
    and coupling constant;
  * copies of the solver with a planted mistake (psi^4 for psi^5, 4 pi for
    2 pi, +2/r -> -2/r, cot(theta) term dropped, 1/sin theta for
    1/sin^2 theta) miss the exact solution."""

import numpy as np
import pytest
from scipy.linalg import lu_factor, lu_solve

from oracle import diagnostics, evolve, spectral, xcts
from xcts_case import boundary_guess, manufactured, matter

R_IN, R_OUT = 1.8, 20.0


def grid(nr, nth, nph, th0=0.05):
    return spectral.Grid(nr, nth, nph, R_IN, R_OUT, th0, np.pi - th0)


def solve_error(solver, nr, nth, nph, th0=0.05, **case):
    g = grid(nr, nth, nph, th0)
    psi, E = manufactured(g.R, g.TH, g.PH, **case)
    got, it, ch = solver(g, E, boundary_guess(psi))
    return np.abs(got - psi).max(), it


def test_laplacian_of_closed_forms():
    g = grid(24, 22, 16)
    L = xcts.laplacian_matrix(g)
    R, TH, PH = g.R, g.TH, g.PH
    x, y, z = R * np.sin(TH) * np.cos(PH), R * np.sin(TH) * np.sin(PH), R * np.cos(TH)
    inner = ~xcts.boundary_mask(g).reshape(-1)
    assert np.abs((L @ (R ** 2).reshape(-1) - 6.0)[inner]).max() < 1e-6
    assert np.abs((L @ x.reshape(-1))[inner]).max() < 1e-8
    f = 1.0 / np.sqrt((x - 0.2) ** 2 + y ** 2 + (z - 0.1) ** 2)     # a point charge inside r_in
    assert np.abs((L @ f.reshape(-1))[inner]).max() < 1e-4 * np.abs(f).max()


def test_conformal_factor_recovers_exact_solution_on_axis():
    e16, _ = solve_error(xcts.solve, 16, 14, 4)
    e24, it = solve_error(xcts.solve, 24, 22, 4)
    assert e24 < 5e-8 and e24 < e16 / 50, (e16, e24)
    assert it < 30


def test_conformal_factor_recovers_exact_solution_off_axis():
    errs = [solve_error(xcts.solve, 16, 14, nph, c=(2.0, 0.0, 0.0), w=4.0)[0] for nph in (8, 12, 16)]
    assert errs[2] < 1e-7 and errs[2] < errs[0] / 20, errs


def test_solved_data_satisfy_the_hamiltonian_constraint():
    """The BSSN state of the solved conformal factor (matter at rest with
    tau + D = E) has H -> 0 under the oracle's BSSN Hamiltonian constraint
    (theta kept away from the axis, where the flat conformal variables
    converge slowly); and a state with psi off by 1% does not."""
    G = 4.0 / 3.0
    out = []
    for n in (24, 32):
        g = grid(n, n, 4, th0=0.4)
        pb = evolve.Problem(g, M=0.0, a=0.0, Gamma=G)
        psi_x, E = manufactured(g.R, g.TH, g.PH)
        psi, _, _ = xcts.solve(g, E, boundary_guess(psi_x))
        rho, p = matter(E, G)
        H = diagnostics.hamiltonian_constraint(pb, xcts.state(g, psi, rho, p, G))
        out.append(np.abs(H).max() / (16 * np.pi * E.max()))
    assert out[1] < 3e-4 and out[1] < out[0] / 20, out
    g = grid(24, 24, 4, th0=0.4)
    pb = evolve.Problem(g, M=0.0, a=0.0, Gamma=G)
    psi_x, E = manufactured(g.R, g.TH, g.PH)
    rho, p = matter(E, G)
    H = diagnostics.hamiltonian_constraint(pb, xcts.state(g, 1.01 * psi_x, rho, p, G))
    assert np.abs(H).max() / (16 * np.pi * E.max()) > 1e-2


# ---- planted mistakes --------------------------------------------------------

def _planted(power=5, coupling=2.0, r_sign=1.0, cot=1.0, sin_pow=2):
    def lap(grid):
        Dr, Drr, Dt, Dtt, Dp, Dpp = xcts.derivative_matrices(grid)
        Ir, It, Ip = np.eye(grid.nr), np.eye(grid.nth), np.eye(grid.nph)
        R, TH = grid.R.reshape(-1), grid.TH.reshape(-1)
        L = np.kron(Ip, np.kron(It, Drr)) + r_sign * (2.0 / R)[:, None] * np.kron(Ip, np.kron(It, Dr))
        ang = np.kron(Ip, np.kron(Dtt, Ir)) + cot * (np.cos(TH) / np.sin(TH))[:, None] * np.kron(Ip, np.kron(Dt, Ir)) \
            + (1.0 / np.sin(TH) ** sin_pow)[:, None] * np.kron(Dpp, np.kron(It, Ir))
        return L + (1.0 / R ** 2)[:, None] * ang

    def solve(grid, E, psi0, tol=1e-11, max_iter=200):
        L = lap(grid)
        b = xcts.boundary_mask(grid).reshape(-1)
        it = ~b
        lu = lu_factor(L[np.ix_(it, it)])
        rhs_b = L[np.ix_(it, b)] @ psi0.reshape(-1)[b]
        psi = psi0.reshape(-1).copy()
        for k in range(max_iter):
            new = psi.copy()
            new[it] = lu_solve(lu, -coupling * np.pi * E.reshape(-1)[it] * psi[it] ** power - rhs_b)
            done = np.abs(new - psi).max() <= tol * np.abs(new).max()
            psi = new
            if done:
                break
        return psi.reshape(grid.shape), k + 1, 0.0
    return solve


PLANTED = {"psi^4": _planted(power=4), "4 pi": _planted(coupling=4.0), "-2/r": _planted(r_sign=-1.0),
           "no cot": _planted(cot=0.0), "1/sin": _planted(sin_pow=1)}


@pytest.mark.parametrize("name", sorted(PLANTED))
def test_xcts_pins_reject_planted_mistakes(name):
    on = solve_error(PLANTED[name], 16, 14, 4)[0]
    off = solve_error(PLANTED[name], 16, 14, 8, c=(2.0, 0.0, 0.0), w=4.0)[0]
    assert max(on, off) > 1e-4, (name, on, off)
