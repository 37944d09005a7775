"""Conformally flat, time-symmetric initial data (the XCTS approximation),
oracle side (plain NumPy FP64; test infrastructure only).

Paper: Methods, "Initial Data: Approximate XCTS Solution" (solve the
Hamiltonian constraint for the conformal factor psi by fixed-point relaxation
with A_ij = 0, then gamma_ij = psi^4 gt_ij and K = 0), and the "Initial Data
Solver XCTS Approximation" item of the coupled-evolution implementation list.

Readings of the paper taken here (where it is silent):
  * the conformal metric is flat (in the solver's spherical coordinates,
    f = diag(1, r^2, r^2 sin^2 theta)); with A_ij = 0 and K = 0 the data are
    time-symmetric and the printed momentum-constraint equation is not solved
    (it then holds only for matter at rest, S_i = 0).
  * the Hamiltonian constraint as printed, Lap psi = -2 pi E psi^5, with E the
    energy density seen by normal observers, held fixed during the iteration.
  * fixed-point relaxation: the Picard iteration psi_{k+1} = the solution of
    the linear problem Lap psi_{k+1} = -2 pi E psi_k^5, with the boundary
    values of the initial guess psi_0 held (Dirichlet data on the r ends and
    the theta ends; phi periodic); it stops once
    max |psi_{k+1} - psi_k| <= tol max |psi_{k+1}|.
  * the flat Laplacian in the solver's coordinates,
      Lap psi = psi_rr + (2/r) psi_r + (psi_thth + cot(theta) psi_th
                + psi_phph / sin^2 theta) / r^2,
    with the oracle's spectral derivatives (spectral.Grid).
  * the linear problem is solved directly: the Laplacian's collocation matrix
    is assembled from the one-dimensional derivative matrices of the oracle's
    route (its derivative routines applied to unit vectors) by Kronecker
    products, restricted to the interior nodes with the boundary values moved
    to the right-hand side; its LU factors (scipy.linalg.lu_factor, computed
    once) solve every iteration's system (sizes of a few thousand nodes).
  * the BSSN state of the data: phi = (1/12) ln det gamma = ln psi +
    (1/6) ln(r^2 sin theta), gt_ij = e^{-4 phi} psi^4 f_ij (the same as for flat
    space, independent of psi), Gamma-tilde^i from spectral derivatives of
    gt_ij, At = 0, K = 0, lapse 1, shift and driver 0; the matter at rest
    without field with D = rho, tau = p / (Gamma - 1) (so tau + D = E),
    densitised by sqrt(gamma) = psi^6 r^2 sin(theta).
"""

import numpy as np
from scipy.linalg import lu_factor, lu_solve

from . import spectral
from .evolve import pack
from .initial_data import kerr_schild_bssn


def derivative_matrices(grid):
    """One-dimensional operators along r, theta, phi of the oracle's route,
    as matrices (column k = the routine applied to the k-th unit vector):
    d_r, d_rr, d_th, d_thth, d_ph, d_phph."""
    def cols(fn, n, axis):
        shape = [1, 1, 1]
        shape[axis] = n
        out = np.empty((n, n))
        for k in range(n):
            e = np.zeros(n)
            e[k] = 1.0
            out[:, k] = fn(e.reshape(shape)).reshape(n)
        return out
    g1 = spectral.Grid(grid.nr, grid.nth, grid.nph, grid.r_in, grid.r_out, grid.th_min, grid.th_max)
    # the radial routines carry the map factors of the nodes: apply them on a
    # grid with one theta and phi point per axis
    gr = spectral.Grid(grid.nr, 4, 4, grid.r_in, grid.r_out, grid.th_min, grid.th_max)
    Dr = cols(lambda f: gr.d_r(np.broadcast_to(f, (1, 1, grid.nr))), grid.nr, 2)
    Drr = cols(lambda f: gr.d_rr(np.broadcast_to(f, (1, 1, grid.nr))), grid.nr, 2)
    Dt = cols(g1.d_th, grid.nth, 1)
    Dtt = cols(g1.d_thth, grid.nth, 1)
    Dp = cols(g1.d_ph, grid.nph, 0)
    Dpp = cols(g1.d_phph, grid.nph, 0)
    return Dr, Drr, Dt, Dtt, Dp, Dpp


def laplacian_matrix(grid):
    """Collocation matrix of the flat Laplacian on the whole grid (index
    (l n_th + k) n_r + j, r fastest)."""
    Dr, Drr, Dt, Dtt, Dp, Dpp = derivative_matrices(grid)
    Ir, It, Ip = np.eye(grid.nr), np.eye(grid.nth), np.eye(grid.nph)
    R = grid.R.reshape(-1)
    TH = grid.TH.reshape(-1)
    L = np.kron(Ip, np.kron(It, Drr)) + (2.0 / R)[:, None] * np.kron(Ip, np.kron(It, Dr))
    ang = np.kron(Ip, np.kron(Dtt, Ir)) + (np.cos(TH) / np.sin(TH))[:, None] * np.kron(Ip, np.kron(Dt, Ir)) \
        + (1.0 / np.sin(TH) ** 2)[:, None] * np.kron(Dpp, np.kron(It, Ir))
    return L + (1.0 / R ** 2)[:, None] * ang


def boundary_mask(grid):
    """True at the r-end and theta-end nodes (the Dirichlet boundary)."""
    m = np.zeros(grid.shape, dtype=bool)
    m[:, :, 0] = m[:, :, -1] = True
    m[:, 0, :] = m[:, -1, :] = True
    return m


def solve(grid, E, psi0, tol=1e-11, max_iter=200):
    """Picard iteration for Lap psi = -2 pi E psi^5 with the boundary values of
    psi0.  Returns (psi, iterations, last relative change)."""
    L = laplacian_matrix(grid)
    b = boundary_mask(grid).reshape(-1)
    it = ~b
    lu = lu_factor(L[np.ix_(it, it)])
    psi_b = psi0.reshape(-1)[b]
    rhs_b = L[np.ix_(it, b)] @ psi_b
    psi = psi0.reshape(-1).copy()
    Ef = E.reshape(-1)
    change = np.inf
    k = 0
    for k in range(1, max_iter + 1):
        rhs = -2.0 * np.pi * Ef[it] * psi[it] ** 5 - rhs_b
        new = psi.copy()
        new[it] = lu_solve(lu, rhs)
        change = np.abs(new - psi).max() / np.abs(new).max()
        psi = new
        if change <= tol:
            break
    return psi.reshape(grid.shape), k, change


def state(grid, psi, rho, p, Gamma):
    """The BSSN + Valencia state (32 fields) of the conformally flat,
    time-symmetric data with conformal factor psi and matter at rest."""
    f = kerr_schild_bssn(grid, 0.0, 0.0)          # flat space: gt_ij, Gamma-tilde^i
    f['phi'] = np.log(psi) + np.log(grid.R ** 2 * np.sin(grid.TH)) / 6.0
    f['At'] = np.zeros_like(f['At'])
    f['K'] = np.zeros(grid.shape)
    f['alpha'] = np.ones(grid.shape)
    f['beta'] = np.zeros((3,) + grid.shape)
    f['Bd'] = np.zeros((3,) + grid.shape)
    sqrtg = psi ** 6 * grid.R ** 2 * np.sin(grid.TH)
    zero = np.zeros((3,) + grid.shape)
    m = dict(sD=sqrtg * rho, sS=zero.copy(), stau=sqrtg * p / (Gamma - 1.0), sB=zero.copy())
    return pack(f, m)
