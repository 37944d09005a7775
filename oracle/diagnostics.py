"""Diagnostics, oracle side: Hamiltonian and momentum constraints, rest mass,
discrete entropy E^n and the magnetic divergence.

Paper: Results, "The Entropy Curve Implies Stability and Convergence"
(E^n = sum rho s sqrt(gamma) dV with s = ln(p/rho^Gamma)/(Gamma-1)), "Magnetic
Constraint" (d_i(sqrt(gamma) B^i) = 0).  Reading: the cell volume dV of the
nonuniform grid is the tensor-product quadrature weight (mapped
Clenshaw-Curtis in r and theta, 2 pi/N in phi), so the sums are integrals.
The constraints the coupled evolution monitors (Results, the coupled-evolution
passage, and Methods, "Initial Data Solver XCTS Approximation": the
Hamiltonian and momentum constraints) are the textbook BSSN forms in
bssn.hamiltonian and bssn.momentum; their norms are
  ||H||_2 = sqrt(sum H^2 w / sum w),  ||M||_2 = sqrt(sum |M|^2 w / sum w),
with |M| = sqrt(gamma^{ij} M_i M_j), and the maxima over the nodes.
"""

import numpy as np

from .spectral import clenshaw_curtis_weights
from .bssn import hamiltonian, momentum, momentum_norm
from .grmhd import matter_3p1
from .evolve import unpack


def weights(grid):
    """w(phi, theta, r) = w_r(r) w_th(theta) (2 pi / n_phi) with dr = r Lh dx."""
    wr = clenshaw_curtis_weights(grid.nr) * grid.r * grid.Lh
    wt = clenshaw_curtis_weights(grid.nth) * grid.Th
    return (2.0 * np.pi / grid.nph) * wt[None, :, None] * wr[None, None, :] * np.ones(grid.shape)


def rest_mass(problem, U):
    return float(np.sum(U[24] * weights(problem.g)))


def entropy(problem, U):
    P = problem.primitives(U)
    G = problem.Gamma
    s = np.log(P['p'] / P['rho'] ** G) / (G - 1.0)
    return float(np.sum(P['rho'] * s * P['sqrtg'] * weights(problem.g)))


def div_B(problem, U):
    g = problem.g
    return sum(g.d1(U[29 + i], i) for i in range(3))


def hamiltonian_constraint(problem, U):
    g = problem.g
    f, _ = unpack(U)
    P = problem.primitives(U)
    E, _ = matter_3p1(P['rho'], P['p'], P['v'], P['B'], P['D'], P['tau'], P['gam'], problem.Gamma)
    d = dict(phi=np.array([g.d1(f['phi'], k) for k in range(3)]),
             gt=np.array([[[g.d1(f['gt'][i, j], k) for j in range(3)] for i in range(3)] for k in range(3)]),
             Gt=np.array([[g.d1(f['Gt'][i], k) for i in range(3)] for k in range(3)]))
    dd = dict(phi=np.array([[g.d2(f['phi'], k, l) for l in range(3)] for k in range(3)]),
              gt=np.array([[[[g.d2(f['gt'][i, j], k, l) for j in range(3)] for i in range(3)]
                            for l in range(3)] for k in range(3)]))
    return hamiltonian(f, d, dd, E)


def momentum_constraint(problem, U):
    """M_i (shape (3, ...)) and |M| of a state; the momentum density is the
    state's densitised S_j divided by sqrt(gamma) (no primitive recovery)."""
    g = problem.g
    f, m = unpack(U)
    _, _, sqrtg = problem.metric(f)
    d = dict(phi=np.array([g.d1(f['phi'], k) for k in range(3)]),
             gt=np.array([[[g.d1(f['gt'][i, j], k) for j in range(3)] for i in range(3)] for k in range(3)]),
             At=np.array([[[g.d1(f['At'][i, j], k) for j in range(3)] for i in range(3)] for k in range(3)]),
             K=np.array([g.d1(f['K'], k) for k in range(3)]))
    M = momentum(f, d, m['sS'] / sqrtg)
    return M, momentum_norm(f, M)


def constraint_norms(problem, U):
    """L2 (quadrature-weighted) and max-norms of H and |M|."""
    w = weights(problem.g)
    H = hamiltonian_constraint(problem, U)
    _, Mn = momentum_constraint(problem, U)
    return dict(ham_l2=float(np.sqrt(np.sum(H * H * w) / np.sum(w))), ham_linf=float(np.abs(H).max()),
                mom_l2=float(np.sqrt(np.sum(Mn * Mn * w) / np.sum(w))), mom_linf=float(Mn.max()))
