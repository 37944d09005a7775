"""Diagnostics, oracle side: Hamiltonian constraint, rest mass, discrete
entropy E^n and the magnetic divergence.

Paper: Results, "The Entropy Curve Implies Stability and Convergence"
(E^n = sum rho s sqrt(gamma) dV with s = ln(p/rho^Gamma)/(Gamma-1)), "Magnetic
Constraint" (d_i(sqrt(gamma) B^i) = 0).  Reading: the cell volume dV of the
nonuniform grid is the tensor-product quadrature weight (mapped
Clenshaw-Curtis in r and theta, 2 pi/N in phi), so the sums are integrals.
"""

import numpy as np

from .spectral import clenshaw_curtis_weights
from .bssn import hamiltonian
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
