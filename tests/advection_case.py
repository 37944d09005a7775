"""A closed-form test case for the matter right-hand side: a density blob
advected at uniform velocity through flat space, written in the solver's
spherical coordinates (r, theta, phi), M = 0, fixed background.

With uniform pressure, uniform velocity and no magnetic field, rho(x, t) =
rho_0(x - V t) is an exact solution of relativistic hydrodynamics (the
pressure, velocity and Lorentz factor W stay uniform, so momentum and energy
are carried with the density).  For the densitised conserved variables of
the Valencia form (Results, "GRMHD Conservative Form"; alpha = 1, beta = 0,
sqrt(gamma) constant in time) the exact rates at t = 0 are, with
d_t rho = -V . grad rho_0:

    d_t(sqrt(gamma) D)   = sqrt(gamma) W d_t rho
    d_t(sqrt(gamma) S_j) = sqrt(gamma) W^2 v_j d_t rho   (rho h = rho + Gamma p / (Gamma - 1))
    d_t(sqrt(gamma) tau) = sqrt(gamma) (W^2 - W) d_t rho
    d_t(sqrt(gamma) B^i) = 0.

In spherical coordinates the flux divergence alone does not give these: the
geometric source (1/2) alpha S^{kl} d_j gamma_kl must cancel the curvilinear
part of the momentum flux, so a dropped or mis-signed source, flux or
velocity component shows as an O(1) error that does not converge.  The
pressure-work term of the tau flux is invisible here (the velocity field is
divergence-free and p uniform); the flux formulas have their own pin against
the covariant definition.

With field=True a magnetic flux tube along the flow, B = b(x, y) z-hat
through the blob (b Gaussian across the tube, which runs parallel to the
polar axis at distance 8, clear of the axis and the inner boundary), rides
with it: b varies only across the flow (div B = 0), the gas pressure
p = P0 - b^2/2 keeps the total pressure uniform, and the tension (b . grad) b
vanishes, so the same blob is still carried unchanged; for v parallel to B,
b^2 = B^2 and v x B = 0, and B and p are static, so the rates above hold
unchanged.  That case checks the magnetic stresses in the momentum flux and
in the geometric source as well."""

import numpy as np

from oracle import evolve, initial_data, spectral
from oracle.grmhd import prim_to_cons

R_IN, R_OUT, TH0, TH1 = 1.8, 20.0, 0.05, np.pi - 0.05
V = 0.5          # speed, along the Cartesian z axis
W_BLOB = 3.0     # Gaussian width
X_C = 8.0        # blob centre (8, 0, 0): on the equator, off the axis
RHO_A, RHO_B, P0 = 1e-2, 5e-3, 1e-3
B_TUBE = 0.03    # peak field of the flux tube (field=True)


def flat_advection_state(nr, nth, nph, field=False, blob=True):
    """Grid, oracle problem, state U, K0 and the exact right-hand side of
    fields 24..31 for the advected blob (with field=True: the field along
    the flow and the balancing pressure; blob=False: the same flow without
    the blob, an exactly steady state)."""
    g = spectral.Grid(nr, nth, nph, R_IN, R_OUT, TH0, TH1)
    pb = evolve.Problem(g, M=0.0, a=0.0, cowling=True)
    f = initial_data.kerr_schild_bssn(g, 0.0, 0.0)
    gam = np.exp(4.0 * f['phi']) * f['gt']
    sqrtg = np.exp(6.0 * f['phi']) * np.sqrt(np.linalg.det(np.moveaxis(f['gt'], (0, 1), (-2, -1))))
    R, TH, PH = g.R, g.TH, g.PH
    x, y, z = R * np.sin(TH) * np.cos(PH), R * np.sin(TH) * np.sin(PH), R * np.cos(TH)
    blob = np.exp(-((x - X_C) ** 2 + y ** 2 + z ** 2) / W_BLOB ** 2) * (1.0 if blob else 0.0)
    rho = RHO_A + RHO_B * blob
    drho = V * RHO_B * blob * 2.0 * z / W_BLOB ** 2          # -V d_z rho_0
    # z-hat in the coordinate basis
    zhat = np.array([np.cos(TH), -np.sin(TH) / R, np.zeros(g.shape)])
    v = V * zhat
    if field:
        b = B_TUBE * np.exp(-((x - X_C) ** 2 + y ** 2) / W_BLOB ** 2)
        B = b * zhat
        p = P0 - 0.5 * b * b
    else:
        B = np.zeros((3,) + g.shape)
        p = np.full(g.shape, P0)
    D, S, tau = prim_to_cons(rho, p, v, B, gam, pb.Gamma)
    U = evolve.pack(f, dict(sD=sqrtg * D, sS=sqrtg * S, stau=sqrtg * tau, sB=sqrtg * B))
    K0 = evolve.gauge_source_k0(g, f)
    W = 1.0 / np.sqrt(1.0 - V * V)
    v_lo = np.einsum('ij...,j...->i...', gam, v)
    exact = np.zeros((8,) + g.shape)
    exact[0] = sqrtg * W * drho
    for j in range(3):
        exact[1 + j] = sqrtg * W * W * v_lo[j] * drho
    exact[4] = sqrtg * (W * W - W) * drho
    return g, pb, U, K0, exact


def advection_errors(rhs, exact):
    """Max error of the D, S_r, S_theta, S_phi, tau rates over the interior
    nodes (the frozen r_out and theta-end nodes left out), each divided by
    the largest exact rate of its group (D | S_j | tau); and the largest
    induction rate."""
    inner = (slice(None), slice(1, -1), slice(1, None))
    groups = {0: (0,), 1: (1, 2, 3), 2: (1, 2, 3), 3: (1, 2, 3), 4: (4,)}
    e = np.zeros(5)
    for q in range(5):
        scale = max(np.abs(exact[k]).max() for k in groups[q])
        e[q] = np.abs(rhs[24 + q][inner] - exact[q][inner]).max() / scale
    return e, np.abs(rhs[29:32]).max()


def exact_density_at(g, t):
    """rho_0(x - V t z-hat) on the grid (the blob at time t)."""
    R, TH, PH = g.R, g.TH, g.PH
    x, y, z = R * np.sin(TH) * np.cos(PH), R * np.sin(TH) * np.sin(PH), R * np.cos(TH)
    return RHO_A + RHO_B * np.exp(-((x - X_C) ** 2 + y ** 2 + (z - V * t) ** 2) / W_BLOB ** 2)
