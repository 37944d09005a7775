"""A closed-form case for the conformal-factor equation of the XCTS initial
data, Lap psi = -2 pi E psi^5 on flat space (shared by the CPU pins and the
GPU parity test).

psi* = 1 + (m/2) (s^2 + w^2)^(-1/2), s the Cartesian distance from a centre
c, is the conformal factor of a Plummer-like mass distribution: since
Lap (s^2 + w^2)^(-1/2) = -3 w^2 (s^2 + w^2)^(-5/2), the energy density
E = 3 m w^2 / (4 pi) (s^2 + w^2)^(-5/2) psi*^(-5) >= 0 makes psi* an exact
solution.  With psi* on the boundary nodes as Dirichlet data the solver must
return psi* to the spectral accuracy of the grid.  The matter is at rest with
specific internal energy EPS0, so rho = E / (1 + EPS0) and
p = (Gamma - 1) EPS0 rho give tau + D = E."""

import numpy as np

EPS0 = 1e-2


def manufactured(R, TH, PH, m=0.5, w=3.0, c=(0.0, 0.0, 4.0)):
    """psi* and E on the nodes (arrays broadcast like R, TH, PH)."""
    x, y, z = R * np.sin(TH) * np.cos(PH), R * np.sin(TH) * np.sin(PH), R * np.cos(TH)
    s2 = (x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2
    psi = 1.0 + 0.5 * m / np.sqrt(s2 + w * w)
    E = 3.0 * m * w * w / (4.0 * np.pi) * (s2 + w * w) ** -2.5 / psi ** 5
    return psi, E


def matter(E, Gamma):
    """rho, p at rest with tau + D = E."""
    rho = E / (1.0 + EPS0)
    return rho, (Gamma - 1.0) * EPS0 * rho


def boundary_guess(psi, nr_axis=-1, th_axis=-2):
    """Initial guess 1 with the exact values on the r-end and theta-end nodes."""
    g = np.ones_like(psi)
    g[..., 0] = psi[..., 0]
    g[..., -1] = psi[..., -1]
    g[..., 0, :] = psi[..., 0, :]
    g[..., -1, :] = psi[..., -1, :]
    return g
