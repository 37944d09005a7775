"""Closed-form test cases for the spacetime right-hand side: a lapse pulse
and a shift pulse on flat space.

Lapse pulse: on flat space, written in the solver's spherical coordinates (r, theta, phi),
M = 0, zero shift, K_ij = 0, with a tenuous uniform fluid at rest.

The slice is flat and momentarily static, so at t = 0 the BSSN + gauge
equations (Methods, "BSSN Evolution Equations", "Gauge Conditions") give
exactly

    d_t K      = -D^i D_i alpha + 4 pi alpha (E + S)
    d_t At_ij  = -e^{-4 phi} (D_i D_j alpha - gamma_ij D^k D_k alpha / 3)
    d_t (phi, gt_ij, Gt^i, alpha, beta^i, B_d^i) = 0

(R_ij = 0, At_ij = 0, beta = 0; the fluid's S_ij = p gamma_ij has no
trace-free part).  The discrete flat-space Ricci tensor in these coordinates
is not zero near the theta ends (the polar truncation of the conformal
variables), and it enters d_t At_ij through alpha R_ij; it does not depend
on alpha, so the check takes the difference of the right-hand sides with
and without the pulse, whose exact value is the list above minus the
pulse-free rates (4 pi (alpha - 1)(E + S) in place of 4 pi alpha (E + S)),
up to (alpha - 1) times that truncation.  D_i D_j alpha is the covariant Hessian: for the Gaussian
pulse alpha = 1 + A exp(-|x - x_c|^2 / w^2) it is the Cartesian Hessian
pulled back with the Jacobian dx^a/dq^i, so the Christoffel symbols of the
spherical coordinates enter the check through both the Hessian and the
Laplacian."""

import numpy as np

from oracle import evolve, initial_data, spectral
from oracle.bssn import SYM
from oracle.grmhd import prim_to_cons

R_IN, R_OUT, TH0, TH1 = 1.8, 20.0, 0.05, np.pi - 0.05
AMP, WID = 1e-3, 2.5
XC = np.array([9.0, 0.0, 2.0])       # pulse centre: off the equator, far from the axis
RHO, PRESS = 1e-12, 1e-14            # tenuous fluid at rest


def lapse_pulse_state(nr, nth, nph):
    """Grid, coupled oracle problem, the state U with the pulse, the same
    state U_flat with alpha = 1, K0 (the same for both) and the exact
    difference of their right-hand sides over the 24 spacetime fields."""
    g = spectral.Grid(nr, nth, nph, R_IN, R_OUT, TH0, TH1)
    pb = evolve.Problem(g, M=0.0, a=0.0)
    f = initial_data.kerr_schild_bssn(g, 0.0, 0.0)
    R, TH, PH = g.R, g.TH, g.PH
    st, ct, sp, cp = np.sin(TH), np.cos(TH), np.sin(PH), np.cos(PH)
    X = np.array([R * st * cp, R * st * sp, R * ct])
    d = X - XC.reshape(3, 1, 1, 1)
    gauss = np.exp(-np.sum(d * d, axis=0) / WID ** 2)
    f_flat = dict(f)
    f = dict(f)
    f['alpha'] = 1.0 + AMP * gauss
    # Cartesian Hessian of alpha and its pull-back J^a_i J^b_j H_ab
    Hc = AMP * gauss * (4.0 * np.einsum('a...,b...->ab...', d, d) / WID ** 4
                        - 2.0 * np.eye(3).reshape(3, 3, 1, 1, 1) / WID ** 2)
    J = np.array([[st * cp, R * ct * cp, -R * st * sp],   # J[a, i] = dx^a / dq^i
                  [st * sp, R * ct * sp, R * st * cp],
                  [ct, -R * st, np.zeros_like(R)]])
    H = np.einsum('ai...,bj...,ab...->ij...', J, J, Hc)
    lap = np.trace(Hc, axis1=0, axis2=1)
    gam = np.exp(4.0 * f['phi']) * f['gt']
    sqrtg = np.exp(6.0 * f['phi']) * np.sqrt(np.linalg.det(np.moveaxis(f['gt'], (0, 1), (-2, -1))))
    rho = np.full(g.shape, RHO)
    p = np.full(g.shape, PRESS)
    zero3 = np.zeros((3,) + g.shape)
    D, S, tau = prim_to_cons(rho, p, zero3, zero3, gam, pb.Gamma)
    m = dict(sD=sqrtg * D, sS=sqrtg * S, stau=sqrtg * tau, sB=sqrtg * zero3)
    U, U_flat = evolve.pack(f, m), evolve.pack(f_flat, m)
    K0 = evolve.gauge_source_k0(g, f)
    E = tau + D
    exact = np.zeros((24,) + g.shape)
    exact[13] = -lap + 4.0 * np.pi * (f['alpha'] - 1.0) * (E + 3.0 * p)
    e4 = np.exp(-4.0 * f['phi'])
    for c, (i, j) in enumerate(SYM):
        exact[7 + c] = -e4 * (H[i, j] - gam[i, j] * lap / 3.0)
    return g, pb, U, U_flat, K0, exact


def lapse_errors(drhs, exact):
    """Max error of the right-hand-side difference drhs over the interior
    nodes (frozen r_out and theta-end nodes left out) of K, of the At group (divided by the largest exact At rate)
    and of the fields whose exact rate is zero (divided by the largest exact
    K rate)."""
    inner = (slice(None), slice(1, -1), slice(1, None))
    sK = np.abs(exact[13]).max()
    sA = np.abs(exact[7:13]).max()
    eK = np.abs(drhs[13][inner] - exact[13][inner]).max() / sK
    eA = max(np.abs(drhs[q][inner] - exact[q][inner]).max() for q in range(7, 13)) / sA
    zero = [q for q in range(24) if q not in range(7, 14)]
    e0 = max(np.abs(drhs[q][inner]).max() for q in zero) / sK
    return eK, eA, e0


# ---------------------------------------------------------------------------
# Shift pulse: beta = EPS exp(-|x - x_c|^2 / w^2) c (a fixed Cartesian
# direction c), alpha = 1, K_ij = 0, on flat space.  At t = 0 the slice
# changes only by the coordinate flow, so with D_k beta^k the (Cartesian)
# divergence and D_i beta_j the Cartesian gradient pulled back:
#
#     d_t phi      = D_k beta^k / 6                 (phi = ln(det gamma) / 12)
#     d_t gt_ij    = e^{-4 phi} (D_i beta_j + D_j beta_i - 2/3 gamma_ij D_k beta^k)
#     d_t Gt^i     = -d_j (d_t gt^{ij}),  d_t gt^{ij} = -gt^{ik} gt^{jl} d_t gt_kl
#                    (Gt^i = -d_j gt^{ij} when det gt = 1, as here)
#     d_t B_d^i    = d_t Gt^i                       (B_d = 0)
#     d_t (K, At_ij, alpha, beta^i) = 0             (alpha = 1, beta . grad alpha = 0,
#                                                    B_d = 0, K0 = K - beta . grad alpha / 2 alpha)
#
# The Gt rate is formed with the oracle's spectral derivative of the closed
# form, so it is exact up to that derivative's truncation.  As for the lapse
# pulse, the pulse-free Ricci truncation cancels in the difference of the
# right-hand sides with and without the shift.
EPS, SWID = 1e-3, 2.5
SDIR = np.array([0.6, -0.48, 0.64])   # unit Cartesian direction of the shift
SXC = np.array([9.0, 0.0, 2.0])


def shift_pulse_state(nr, nth, nph):
    """Grid, coupled oracle problem, the state U with the shift pulse, the
    same state U_flat without it, K0 and the exact difference of their
    right-hand sides over the 24 spacetime fields."""
    g = spectral.Grid(nr, nth, nph, R_IN, R_OUT, TH0, TH1)
    pb = evolve.Problem(g, M=0.0, a=0.0)
    f = initial_data.kerr_schild_bssn(g, 0.0, 0.0)
    R, TH, PH = g.R, g.TH, g.PH
    st, ct, sp, cp = np.sin(TH), np.cos(TH), np.sin(PH), np.cos(PH)
    X = np.array([R * st * cp, R * st * sp, R * ct])
    d = X - SXC.reshape(3, 1, 1, 1)
    gauss = np.exp(-np.sum(d * d, axis=0) / SWID ** 2)
    J = np.array([[st * cp, R * ct * cp, -R * st * sp],
                  [st * sp, R * ct * sp, R * st * cp],
                  [ct, -R * st, np.zeros_like(R)]])
    Jinv = np.moveaxis(np.linalg.inv(np.moveaxis(J, (0, 1), (-2, -1))), (-2, -1), (0, 1))  # dq^i / dx^a
    beta_c = EPS * gauss * SDIR.reshape(3, 1, 1, 1)                 # Cartesian components
    grad = -2.0 * d / SWID ** 2                                    # d_a gauss / gauss
    dbeta_c = EPS * gauss * np.einsum('a...,b->ab...', grad, SDIR)  # d_a beta^b
    div = np.einsum('aa...->...', dbeta_c)
    f_flat = dict(f)
    f = dict(f)
    f['beta'] = np.einsum('ia...,a...->i...', Jinv, beta_c)         # coordinate components
    Dbeta = np.einsum('ai...,bj...,ab...->ij...', J, J, dbeta_c)    # D_i beta_j (flat, Cartesian pulled back)
    gam = np.exp(4.0 * f['phi']) * f['gt']
    sqrtg = np.exp(6.0 * f['phi']) * np.sqrt(np.linalg.det(np.moveaxis(f['gt'], (0, 1), (-2, -1))))
    zero3 = np.zeros((3,) + g.shape)
    rho, p = np.full(g.shape, RHO), np.full(g.shape, PRESS)
    D, S, tau = prim_to_cons(rho, p, zero3, zero3, gam, pb.Gamma)
    m = dict(sD=sqrtg * D, sS=sqrtg * S, stau=sqrtg * tau, sB=sqrtg * zero3)
    U, U_flat = evolve.pack(f, m), evolve.pack(f_flat, m)
    K0 = evolve.gauge_source_k0(g, f)
    e4 = np.exp(-4.0 * f['phi'])
    dgt = e4 * (Dbeta + np.swapaxes(Dbeta, 0, 1) - (2.0 / 3.0) * gam * div)
    gtu = np.moveaxis(np.linalg.inv(np.moveaxis(f['gt'], (0, 1), (-2, -1))), (-2, -1), (0, 1))
    dgtu = -np.einsum('ik...,jl...,kl...->ij...', gtu, gtu, dgt)
    exact = np.zeros((24,) + g.shape)
    exact[0] = div / 6.0
    for c, (i, j) in enumerate(SYM):
        exact[1 + c] = dgt[i, j]
    for i in range(3):
        exact[14 + i] = -sum(g.d1(dgtu[i, j], j) for j in range(3))
    exact[21:24] = exact[14:17]
    return g, pb, U, U_flat, K0, exact


def shift_errors(drhs, exact):
    """Max error of the right-hand-side difference over the interior nodes,
    per group (phi | gt | Gt and B_d), each divided by the group's largest
    exact rate; and the largest rate of the fields whose exact rate is zero,
    divided by the largest exact gt rate."""
    inner = (slice(None), slice(1, -1), slice(1, None))
    groups = [(0,), tuple(range(1, 7)), (14, 15, 16, 21, 22, 23)]
    e = []
    for grp in groups:
        scale = max(np.abs(exact[q]).max() for q in grp)
        e.append(max(np.abs(drhs[q][inner] - exact[q][inner]).max() for q in grp) / scale)
    sg = np.abs(exact[1:7]).max()
    zero = [q for q in range(24) if q not in (0, 1, 2, 3, 4, 5, 6, 14, 15, 16, 21, 22, 23)]
    e0 = max(np.abs(drhs[q][inner]).max() for q in zero) / sg
    return e[0], e[1], e[2], e0
