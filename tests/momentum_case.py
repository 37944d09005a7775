"""Closed-form test cases for the momentum constraint (shared by the CPU pins
and the GPU parity test).

Flat space (M = 0) in the solver's spherical coordinates carries, with the
conformal factor psi = 1 and K = 0, the Bowen-York extrinsic curvature of a
linear momentum P,
    A_ij = 3/(2 r^2) (P_i n_j + P_j n_i - (delta_ij - n_i n_j) P.n)   (Cartesian),
which is trace-free and divergence-free away from r = 0, so
D_j (K^j_i - delta^j_i K) = 0 holds exactly on the shell r in [r_in, r_out].
A trace K = k0 x (Cartesian x) added to it is balanced by the matter momentum
S_i = -d_i K / (12 pi): then -(2/3) d_i K - 8 pi S_i = 0 as well.  With both
the momentum constraint vanishes identically; the discrete one converges to
zero spectrally.  The polar range is kept away from the axis (theta in
[0.4, pi - 0.4]), where the conformal variables of the spherical flat metric
carry the sin^(-2/3) theta factors that slow the theta convergence."""

import numpy as np

from oracle import evolve, initial_data, spectral

R_IN, R_OUT, TH0, TH1 = 1.8, 20.0, 0.4, np.pi - 0.4
P_BY = (0.3, -0.2, 0.5)
K0_SLOPE = 0.02


def jacobian(g):
    """J[i, a] = d x^i / d q^a for q = (r, theta, phi)."""
    R, TH, PH = g.R, g.TH, g.PH
    st, ct, sp, cp = np.sin(TH), np.cos(TH), np.sin(PH), np.cos(PH)
    return np.array([[st * cp, R * ct * cp, -R * st * sp],
                     [st * sp, R * ct * sp, R * st * cp],
                     [ct, -R * st, np.zeros_like(R)]])


def bowen_york_state(nr, nth, nph, P=P_BY, k0=K0_SLOPE, D=1e-3, tau=1e-3):
    """Grid, oracle problem, state U and the Cartesian-free pieces: flat
    space with the Bowen-York A_ij, K = k0 x and the balancing momentum
    density in the matter fields (D and tau set so that the matter is a
    physical state; they do not enter the momentum constraint)."""
    g = spectral.Grid(nr, nth, nph, R_IN, R_OUT, TH0, TH1)
    pb = evolve.Problem(g, M=0.0, a=0.0)
    f = initial_data.kerr_schild_bssn(g, 0.0, 0.0)
    R, TH, PH = g.R, g.TH, g.PH
    x = np.array([R * np.sin(TH) * np.cos(PH), R * np.sin(TH) * np.sin(PH), R * np.cos(TH)])
    n = x / R
    Pv = np.array(P, dtype=float)[:, None, None, None] * np.ones(g.shape)
    Pn = np.sum(Pv * n, axis=0)
    delta = np.eye(3)[:, :, None, None, None]
    A = 1.5 / R ** 2 * (np.einsum('i...,j...->ij...', Pv, n) + np.einsum('i...,j...->ij...', n, Pv)
                        - (delta - np.einsum('i...,j...->ij...', n, n)) * Pn)
    J = jacobian(g)
    A_sph = np.einsum('ia...,jb...,ij...->ab...', J, J, A)
    f['At'] = np.exp(-4.0 * f['phi']) * A_sph
    f['K'] = k0 * x[0]
    S_cart = np.zeros((3,) + g.shape)
    S_cart[0] = -k0 / (12.0 * np.pi)
    S_sph = np.einsum('ia...,i...->a...', J, S_cart)
    _, _, sqrtg = pb.metric(f)
    m = dict(sD=sqrtg * D, sS=sqrtg * S_sph, stau=sqrtg * tau, sB=np.zeros((3,) + g.shape))
    U = evolve.pack(f, m)
    return g, pb, U, f, S_sph


def scale(f, S):
    """Magnitude of the terms that cancel: |8 pi S| (the K and S terms) plus
    the largest Bowen-York term, |gamma^{ij}| weighted."""
    return max(np.abs(8.0 * np.pi * S).max(), 1.5 * np.linalg.norm(P_BY) / R_IN ** 2)
