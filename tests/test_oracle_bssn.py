"""Pins for the oracle's BSSN + gauge right-hand side (Methods: BSSN Evolution
Equations, Gauge Conditions, Stress-Energy Tensor)."""

import numpy as np
import pytest

from oracle import spectral, initial_data, bssn, grmhd, evolve

R_IN, R_OUT, TH0, TH1 = 1.8, 20.0, 0.05, np.pi - 0.05


def derivs(g, f):
    d = {}
    d['phi'] = np.array([g.d1(f['phi'], k) for k in range(3)])
    d['gt'] = np.array([[[g.d1(f['gt'][i, j], k) for j in range(3)] for i in range(3)] for k in range(3)])
    d['At'] = np.array([[[g.d1(f['At'][i, j], k) for j in range(3)] for i in range(3)] for k in range(3)])
    d['K'] = np.array([g.d1(f['K'], k) for k in range(3)])
    d['Gt'] = np.array([[g.d1(f['Gt'][i], k) for i in range(3)] for k in range(3)])
    d['alpha'] = np.array([g.d1(f['alpha'], k) for k in range(3)])
    d['beta'] = np.array([[g.d1(f['beta'][i], k) for i in range(3)] for k in range(3)])
    dd = {}
    dd['phi'] = np.array([[g.d2(f['phi'], k, l) for l in range(3)] for k in range(3)])
    dd['gt'] = np.array([[[[g.d2(f['gt'][i, j], k, l) for j in range(3)] for i in range(3)]
                          for l in range(3)] for k in range(3)])
    dd['alpha'] = np.array([[g.d2(f['alpha'], k, l) for l in range(3)] for k in range(3)])
    dd['beta'] = np.array([[[g.d2(f['beta'][i], k, l) for i in range(3)] for l in range(3)] for k in range(3)])
    return d, dd


def vacuum_rhs(nr, nth, nph, a):
    g = spectral.Grid(nr, nth, nph, R_IN, R_OUT, TH0, TH1)
    f = initial_data.kerr_schild_bssn(g, 1.0, a)
    K0 = evolve.gauge_source_k0(g, f)
    d, dd = derivs(g, f)
    z = np.zeros(g.shape)
    r = bssn.bssn_rhs(f, d, dd, z, np.zeros((3,) + g.shape), np.zeros((3, 3) + g.shape), K0, 2.0)
    H = bssn.hamiltonian(f, d, dd, z)
    inner = (Ellipsis, slice(None), slice(1, -1), slice(1, None))
    worst = max(np.abs(v[inner]).max() for v in r.values())
    return worst, np.abs(H[inner]).max()


@pytest.mark.parametrize("a", [0.0, 0.5])
def test_kerr_schild_is_stationary_exponentially_in_n(a):
    """Vacuum Kerr-Schild data in BSSN variables: the RHS and the Hamiltonian
    constraint vanish up to truncation, which falls geometrically with the
    theta resolution (the limiting direction: the conformal factor carries
    ln(sin theta), singular at the axis just outside the grid)."""
    res = [vacuum_rhs(12, n, 4, a) for n in (16, 32, 48)]
    rhs = np.array([x[0] for x in res])
    ham = np.array([x[1] for x in res])
    assert np.all(rhs[1:] < rhs[:-1] / 10.0)
    assert np.all(ham[1:] < ham[:-1] / 10.0)
    assert rhs[-1] < 2e-2 and ham[-1] < 2e-2


def test_kerr_schild_radial_direction_converges_fast():
    """At fixed theta resolution the r resolution stops mattering quickly
    (log-mapped Chebyshev resolves the radial profile)."""
    a = vacuum_rhs(12, 16, 4, 0.5)[0]
    b = vacuum_rhs(20, 16, 4, 0.5)[0]
    assert abs(a - b) < 2e-3 * b


def _ks_with_fluid(nr=8, nth=10, nph=4, a=0.5, seed=3):
    g = spectral.Grid(nr, nth, nph, R_IN, R_OUT, TH0, TH1)
    f = initial_data.kerr_schild_bssn(g, 1.0, a)
    rng = np.random.default_rng(seed)
    gam = np.exp(4 * f['phi']) * f['gt']
    rho = rng.uniform(0.5, 1.0, g.shape)
    p = rng.uniform(0.1, 0.5, g.shape)
    v = rng.uniform(-0.2, 0.2, (3,) + g.shape) / np.sqrt(np.einsum('ii...->i...', gam))
    B = rng.uniform(-0.3, 0.3, (3,) + g.shape) / np.sqrt(np.einsum('ii...->i...', gam))
    return g, f, gam, rho, p, v, B


def test_matter_coupling_terms_match_covariant_projections():
    """RHS(with matter) - RHS(vacuum) equals the matter terms
    K: 4 pi alpha (E + S); A_ij: -8 pi alpha e^{-4 phi} [S_ij]^TF;
    Gamma^i: -16 pi alpha gt^{ij} S_j; B-driver: same as Gamma^i;
    with E, S_j, S_ij the normal-observer projections of T^{mu nu}."""
    g, f, gam, rho, p, v, B = _ks_with_fluid()
    G = 4.0 / 3.0
    alpha, beta = f['alpha'], f['beta']
    D, S, tau = grmhd.prim_to_cons(rho, p, v, B, gam, G)
    E, Sij = grmhd.matter_3p1(rho, p, v, B, D, tau, gam, G)
    d, dd = derivs(g, f)
    K0 = f['K']
    zero = np.zeros(g.shape)
    r0 = bssn.bssn_rhs(f, d, dd, zero, np.zeros((3,) + g.shape), np.zeros((3, 3) + g.shape), K0, 2.0)
    r1 = bssn.bssn_rhs(f, d, dd, E, S, Sij, K0, 2.0)
    # covariant route
    W = grmhd.lorentz(v, gam)
    u = np.concatenate([(W / alpha)[None], W * (v - beta / alpha)])
    beta_lo = grmhd.lower(gam, beta)
    g4 = np.zeros((4, 4) + g.shape)
    g4[0, 0] = -alpha ** 2 + np.einsum('i...,i...->...', beta_lo, beta)
    g4[0, 1:] = beta_lo
    g4[1:, 0] = beta_lo
    g4[1:, 1:] = gam
    g4inv = np.moveaxis(np.linalg.inv(np.moveaxis(g4, (0, 1), (-2, -1))), (-2, -1), (0, 1))
    u_lo = np.einsum('mn...,n...->m...', g4, u)
    Fh = np.concatenate([np.zeros((1,) + g.shape), B / alpha])
    proj = np.eye(4).reshape(4, 4, 1, 1, 1) + np.einsum('m...,n...->mn...', u, u_lo)
    b = np.einsum('mn...,n...->m...', proj, Fh) / u[0]
    b2 = np.einsum('mn...,m...,n...->...', g4, b, b)
    h = 1 + p / rho * G / (G - 1)
    T = (rho * h + b2) * np.einsum('m...,n...->mn...', u, u) + (p + 0.5 * b2) * g4inv \
        - np.einsum('m...,n...->mn...', b, b)
    T_lo = np.einsum('am...,bn...,mn...->ab...', g4, g4, T)
    E_cov = alpha ** 2 * T[0, 0]
    Sj_cov = -np.einsum('m...,mj...->j...', np.concatenate([-alpha[None], np.zeros((3,) + g.shape)]),
                        np.einsum('mn...,nj...->mj...', T, g4[:, 1:]))
    Sij_cov = T_lo[1:, 1:]
    assert np.abs(E - E_cov).max() < 1e-12 * np.abs(E).max()
    assert np.abs(S - Sj_cov).max() < 1e-12 * np.abs(S).max()
    assert np.abs(Sij - Sij_cov).max() < 1e-12 * np.abs(Sij).max()
    gu = np.exp(-4 * f['phi']) * grmhd.inv3(f['gt'])
    S_tr = np.einsum('ij...,ij...->...', gu, Sij_cov)
    TF = Sij_cov - gam * S_tr / 3.0
    gtu = grmhd.inv3(f['gt'])
    assert np.abs((r1['K'] - r0['K']) - 4 * np.pi * alpha * (E_cov + S_tr)).max() < 1e-12
    assert np.abs((r1['At'] - r0['At']) + 8 * np.pi * alpha * np.exp(-4 * f['phi']) * TF).max() < 1e-12
    jt = -16 * np.pi * alpha * np.einsum('ij...,j...->i...', gtu, Sj_cov)
    assert np.abs((r1['Gt'] - r0['Gt']) - jt).max() < 1e-12
    assert np.abs((r1['Bd'] - r0['Bd']) - jt).max() < 1e-12
    for k in ('phi', 'gt', 'alpha', 'beta'):
        assert np.abs(r1[k] - r0[k]).max() == 0.0


def test_gauge_terms():
    """d_t alpha = beta^k d_k alpha - 2 alpha (K - K0); d_t beta = 3/4 Bd;
    d_t Bd = d_t Gamma-tilde - eta Bd."""
    g = spectral.Grid(8, 10, 4, R_IN, R_OUT, TH0, TH1)
    f = initial_data.kerr_schild_bssn(g, 1.0, 0.5)
    K0 = f['K'].copy()
    f['Bd'] = np.random.default_rng(1).standard_normal((3,) + g.shape)
    d, dd = derivs(g, f)
    z = np.zeros(g.shape)
    zS, zSS = np.zeros((3,) + g.shape), np.zeros((3, 3) + g.shape)
    r0 = bssn.bssn_rhs(f, d, dd, z, zS, zSS, K0, 2.0)
    r1 = bssn.bssn_rhs(f, d, dd, z, zS, zSS, K0 - 0.1, 2.0)
    assert np.abs((r1['alpha'] - r0['alpha']) + 2 * f['alpha'] * 0.1).max() < 1e-14
    assert np.abs(r0['beta'] - 0.75 * f['Bd']).max() == 0.0
    assert np.abs(r0['Bd'] - (r0['Gt'] - 2.0 * f['Bd'])).max() < 1e-12
    r2 = bssn.bssn_rhs(f, d, dd, z, zS, zSS, K0, 2.0, gauge_k0=False)
    assert np.abs((r2['alpha'] - r0['alpha']) + 2 * f['alpha'] * K0).max() < 1e-14


def test_lapse_pulse_rates_closed_form():
    """Spacetime right-hand side pinned by closed forms away from a stationary
    state: a lapse pulse on flat space in the solver's spherical coordinates
    (tests/gauge_case.py).  d_t K = -Laplacian(alpha) and d_t At_ij =
    -e^{-4 phi} (D_i D_j alpha)^TF converge spectrally to the exact rates
    (>= 5x per refinement), every other spacetime rate is zero.  Flipping or
    dropping the Christoffel term of D_i D_j alpha fails it."""
    from gauge_case import lapse_errors, lapse_pulse_state
    errs = []
    for n in ((32, 32, 48), (40, 40, 64)):
        g, pb, U, U_flat, K0, exact = lapse_pulse_state(*n)
        drhs = pb.rhs(U, K0)[:24] - pb.rhs(U_flat, K0)[:24]
        errs.append(lapse_errors(drhs, exact))
    (cK, cA, c0), (fK, fA, f0) = errs
    assert c0 < 1e-14 and f0 < 1e-14
    assert fK < 1e-3 and fK < cK / 5, (cK, fK)
    assert fA < 1e-2 and fA < cA / 5, (cA, fA)


def test_shift_pulse_rates_closed_form():
    """Shift terms pinned by closed forms: a shift pulse (fixed Cartesian
    direction, Gaussian envelope) on flat space (tests/gauge_case.py).  The
    phi, gt and Gt (and driver) rates converge spectrally to the coordinate
    flow's (>= 5x per refinement); K, At, alpha and beta rates are zero.  A
    flipped trace term or a dropped gt.dbeta term in the gt rate, a dropped
    (1/3) gt^{ij} d_j d_k beta^k or a flipped Gt^j d_j beta^i term in the Gt
    rate, or a wrong factor on div beta in the phi rate fail it."""
    from gauge_case import shift_errors, shift_pulse_state
    errs = []
    for n in ((32, 32, 48), (40, 40, 64)):
        g, pb, U, U_flat, K0, exact = shift_pulse_state(*n)
        drhs = pb.rhs(U, K0)[:24] - pb.rhs(U_flat, K0)[:24]
        errs.append(shift_errors(drhs, exact))
    coarse, fine = errs
    assert coarse[3] < 1e-14 and fine[3] < 1e-14
    for k in range(3):  # phi, gt, Gt
        assert fine[k] < 1e-3 and fine[k] < coarse[k] / 5, (k, coarse, fine)
