"""Pins of the oracle's Fishbone-Moncrief torus initial data.

* hydrostatic equilibrium: for circular flow in a stationary axisymmetric
  metric the Euler equation reads d_i ln h = (1/2) (d_i g_{mu nu}) u^mu u^nu
  (i = r, theta); checked with complex-step derivatives of the closed form
  and of the metric at interior points;
* the closed form equals Fishbone & Moncrief's printed structure
  1/2 ln((1 + sqrt(1 + 4c^2)) / alpha_Z^2) - 1/2 sqrt(1 + 4c^2) - ell omega
  up to a constant, with c = ell alpha_Z / sqrt(g_phiphi);
* the pressure maximum sits at r_max on the equator (d_r ln h = 0 there),
  the inner edge at r_in, rho(r_max) = rho_max;
* the magnetised initial data: discrete div(sqrt(gamma) B) = 0, minimum
  plasma beta over the loop = beta_min, the perturbation stream."""

import numpy as np
import pytest

from oracle import kerr_schild as ks
from oracle import spectral
from oracle.initial_data import FMTorus, fm_torus, kerr_schild_bssn, uniform01
from oracle.grmhd import det3, magnetic

M, A, RIN, RMAX, GAM, RHOMAX = 1.0, 0.9375, 6.0, 12.0, 13.0 / 9.0, 1e-8
H = 1e-30


@pytest.fixture(scope="module")
def tor():
    return FMTorus(M, A, RIN, RMAX, GAM, RHOMAX)


def test_hydrostatic_equilibrium(tor):
    pts = [(7.0, 1.5), (10.0, 1.2), (12.0, 1.57), (15.0, 1.9), (20.0, 1.4), (9.0, 1.0)]
    for r, th in pts:
        ut, uph, _, _ = tor.velocity(np.array(r), np.array(th))
        u = np.array([ut, 0.0, 0.0, uph])
        dlnh_r = np.imag(tor.lnh(np.array(r + 1j * H), np.array(th + 0j))) / H
        dlnh_t = np.imag(tor.lnh(np.array(r + 0j), np.array(th + 1j * H))) / H
        dg_r = np.imag(ks.metric4(r + 1j * H, th + 0j, M, A)) / H
        dg_t = np.imag(ks.metric4(r + 0j, th + 1j * H, M, A)) / H
        rhs_r = 0.5 * u @ dg_r @ u
        rhs_t = 0.5 * u @ dg_t @ u
        assert abs(dlnh_r - rhs_r) < 1e-12 * max(abs(rhs_r), 1e-3), (r, th)
        assert abs(dlnh_t - rhs_t) < 1e-12 * max(abs(rhs_t), 1e-3), (r, th)


def test_matches_fishbone_moncrief_form(tor):
    rs = np.array([7.0, 9.0, 12.0, 16.0, 25.0])
    ths = np.array([1.57, 1.3, 1.0, 1.8, 1.5])
    g = ks.metric4(rs, ths, M, A)
    gtt, gtp, gpp = g[0, 0], g[0, 3], g[3, 3]
    omega = -gtp / gpp
    alz2 = omega * omega * gpp - gtt
    c2 = tor.ell ** 2 * alz2 / gpp
    fm = 0.5 * np.log((1.0 + np.sqrt(1.0 + 4.0 * c2)) / alz2) - 0.5 * np.sqrt(1.0 + 4.0 * c2) - tor.ell * omega
    diff = tor.lnh(rs, ths) - fm
    assert np.ptp(diff) < 1e-13


def test_pressure_maximum_and_edges(tor):
    d = np.imag(tor.lnh(np.array(RMAX + 1j * H), np.array(np.pi / 2 + 0j))) / H
    assert abs(d) < 1e-13
    assert abs(tor.density(RMAX, np.pi / 2) - RHOMAX) < 1e-13 * RHOMAX
    assert tor.density(RIN - 1e-6, np.pi / 2) == 0.0
    assert tor.density(RIN + 1e-3, np.pi / 2) > 0.0
    # the maximum over a radial scan of the equator is at r_max
    r = np.linspace(6.5, 40.0, 2001)
    rho = tor.density(r, np.full_like(r, np.pi / 2))
    assert abs(r[np.argmax(rho)] - RMAX) < 0.02
    # the flow reproduces its own ell = u^t u_phi
    ut, uph, Om, u_t = tor.velocity(np.array(RMAX), np.array(np.pi / 2))
    assert abs(tor.ell - ut * (ut * Om) * ks.metric4(RMAX, np.pi / 2, M, A)[3, 3]
               - ut * ut * ks.metric4(RMAX, np.pi / 2, M, A)[0, 3]) < 1e-12 * tor.ell


def test_magnetised_initial_data():
    r_in = 1.8 * ks.horizon_radius(M, A) / ks.horizon_radius(M, 0.5)
    g = spectral.Grid(24, 20, 8, r_in, 60.0, 0.05, np.pi - 0.05)
    f = kerr_schild_bssn(g, M, A)
    mat = fm_torus(g, f, M, A, GAM, RIN, RMAX, RHOMAX, 100.0, 0.04, 5)
    sB = mat["sB"]
    div = g.d_r(sB[0]) + g.d_th(sB[1]) + g.d_ph(sB[2])
    assert np.abs(div).max() < 1e-12 * np.abs(g.d_r(sB[0])).max()
    gam = np.exp(4.0 * f["phi"]) * f["gt"]
    sqrtg = np.exp(6.0 * f["phi"]) * np.sqrt(det3(f["gt"]))
    _, _, _, b2 = magnetic(mat["v"], mat["B"], gam)
    tor = FMTorus(M, A, RIN, RMAX, GAM, RHOMAX)
    loop = tor.density(g.R, g.TH) / RHOMAX > 0.2
    p0 = mat["p"] / (1.0 + 0.04 * (2.0 * uniform01(5, g.npts).reshape(g.shape) - 1.0))
    assert abs(np.min(2.0 * p0[loop] / b2[loop]) - 100.0) < 1e-9
    # perturbation within +-4 %, density untouched by it
    ratio = mat["p"] / p0
    assert np.all(np.abs(ratio - 1.0) <= 0.04 + 1e-15)
    assert np.all(mat["rho"] > 0.0) and np.all(mat["p"] > 0.0)
    # the flow inside the torus is subluminal
    vl = np.einsum("ij...,j...->i...", gam, mat["v"])
    assert np.all(np.sum(vl * mat["v"], axis=0) < 1.0)
    assert np.allclose(sqrtg * mat["B"], sB)
