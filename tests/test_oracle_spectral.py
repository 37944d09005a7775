"""Pins for the oracle's grid, derivative, filter and quadrature operators
against closed forms (Methods: Grid Discretization, Spectral Derivative
Operators, Dealiasing and Spectral Filtering)."""

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import spectral

R_IN, R_OUT, TH0, TH1 = 1.8, 20.0, 0.05, np.pi - 0.05


def test_cgl_nodes_closed_form():
    x = spectral.cgl_nodes(9)
    assert x[0] == 1.0 and abs(x[-1] + 1.0) < 1e-15
    assert np.allclose(x, [np.cos(j * np.pi / 8) for j in range(9)], atol=0, rtol=0)
    g = spectral.Grid(9, 7, 6, R_IN, R_OUT, TH0, TH1)
    assert abs(g.r[0] - R_OUT) < 1e-13 and abs(g.r[-1] - R_IN) < 1e-14
    assert abs(g.th[0] - TH1) < 1e-15 and abs(g.th[-1] - TH0) < 1e-15
    assert np.allclose(g.ph, 2 * np.pi * np.arange(6) / 6)


@pytest.mark.parametrize("n", [5, 12, 17])
def test_chebyshev_exact_on_polynomials_in_ln_r(n):
    """P(ln r) of degree n-1 is reproduced exactly: d_r P = P'(ln r)/r,
    d_rr P = (P'' - P')/r^2."""
    g = spectral.Grid(n, 4, 4, R_IN, R_OUT, TH0, TH1)
    rng = np.random.default_rng(n)
    c = rng.standard_normal(n)          # power-series coefficients in s = ln r - 2
    s = np.log(g.r) - 2.0
    P = np.polynomial.polynomial.polyval(s, c)
    P1 = np.polynomial.polynomial.polyval(s, np.polynomial.polynomial.polyder(c, 1))
    P2 = np.polynomial.polynomial.polyval(s, np.polynomial.polynomial.polyder(c, 2))
    f = np.broadcast_to(P, g.shape)
    scale1 = np.abs(P1 / g.r).max()
    scale2 = np.abs((P2 - P1) / g.r ** 2).max()
    assert np.abs(g.d_r(f) - P1 / g.r).max() <= 1e-12 * scale1 * n
    assert np.abs(g.d_rr(f) - (P2 - P1) / g.r ** 2).max() <= 1e-11 * scale2 * n ** 2


@pytest.mark.parametrize("n", [6, 16])
def test_chebyshev_exact_on_polynomials_in_theta(n):
    g = spectral.Grid(4, n, 4, R_IN, R_OUT, TH0, TH1)
    rng = np.random.default_rng(100 + n)
    c = rng.standard_normal(n)
    t = g.th - 1.5
    P = np.polynomial.polynomial.polyval(t, c)
    P1 = np.polynomial.polynomial.polyval(t, np.polynomial.polynomial.polyder(c, 1))
    P2 = np.polynomial.polynomial.polyval(t, np.polynomial.polynomial.polyder(c, 2))
    f = np.broadcast_to(P[None, :, None], g.shape)
    assert np.abs(g.d_th(f) - P1[None, :, None]).max() <= 1e-12 * np.abs(P1).max() * n
    assert np.abs(g.d_thth(f) - P2[None, :, None]).max() <= 1e-11 * np.abs(P2).max() * n ** 2


def test_chebder_m2_equals_twice_m1():
    """The m = 2 route and applying the m = 1 route twice agree to round-off
    (both are the second derivative of the same interpolant)."""
    rng = np.random.default_rng(3)
    f = rng.standard_normal((4, 16))
    a = spectral.cheb_deriv(f, -1, 2)
    b = spectral.cheb_deriv(spectral.cheb_deriv(f, -1, 1), -1, 1)
    assert np.abs(a - b).max() <= 1e-11 * np.abs(a).max()


@pytest.mark.parametrize("n", [8, 16, 32])
def test_fourier_exact_on_trig_modes_and_nyquist_rule(n):
    g = spectral.Grid(4, 4, n, R_IN, R_OUT, TH0, TH1)
    ph = g.ph
    for k in range(1, n // 2):
        for fn, d1, d2 in ((np.cos(k * ph), -k * np.sin(k * ph), -k * k * np.cos(k * ph)),
                           (np.sin(k * ph), k * np.cos(k * ph), -k * k * np.sin(k * ph))):
            f = np.broadcast_to(fn[:, None, None], g.shape)
            assert np.abs(g.d_ph(f) - d1[:, None, None]).max() < 1e-13 * k * n
            assert np.abs(g.d_phph(f) - d2[:, None, None]).max() < 1e-12 * k * k * n
    # Nyquist: cos(n phi / 2) -> first derivative 0, second -(n/2)^2 cos
    ny = np.cos(0.5 * n * ph)
    f = np.broadcast_to(ny[:, None, None], g.shape)
    assert np.abs(g.d_ph(f)).max() < 1e-12 * n
    assert np.abs(g.d_phph(f) + (n / 2) ** 2 * ny[:, None, None]).max() < 1e-11 * n * n


def test_spectral_convergence_is_exponential():
    """Derivative error of analytic functions falls geometrically with N."""
    errs_r, errs_p = [], []
    for n in (8, 12, 16, 20, 24):
        g = spectral.Grid(n, 4, n, R_IN, R_OUT, TH0, TH1)
        f = np.broadcast_to(1.0 / (g.r + 1.0), g.shape)
        errs_r.append(np.abs(g.d_r(f) + 1.0 / (g.r + 1.0) ** 2).max())
        fp = np.broadcast_to(np.exp(np.sin(g.ph))[:, None, None], g.shape)
        exact = (np.cos(g.ph) * np.exp(np.sin(g.ph)))[:, None, None]
        errs_p.append(np.abs(g.d_ph(fp) - exact).max())
    errs_r, errs_p = np.array(errs_r), np.array(errs_p)
    assert np.all(np.diff(np.log(errs_r)) < -1.0)          # at least e^-1 per 4 modes
    assert np.all(np.diff(np.log(errs_p[:3])) < -3.0)
    assert errs_r[-1] < 1e-8 and errs_p[-1] < 1e-12


def test_mixed_derivatives_commute_on_products():
    g = spectral.Grid(10, 9, 8, R_IN, R_OUT, TH0, TH1)
    f = (np.log(g.R) ** 3) * (g.TH - 1.5) ** 3 * np.sin(2 * g.PH)
    exact_rth = (3 * np.log(g.R) ** 2 / g.R) * 3 * (g.TH - 1.5) ** 2 * np.sin(2 * g.PH)
    assert np.abs(g.d2(f, 0, 1) - exact_rth).max() < 1e-9
    assert np.abs(g.d2(f, 0, 1) - g.d1(g.d1(f, 1), 0)).max() < 1e-10


def test_filter_modal_identities():
    n = 12
    g = spectral.Grid(n, 4, 4, R_IN, R_OUT, TH0, TH1)
    # constants untouched (sigma(0) = 1)
    c = np.full(g.shape, 2.5)
    assert np.abs(spectral.cheb_filter(c, -1, 36.0, 16) - 2.5).max() < 1e-14
    # T_{n-1}(x) -> exp(-36) T_{n-1}(x); T_k -> exp(-36 (k/(n-1))^16) T_k
    x = spectral.cgl_nodes(n)
    for k in (0, 3, n // 2, n - 1):
        Tk = npcheb.chebval(x, [0] * k + [1])
        out = spectral.cheb_filter(np.broadcast_to(Tk, g.shape), -1, 36.0, 16)
        sig = np.exp(-36.0 * (k / (n - 1)) ** 16)
        assert np.abs(out - sig * Tk).max() < 1e-14
    # Fourier: cos(k phi) -> sigma(k) cos(k phi); Nyquist sigma = e^-36
    m = 16
    gp = spectral.Grid(4, 4, m, R_IN, R_OUT, TH0, TH1)
    for k in (1, 5, m // 2):
        f = np.broadcast_to(np.cos(k * gp.ph)[:, None, None], gp.shape)
        out = spectral.fourier_filter(f, -3, 36.0, 16)
        sig = np.exp(-36.0 * (k / (m // 2)) ** 16)
        assert np.abs(out - sig * f).max() < 1e-15
    assert abs(np.exp(-36.0) - 2.319522830243569e-16) < 1e-30


def test_dealias_two_thirds_rule():
    m = 12
    g = spectral.Grid(4, 4, m, R_IN, R_OUT, TH0, TH1)
    keep = np.broadcast_to(np.cos(4 * g.ph)[:, None, None], g.shape)   # 4 <= 12/3
    drop = np.broadcast_to(np.cos(5 * g.ph)[:, None, None], g.shape)
    assert np.abs(spectral.fourier_truncate(keep, -3) - keep).max() < 1e-14
    assert np.abs(spectral.fourier_truncate(drop, -3)).max() < 1e-14


@pytest.mark.parametrize("n", [5, 16, 33])
def test_clenshaw_curtis_weights_integrate_polynomials(n):
    w = spectral.clenshaw_curtis_weights(n)
    x = spectral.cgl_nodes(n)
    for m in range(0, n):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.sum(w * x ** m) - exact) < 1e-13
