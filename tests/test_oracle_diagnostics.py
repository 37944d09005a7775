"""Pins for three oracle functions that the diagnostics and the dealiasing
variant rest on, each against values fixed by the mathematics rather than by
the oracle itself:

  * diagnostics.weights: the mapped Clenshaw-Curtis x trapezoid weights (the
    cell volume of the nonuniform grid in the entropy and rest-mass sums,
    Results "The Entropy Curve Implies Stability and Convergence") must
    integrate closed forms over the wedge r in [r_in, r_out], theta in
    [th_min, th_max], phi in [0, 2 pi): the coordinate volume, r^k moments,
    polar moments and the shell-wedge volume int r^2 sin(theta);
  * diagnostics.entropy: E^n = sum rho s sqrt(gamma) dV with
    s = ln(p / rho^Gamma) / (Gamma - 1) for a uniform fluid at rest on flat
    space is rho s times the wedge volume, and for a fluid with a radial and
    polar density profile it is a one-dimensional integral done by scipy's
    adaptive quadrature;
  * spectral.cheb_truncate: the 2/3 rule of "Dealiasing and Spectral
    Filtering" keeps Chebyshev modes k <= 2(N - 1)/3 exactly and removes the
    ones above, along r and along theta.

Each pin is a function of the routine under test, so the same check is also
run on copies of the routine with a planted mistake (a dropped map factor, a
wrong measure, rho in place of rho^Gamma, an off-by-one cut-off) and must
reject every one of them."""

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb
from scipy import integrate

from oracle import diagnostics, evolve, initial_data, spectral
from oracle.grmhd import prim_to_cons

R_IN, R_OUT, TH0, TH1 = 1.8, 20.0, 0.05, np.pi - 0.05


# ---- quadrature weights -------------------------------------------------------

def weight_errors(weights_fn, nr=32, nth=28, nph=8):
    """Relative errors of sum f w against the exact integral over the wedge
    for a set of closed forms."""
    g = spectral.Grid(nr, nth, nph, R_IN, R_OUT, TH0, TH1)
    w = weights_fn(g)
    R, TH, PH = g.R, g.TH, g.PH
    dth = TH1 - TH0
    cases = {
        "volume": (np.ones(g.shape), (R_OUT - R_IN) * dth * 2 * np.pi),
        "r": (R, 0.5 * (R_OUT ** 2 - R_IN ** 2) * dth * 2 * np.pi),
        "r^2": (R ** 2, (R_OUT ** 3 - R_IN ** 3) / 3 * dth * 2 * np.pi),
        "1/r": (1.0 / R, np.log(R_OUT / R_IN) * dth * 2 * np.pi),
        "sin": (np.sin(TH), (R_OUT - R_IN) * (np.cos(TH0) - np.cos(TH1)) * 2 * np.pi),
        "cos^2": (np.cos(TH) ** 2, (R_OUT - R_IN) * (0.5 * dth + 0.25 * (np.sin(2 * TH1) - np.sin(2 * TH0)))
                  * 2 * np.pi),
        "shell": (R ** 2 * np.sin(TH), (R_OUT ** 3 - R_IN ** 3) / 3 * (np.cos(TH0) - np.cos(TH1)) * 2 * np.pi),
        "cos(phi)^2": (np.cos(PH) ** 2, (R_OUT - R_IN) * dth * np.pi),
    }
    return {k: abs(np.sum(f * w) - ex) / abs(ex) for k, (f, ex) in cases.items()}


def test_weights_integrate_closed_forms_over_the_mapped_wedge():
    err = weight_errors(diagnostics.weights)
    assert max(err.values()) < 1e-13, err
    # a Fourier mode integrates to zero over the period
    g = spectral.Grid(16, 12, 10, R_IN, R_OUT, TH0, TH1)
    w = diagnostics.weights(g)
    for m in (1, 2, 4):
        assert abs(np.sum(np.cos(m * g.PH) * w)) < 1e-13 * np.sum(w)


def _w_no_r_map(grid):          # planted: dr = dx (drops r Lh)
    wr = spectral.clenshaw_curtis_weights(grid.nr)
    wt = spectral.clenshaw_curtis_weights(grid.nth) * grid.Th
    return (2 * np.pi / grid.nph) * wt[None, :, None] * wr[None, None, :] * np.ones(grid.shape)


def _w_linear_map(grid):        # planted: dr = Lh dx as for a linear map
    wr = spectral.clenshaw_curtis_weights(grid.nr) * 0.5 * (grid.r_out - grid.r_in)
    wt = spectral.clenshaw_curtis_weights(grid.nth) * grid.Th
    return (2 * np.pi / grid.nph) * wt[None, :, None] * wr[None, None, :] * np.ones(grid.shape)


def _w_no_theta_map(grid):      # planted: d theta = dy
    wr = spectral.clenshaw_curtis_weights(grid.nr) * grid.r * grid.Lh
    wt = spectral.clenshaw_curtis_weights(grid.nth)
    return (2 * np.pi / grid.nph) * wt[None, :, None] * wr[None, None, :] * np.ones(grid.shape)


def _w_phi_measure(grid):       # planted: 1/N in place of 2 pi/N
    wr = spectral.clenshaw_curtis_weights(grid.nr) * grid.r * grid.Lh
    wt = spectral.clenshaw_curtis_weights(grid.nth) * grid.Th
    return (1.0 / grid.nph) * wt[None, :, None] * wr[None, None, :] * np.ones(grid.shape)


def _w_sin_theta(grid):         # planted: spherical measure folded into w
    return diagnostics.weights(grid) * grid.R ** 2 * np.sin(grid.TH)


@pytest.mark.parametrize("planted", [_w_no_r_map, _w_linear_map, _w_no_theta_map, _w_phi_measure, _w_sin_theta])
def test_weights_pin_rejects_planted_mistakes(planted):
    assert max(weight_errors(planted).values()) > 1e-3


# ---- discrete entropy -----------------------------------------------------------

def flat_fluid(nr, nth, nph, rho, p, Gamma=4.0 / 3.0):
    """Oracle problem and state of a fluid at rest without field on flat space
    (M = 0), densities given on the grid."""
    g = spectral.Grid(nr, nth, nph, R_IN, R_OUT, TH0, TH1)
    pb = evolve.Problem(g, M=0.0, a=0.0, Gamma=Gamma, cowling=True)
    f = initial_data.kerr_schild_bssn(g, 0.0, 0.0)
    gam = np.exp(4.0 * f['phi']) * f['gt']
    sqrtg = np.exp(6.0 * f['phi']) * np.sqrt(np.linalg.det(np.moveaxis(f['gt'], (0, 1), (-2, -1))))
    rho = np.broadcast_to(rho, g.shape).copy()
    p = np.broadcast_to(p, g.shape).copy()
    zero = np.zeros((3,) + g.shape)
    D, S, tau = prim_to_cons(rho, p, zero, zero, gam, Gamma)
    U = evolve.pack(f, dict(sD=sqrtg * D, sS=sqrtg * S, stau=sqrtg * tau, sB=sqrtg * zero))
    return g, pb, U


def entropy_errors(entropy_fn, Gamma=4.0 / 3.0):
    """Relative errors of E^n against closed forms: (a) uniform rho0, p0 at
    rest, E = rho0 ln(p0/rho0^Gamma)/(Gamma-1) x the wedge volume; (b) rho =
    rho0 (r_in/r)(1 + cos^2 theta / 2), uniform p0, against scipy's quadrature
    of the same integrand in r and theta."""
    rho0, p0 = 2.5e-3, 4.0e-5          # rho0 != 1 so that rho^Gamma matters
    out = {}
    g, pb, U = flat_fluid(30, 28, 6, rho0, p0, Gamma)
    vol = 2 * np.pi * (R_OUT ** 3 - R_IN ** 3) / 3 * (np.cos(TH0) - np.cos(TH1))
    s0 = np.log(p0 / rho0 ** Gamma) / (Gamma - 1)
    ex = rho0 * s0 * vol
    out["uniform"] = abs(entropy_fn(pb, U) - ex) / abs(ex)

    def rho_of(r, th):
        return rho0 * (R_IN / r) * (1 + 0.5 * np.cos(th) ** 2)

    gp = spectral.Grid(40, 32, 6, R_IN, R_OUT, TH0, TH1)
    g, pb, U = flat_fluid(40, 32, 6, rho_of(gp.R, gp.TH), p0, Gamma)

    def integrand(r, th):
        rh = rho_of(r, th)
        return rh * np.log(p0 / rh ** Gamma) / (Gamma - 1) * r * r * np.sin(th)

    val, abserr = integrate.dblquad(integrand, TH0, TH1, R_IN, R_OUT, epsabs=0, epsrel=1e-12)
    ex = 2 * np.pi * val
    out["profile"] = abs(entropy_fn(pb, U) - ex) / abs(ex)
    return out


def test_entropy_matches_closed_forms():
    err = entropy_errors(diagnostics.entropy)
    assert err["uniform"] < 1e-12, err
    assert err["profile"] < 1e-10, err


def _s_no_gamma(problem, U):    # planted: ln(p/rho) in place of ln(p/rho^Gamma)
    P = problem.primitives(U)
    s = np.log(P['p'] / P['rho']) / (problem.Gamma - 1.0)
    return float(np.sum(P['rho'] * s * P['sqrtg'] * diagnostics.weights(problem.g)))


def _s_no_sqrtg(problem, U):    # planted: coordinate volume without sqrt(gamma)
    P = problem.primitives(U)
    s = np.log(P['p'] / P['rho'] ** problem.Gamma) / (problem.Gamma - 1.0)
    return float(np.sum(P['rho'] * s * diagnostics.weights(problem.g)))


def _s_densitised(problem, U):  # planted: the densitised D in place of rho
    P = problem.primitives(U)
    s = np.log(P['p'] / P['rho'] ** problem.Gamma) / (problem.Gamma - 1.0)
    return float(np.sum(U[24] * s * P['sqrtg'] * diagnostics.weights(problem.g)))


def _s_gamma_sign(problem, U):  # planted: (Gamma + 1) in the denominator
    P = problem.primitives(U)
    s = np.log(P['p'] / P['rho'] ** problem.Gamma) / (problem.Gamma + 1.0)
    return float(np.sum(P['rho'] * s * P['sqrtg'] * diagnostics.weights(problem.g)))


@pytest.mark.parametrize("planted", [_s_no_gamma, _s_no_sqrtg, _s_densitised, _s_gamma_sign])
def test_entropy_pin_rejects_planted_mistakes(planted):
    assert max(entropy_errors(planted).values()) > 1e-3


# ---- 2/3 truncation of Chebyshev modes ----------------------------------------

def truncate_errors(trunc_fn):
    """Largest deviation from the 2/3 rule over single Chebyshev modes T_k
    along r (axis -1) and theta (axis -2), for N = 16 (cut-off exactly 10),
    N = 17 (10.67) and N = 13 (8): a kept mode must come back unchanged, a
    removed one as zero."""
    worst = 0.0
    for n in (16, 17, 13):
        x = spectral.cgl_nodes(n)
        cut = 2.0 * (n - 1) / 3.0
        for k in range(n):
            Tk = npcheb.chebval(x, [0] * k + [1])
            want = Tk if k <= cut else np.zeros(n)
            for axis, shape in ((-1, (3, 2, n)), (-2, (3, n, 2))):
                f = np.broadcast_to(Tk[:, None] if axis == -2 else Tk, shape)
                got = trunc_fn(f, axis)
                exp = np.broadcast_to(want[:, None] if axis == -2 else want, shape)
                worst = max(worst, np.abs(got - exp).max())
    return worst


def test_cheb_truncate_two_thirds_rule():
    assert truncate_errors(spectral.cheb_truncate) < 1e-13


def test_dealias_composes_the_three_axes():
    """Grid.dealias on T_a(x) T_b(y) cos(m phi): kept exactly when all three
    modes are within the rule, removed when any one is above it."""
    g = spectral.Grid(16, 13, 12, R_IN, R_OUT, TH0, TH1)
    X = np.broadcast_to(g.x[None, None, :], g.shape)
    Y = np.broadcast_to(g.y[None, :, None], g.shape)
    for a, b, m, kept in ((10, 8, 4, True), (11, 8, 4, False), (10, 9, 4, False), (10, 8, 5, False),
                          (0, 0, 0, True), (3, 2, 1, True)):
        f = npcheb.chebval(X, [0] * a + [1]) * npcheb.chebval(Y, [0] * b + [1]) * np.cos(m * g.PH)
        out = g.dealias(f)
        assert np.abs(out - (f if kept else 0.0)).max() < 1e-13


def _tr_strict(f, axis):        # planted: k < 2(N-1)/3 (drops the boundary mode)
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    coef, shp = spectral._to_coeffs(f, axis)
    coef = coef * (np.arange(n) < 2.0 * (n - 1) / 3.0)[:, None]
    return spectral._from_coeffs(coef, n, shp, axis)


def _tr_n_not_nm1(f, axis):     # planted: 2N/3 in place of 2(N-1)/3
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    coef, shp = spectral._to_coeffs(f, axis)
    coef = coef * (np.arange(n) <= 2.0 * n / 3.0)[:, None]
    return spectral._from_coeffs(coef, n, shp, axis)


def _tr_nodal(f, axis):         # planted: cut applied to node values, not modes
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    keep = (np.arange(n) <= 2.0 * (n - 1) / 3.0).astype(float)
    shape = [1] * f.ndim
    shape[axis] = n
    return f * keep.reshape(shape)


@pytest.mark.parametrize("planted", [_tr_strict, _tr_n_not_nm1, _tr_nodal])
def test_cheb_truncate_pin_rejects_planted_mistakes(planted):
    assert truncate_errors(planted) > 0.5
