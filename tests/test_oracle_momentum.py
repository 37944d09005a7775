"""Pins for the oracle's momentum constraint (bssn.momentum; the coupled
evolution's constraint monitoring, Results, coupled-evolution passage, and
Methods, "Initial Data Solver XCTS Approximation": the Hamiltonian and
momentum constraints):

  * exact data on flat space (tests/momentum_case.py): Bowen-York extrinsic
    curvature, a trace K = k0 x and the balancing momentum density: M_i
    converges to 0 spectrally (below 1e-8 of the cancelling terms at 32^2);
  * a fluid in motion on flat space with K_ij = 0: M_i = -8 pi S_i exactly;
  * vacuum Kerr-Schild (stationary, so its constraints vanish): M_i converges
    to 0 geometrically in the resolution.

Each pin runs on planted copies of the formula too (a dropped 6 At d phi
term, a dropped Christoffel term, (1/3) for (2/3) d K, the opposite sign of
the matter term, S^i in place of S_i, the derivative of the inverse metric
left out) and must reject them."""

import numpy as np
import pytest

from momentum_case import bowen_york_state, scale
from oracle import bssn, diagnostics, initial_data, spectral
from oracle.bssn import conformal_christoffel, inv3

PI = np.pi


def derivs(g, f):
    return dict(phi=np.array([g.d1(f['phi'], k) for k in range(3)]),
                gt=np.array([[[g.d1(f['gt'][i, j], k) for j in range(3)] for i in range(3)] for k in range(3)]),
                At=np.array([[[g.d1(f['At'][i, j], k) for j in range(3)] for i in range(3)] for k in range(3)]),
                K=np.array([g.d1(f['K'], k) for k in range(3)]))


def by_error(mom_fn, n):
    g, pb, U, f, S = bowen_york_state(n, n, 8)
    M = mom_fn(f, derivs(g, f), S)
    return np.abs(bssn.momentum_norm(f, M)).max() / scale(f, S)


def fluid_error(mom_fn):
    """Flat space, K_ij = 0, a fluid with momentum density S_i: M = -8 pi S."""
    g, pb, U, f, S = bowen_york_state(12, 10, 8, P=(0.0, 0.0, 0.0), k0=0.0)
    R, TH = g.R, g.TH
    S = np.array([1e-3 * np.cos(TH) / R, 2e-3 * np.sin(TH), 5e-4 * R * np.sin(TH) ** 2])
    M = mom_fn(f, derivs(g, f), S)
    return np.abs(M + 8.0 * PI * S).max() / np.abs(8.0 * PI * S).max()


def ks_errors(mom_fn):
    out = []
    for n in (16, 24):
        g = spectral.Grid(n, n, 4, 1.8, 20.0, 0.4, np.pi - 0.4)
        f = initial_data.kerr_schild_bssn(g, 1.0, 0.5)
        M = mom_fn(f, derivs(g, f), np.zeros((3,) + g.shape))
        out.append(np.abs(bssn.momentum_norm(f, M)).max())
    return out


def test_momentum_constraint_vanishes_on_bowen_york_data():
    e24, e32 = by_error(bssn.momentum, 24), by_error(bssn.momentum, 32)
    assert e32 < 1e-8
    assert e32 < 1e-2 * e24           # spectral convergence


def test_momentum_constraint_of_a_fluid_is_minus_8_pi_S():
    assert fluid_error(bssn.momentum) < 1e-14


def test_momentum_constraint_vanishes_on_vacuum_kerr_schild():
    e16, e24 = ks_errors(bssn.momentum)
    assert e24 < 1e-6 and e24 < 1e-2 * e16


def test_diagnostics_momentum_constraint_reads_the_state():
    """diagnostics.momentum_constraint takes S_i from the densitised state
    (no primitive recovery) and reports the same M as bssn.momentum; the
    norms of constraint_norms are the weighted L2 and the max."""
    g, pb, U, f, S = bowen_york_state(24, 24, 8)
    M, Mn = diagnostics.momentum_constraint(pb, U)
    ref = bssn.momentum(f, derivs(g, f), S)
    assert np.abs(M - ref).max() < 1e-13 * scale(f, S)
    c = diagnostics.constraint_norms(pb, U)
    w = diagnostics.weights(g)
    assert abs(c['mom_l2'] - np.sqrt(np.sum(Mn ** 2 * w) / np.sum(w))) < 1e-15
    assert c['mom_linf'] == Mn.max()


# ---- planted mistakes --------------------------------------------------------

def _planted(drop_phi=False, drop_gamma=False, k_third=False, s_sign=1.0, s_up=False, drop_dgtu=False):
    def mom(f, d, S_lo):
        gt, At = f['gt'], f['At']
        gtu = inv3(gt)
        dgt = d['gt']
        _, Gu = conformal_christoffel(gtu, dgt)
        dgtu = -np.einsum('ja...,lb...,kab...->kjl...', gtu, gtu, dgt)
        Amix = np.einsum('jk...,ki...->ji...', gtu, At)
        divA = np.einsum('jk...,jki...->i...', gtu, d['At'])
        if not drop_dgtu:
            divA = divA + np.einsum('jjk...,ki...->i...', dgtu, At)
        trG = np.einsum('jjk...->k...', Gu)
        DdivA = divA + np.einsum('k...,ki...->i...', trG, Amix)
        if not drop_gamma:
            DdivA = DdivA - np.einsum('kji...,jk...->i...', Gu, Amix)
        out = DdivA - (1.0 / 3.0 if k_third else 2.0 / 3.0) * d['K']
        if not drop_phi:
            out = out + 6.0 * np.einsum('ji...,j...->i...', Amix, d['phi'])
        S = S_lo
        if s_up:
            S = np.exp(-4.0 * f['phi']) * np.einsum('ij...,j...->i...', gtu, S_lo)
        return out - s_sign * 8.0 * PI * S
    return mom


PLANTED = {
    "no 6 At dphi": _planted(drop_phi=True),
    "no Christoffel term": _planted(drop_gamma=True),
    "(1/3) dK": _planted(k_third=True),
    "+8 pi S": _planted(s_sign=-1.0),
    "S^i for S_i": _planted(s_up=True),
    "no d gt^-1": _planted(drop_dgtu=True),
}


@pytest.mark.parametrize("name", sorted(PLANTED))
def test_momentum_pins_reject_planted_mistakes(name):
    fn = PLANTED[name]
    caught = by_error(fn, 24) > 1e-3 or fluid_error(fn) > 1e-3 or ks_errors(fn)[1] > 1e-3
    assert caught, name
