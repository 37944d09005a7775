"""Pins of the oracle's GLM constraint-damping terms (Methods, "GLM Constraint
Damping Source") in flat space (M = 0, spherical coordinates), against
closed forms obtained by transforming Cartesian fields:

* psi = x = r sin(theta) cos(phi) has the constant Cartesian gradient e_x,
  so the induction source sqrt(gamma) S^i = -sqrt(gamma) gamma^{ij} d_j psi
  must equal -sqrt(gamma) times the spherical components of e_x, and the
  psi right-hand side with B = 0 is the pure damping -psi / tau;
* B = b (x, 0, 0) has divergence b and B = b (x, y, z) has divergence 3 b, so
  with psi = 0 the psi right-hand side is -c_h^2 b and -3 c_h^2 b."""

import numpy as np
import pytest

from oracle import spectral, evolve, initial_data
from oracle.grmhd import prim_to_cons

R_IN, R_OUT, TH0, TH1 = 1.8, 20.0, 0.05, np.pi - 0.05
CH, TAU = 0.8, 1.7


def cartesian_to_spherical(g, vx, vy, vz):
    """Contravariant spherical components (V^r, V^theta, V^phi) of a Cartesian vector."""
    st, ct, sp, cp = np.sin(g.TH), np.cos(g.TH), np.sin(g.PH), np.cos(g.PH)
    vr = st * cp * vx + st * sp * vy + ct * vz
    vth = (ct * cp * vx + ct * sp * vy - st * vz) / g.R
    vph = (-sp * vx + cp * vy) / (g.R * st)
    return np.array([vr, vth, vph])


def flat_state(g, pb, B, psi):
    f = initial_data.kerr_schild_bssn(g, 0.0, 0.0)
    gam = np.exp(4.0 * f['phi']) * f['gt']
    sqrtg = np.exp(6.0 * f['phi']) * np.sqrt(np.linalg.det(np.moveaxis(f['gt'], (0, 1), (-2, -1))))
    rho = np.full(g.shape, 1e-2)
    p = np.full(g.shape, 1e-3)
    v = np.zeros((3,) + g.shape)
    D, S, tau = prim_to_cons(rho, p, v, B, gam, pb.Gamma)
    U = evolve.pack(f, dict(sD=sqrtg * D, sS=sqrtg * S, stau=sqrtg * tau, sB=sqrtg * B))
    return np.concatenate([U, psi[None]]), evolve.gauge_source_k0(g, f), sqrtg


def problem(n):
    g = spectral.Grid(n, n, 8, R_IN, R_OUT, TH0, TH1)
    return g, evolve.Problem(g, M=0.0, a=0.0, cowling=True, glm=True, glm_ch=CH, glm_tau=TAU)


INNER = (slice(1, -1), slice(1, None))  # theta interior, r without the frozen outer node


def test_gradient_source_and_damping():
    for n in (16, 24):
        g, pb = problem(n)
        ones = np.ones(g.shape)
        psi = g.R * np.sin(g.TH) * np.cos(g.PH) * ones
        U, K0, sqrtg = flat_state(g, pb, np.zeros((3,) + g.shape), psi)
        R = pb.rhs(U, K0)
        want = -sqrtg * cartesian_to_spherical(g, ones, 0 * ones, 0 * ones)
        for i in range(3):
            err = np.abs(R[29 + i][(slice(None),) + INNER] - want[i][(slice(None),) + INNER]).max()
            assert err < 1e-9 * np.abs(want[i]).max(), (n, i, err)
        damp = R[32][(slice(None),) + INNER] - (-psi / TAU)[(slice(None),) + INNER]
        assert np.abs(damp).max() < 1e-15 * np.abs(psi).max()
        assert np.abs(R[32][:, :, 0]).max() == 0.0  # frozen outer boundary


@pytest.mark.parametrize("kind", ["x_only", "radial"])
def test_divergence_source(kind):
    b = 1e-3
    g, pb = problem(20)
    ones = np.ones(g.shape)
    x = g.R * np.sin(g.TH) * np.cos(g.PH)
    y = g.R * np.sin(g.TH) * np.sin(g.PH)
    z = g.R * np.cos(g.TH) * ones
    if kind == "x_only":
        B = cartesian_to_spherical(g, b * x, 0 * ones, 0 * ones)
        div = b
    else:
        B = cartesian_to_spherical(g, b * x, b * y, b * z)
        div = 3.0 * b
    U, K0, _ = flat_state(g, pb, B, np.zeros(g.shape))
    R = pb.rhs(U, K0)
    got = R[32][(slice(None),) + INNER]
    assert np.abs(got + CH ** 2 * div).max() < 1e-9 * CH ** 2 * div


def test_glm_off_leaves_the_system_unchanged():
    """With the flag off the state has 32 fields and the right-hand side is
    the plain one; with it on and psi = 0, B divergence-free, the first 32
    right-hand sides are identical and psi is driven only by the discrete
    divergence of the initial field (round-off for the monopole)."""
    g = spectral.Grid(12, 12, 8, R_IN, R_OUT, TH0, TH1)
    pb0 = evolve.Problem(g)
    pb1 = evolve.Problem(g, glm=True)
    U0, K0, _ = evolve.initial_state(g, pb0)
    U1, K1, _ = evolve.initial_state(g, pb1)
    assert U0.shape[0] == 32 and U1.shape[0] == 33 and np.array_equal(U1[:32], U0)
    R0 = pb0.rhs(U0, K0)
    R1 = pb1.rhs(U1, K1)
    assert np.array_equal(R1[:32], R0)
    assert np.abs(R1[32]).max() < 1e-9 * np.abs(U1[29]).max()
