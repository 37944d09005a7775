"""Pins for the oracle's time stepping, boundary treatment, initial data and
diagnostics (Methods: Time Integration, The Stability and Complexity; Results:
Magnetic Constraint, Entropy Curve)."""

import json
import os

import numpy as np
import pytest

from oracle import spectral, evolve, initial_data, diagnostics, kerr_schild as ks

R_IN, R_OUT, TH0, TH1 = 1.8, 20.0, 0.05, np.pi - 0.05
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def grid16():
    return spectral.Grid(16, 16, 16, R_IN, R_OUT, TH0, TH1)


def test_cfl_time_step_closed_form():
    """dt = 0.25 min(dr, r dtheta, r sin(theta) dphi); on the 16^3 grid the
    azimuthal spacing at r_in, theta = 0.05 is the smallest."""
    pb = evolve.Problem(grid16())
    assert abs(pb.dt() - 0.25 * 1.8 * np.sin(0.05) * 2 * np.pi / 16) < 1e-16
    g = spectral.Grid(64, 64, 128, R_IN, R_OUT, TH0, TH1)
    dr = 1.8 * (np.exp(0.5 * np.log(20 / 1.8) * (1 - np.cos(np.pi / 63))) - 1)
    assert abs(evolve.Problem(g).dt() - 0.25 * dr) < 1e-15


def test_rk4_global_order_four(monkeypatch):
    """Classic RK4 tableau: global error O(dt^4) on y' = lambda y."""
    g = spectral.Grid(4, 4, 4, R_IN, R_OUT, TH0, TH1)
    pb = evolve.Problem(g, filter_on=False)
    lam = -1.3 + 0.0
    monkeypatch.setattr(pb, "rhs", lambda U, K0: lam * U)
    U0 = np.ones((32,) + g.shape)
    errs = []
    for n in (10, 20, 40, 80):
        U = pb.evolve(U0, None, 1.0 / n, n)
        errs.append(abs(U[0, 0, 0, 0] - np.exp(lam)))
    slopes = -np.diff(np.log(errs)) / np.log(2)
    assert np.all(np.abs(slopes - 4) < 0.1)


def test_boundary_nodes_are_frozen():
    g = spectral.Grid(10, 8, 6, R_IN, R_OUT, TH0, TH1)
    pb = evolve.Problem(g)
    U, K0, _ = evolve.initial_state(g, pb)
    R = pb.rhs(U, K0)
    assert np.all(R[..., 0] == 0) and np.all(R[:, :, 0, :] == 0) and np.all(R[:, :, -1, :] == 0)
    assert np.abs(R[..., 1:]).max() > 0


def test_splitmix64_reference_outputs():
    tab = json.load(open(os.path.join(GOLD, "splitmix64_seed0.json")))
    step = int(tab["state_step"], 16)
    for n, out in enumerate(tab["outputs"]):
        assert initial_data.splitmix64((n * step) & ((1 << 64) - 1)) == int(out, 16)
    u = initial_data.uniform01(1, 1000)
    assert u.min() >= 0 and u.max() < 1 and abs(u.mean() - 0.5) < 0.05


def test_michel_closed_form_relations():
    """Mass flux rho u r^2 and Bernoulli h^2 (1 - 2M/r + u^2) are constant;
    at r_c: u^2 = M/(2 r_c) and c_s^2 = u^2/(1 - 3u^2); inflow is supersonic
    inside r_c and subsonic outside."""
    G = 4.0 / 3.0
    mic = initial_data.Michel(1.0, G, 8.0, 1e-8)
    r = spectral.Grid(32, 4, 4, R_IN, R_OUT, TH0, TH1).r
    rho, p, ur = mic.profile(r)
    T = p / rho
    h = 1 + T * G / (G - 1)
    flux = rho * ur * r ** 2
    bern = h ** 2 * (1 - 2 / r + ur ** 2)
    assert np.abs(flux / flux[0] - 1).max() < 1e-12
    assert np.abs(bern / bern[0] - 1).max() < 1e-13
    assert abs(-flux[0] - mic.rho_c * 0.25 * 64) < 1e-20
    cs2 = G * T / h
    V2 = ur ** 2 / (1 - 2 / r + ur ** 2)
    outside = r > 8.2
    inside = (r < 7.8) & (r > 2.0)
    assert np.all(V2[outside] < cs2[outside]) and np.all(V2[inside] > cs2[inside])
    Tc = mic.temperature(8.0)
    assert abs(Tc / mic.Tc - 1) < 1e-6
    assert abs(G * mic.Tc / (1 + 4 * mic.Tc) - (1 / 16) / (1 - 3 / 16)) < 1e-15


def test_initial_data_properties():
    g = grid16()
    pb = evolve.Problem(g)
    U, K0, mat = evolve.initial_state(g, pb)
    f, m = evolve.unpack(U)
    # BSSN metric reproduces the Kerr-Schild spatial metric and sqrt(gamma)
    alpha, beta, gam = ks.adm(g.R, g.TH, 1.0, 0.5)
    gam_b = np.exp(4 * f['phi']) * f['gt']
    assert np.abs(gam_b - gam).max() < 1e-12 * np.abs(gam).max()
    from oracle.grmhd import det3
    assert np.abs(det3(f['gt']) - 1).max() < 1e-13
    # minimum plasma beta is the requested 100 (before the density perturbation)
    from oracle.grmhd import magnetic
    _, _, _, b2 = magnetic(mat['v'], mat['B'], gam_b)
    assert abs(np.min(2 * mat['p'] / b2) - 100.0) < 1e-9
    # seeded perturbation is within +-1e-6 and matches the SplitMix64 stream
    pb0 = evolve.Problem(g)
    _, _, mat0 = evolve.initial_state(g, pb0, pert_amp=0.0)
    rel = mat['rho'] / mat0['rho'] - 1
    assert np.abs(rel).max() <= 1e-6 * (1 + 1e-9)
    u = initial_data.uniform01(1, g.npts).reshape(g.shape)
    assert np.abs(rel - 1e-6 * (2 * u - 1)).max() < 1e-15
    # con2prim recovers the primitives the data were built from
    P = pb.primitives(U)
    assert not P['fail'].any()
    assert np.abs(P['rho'] / mat['rho'] - 1).max() < 1e-13
    # magnetic constraint: the monopole is discretely divergence free
    divB = diagnostics.div_B(pb, U)
    assert np.abs(divB).max() < 1e-12 * np.abs(U[29]).max()


def test_michel_cowling_stationary_a0():
    """a = 0, fixed metric: magnetised Michel flow is an exact stationary
    solution, so the GRMHD right-hand side of D, S_r, tau vanishes to
    truncation + round-off and that of S_theta falls geometrically with the
    theta resolution."""
    out = []
    for nth in (16, 32):
        g = spectral.Grid(24, nth, 4, R_IN, R_OUT, TH0, TH1)
        pb = evolve.Problem(g, a=0.0, cowling=True)
        U, K0, _ = evolve.initial_state(g, pb, pert_amp=0.0)
        R = pb.rhs(U, K0)
        inner = (slice(None), slice(1, -1), slice(1, None))
        for v in (24, 25, 28):
            assert np.abs(R[v][inner]).max() < 1e-11 * np.abs(U[v]).max()
        assert np.abs(R[:24]).max() == 0
        out.append(np.abs(R[26][inner]).max() / np.abs(U[25]).max())
    assert out[1] < out[0] / 20


def test_cowling_background_fixed_through_steps():
    """Fixed-background form: after RK4 steps with the filter on, the 24
    spacetime fields are bit-identical to the initial data while the GRMHD
    fields have moved (a = 0.5, where the Michel flow is not stationary)."""
    g = spectral.Grid(10, 8, 6, R_IN, R_OUT, TH0, TH1)
    pb = evolve.Problem(g, a=0.5, cowling=True, filter_on=True)
    U, K0, _ = evolve.initial_state(g, pb, pert_amp=1e-4)
    V = pb.evolve(U, K0, pb.dt(), 2)
    assert np.array_equal(V[:24], U[:24])
    assert np.abs(V[24:] - U[24:]).max() > 0
    # the coupled form does change the spacetime (filter and RHS)
    pc = evolve.Problem(g, a=0.5, cowling=False, filter_on=True)
    W = pc.evolve(U, K0, pc.dt(), 1)
    assert np.abs(W[:24] - U[:24]).max() > 0


def test_split_step_sub_steps_and_first_order():
    """Operator-split coupled step (symmetric reading): its fluid sub-step
    leaves the spacetime bit for bit and its Euler sub-step the matter; and
    it converges to the unsplit RK4 solution at first order in dt (the
    forward-Euler spacetime update): halving dt halves the difference, for the
    spacetime and the matter fields alike."""
    g = spectral.Grid(8, 8, 6, R_IN, R_OUT, TH0, TH1)
    pu = evolve.Problem(g, a=0.5, filter_on=False)
    ps = evolve.Problem(g, a=0.5, filter_on=False, split=True)
    U, K0, _ = evolve.initial_state(g, pu, pert_amp=1e-3)
    dt = pu.dt()
    V = ps.fluid_rk4(U, K0, 0.5 * dt)
    assert np.array_equal(V[:24], U[:24]) and np.abs(V[24:] - U[24:]).max() > 0
    T = 2 * dt
    ref = pu.evolve(U, K0, T / 32, 32)
    groups = [list(range(24)), [24], [25, 26, 27], [28], [29, 30, 31]]
    errs = []
    for n in (2, 4, 8):
        W = ps.evolve(U, K0, T / n, n)
        errs.append([np.abs(W[q] - ref[q]).max() / np.abs(ref[q]).max() for q in groups])
    errs = np.array(errs)
    assert np.all(errs[0] > 0)
    ratios = errs[:-1] / errs[1:]
    assert np.all(ratios[:, 0] > 1.9) and np.all(ratios[:, 0] < 2.1), ratios
    assert np.all(ratios > 1.6) and np.all(ratios < 2.6), ratios
    with pytest.raises(ValueError):
        evolve.Problem(g, cowling=True, split=True)


@pytest.mark.slow
def test_ten_steps_small_grid_sane():
    g = grid16()
    pb = evolve.Problem(g)
    U, K0, _ = evolve.initial_state(g, pb)
    m0 = diagnostics.rest_mass(pb, U)
    V = pb.evolve(U, K0, pb.dt(), 10)
    assert np.all(np.isfinite(V))
    assert not pb.last_fail.any()
    assert abs(diagnostics.rest_mass(pb, V) / m0 - 1) < 1e-4


@pytest.mark.parametrize("field", [False, True])
def test_flat_space_hydrostatic_balance(field):
    """Flat space (M = 0, spherical coordinates r, theta, phi): a uniform fluid
    at rest is static.  In the conservative form the flux divergence
    -d_r(alpha sqrt(gamma) p) is nonzero (sqrt(gamma) = r^2 sin(theta)) and
    must be cancelled by the geometric source (1/2) alpha sqrt(gamma)
    S^{kl} d_r gamma_kl, which the oracle builds from the spectral
    derivatives of the BSSN variables; with a uniform Cartesian field B_z
    (B^r = cos(theta) B, B^theta = -sin(theta) B / r) the magnetic stresses
    balance as well.  The radial momentum right-hand side vanishes to
    round-off once r is resolved; the polar one (through the conformal
    variables, singular just outside the theta interval) falls geometrically
    with the resolution; nothing drives D, S_phi, tau or B."""
    from oracle.grmhd import prim_to_cons
    s_r, s_th = [], []
    for n in (12, 20, 28):
        g = spectral.Grid(n, n, 4, R_IN, R_OUT, TH0, TH1)
        pb = evolve.Problem(g, M=0.0, a=0.0, cowling=True)
        f = initial_data.kerr_schild_bssn(g, 0.0, 0.0)
        gam = np.exp(4.0 * f['phi']) * f['gt']
        sqrtg = np.exp(6.0 * f['phi']) * np.sqrt(np.linalg.det(np.moveaxis(f['gt'], (0, 1), (-2, -1))))
        rho = np.full(g.shape, 1e-2)
        p = np.full(g.shape, 1e-3)
        v = np.zeros((3,) + g.shape)
        B = np.zeros((3,) + g.shape)
        if field:
            B[0] = 0.05 * np.cos(g.TH)
            B[1] = -0.05 * np.sin(g.TH) / g.R
        D, S, tau = prim_to_cons(rho, p, v, B, gam, pb.Gamma)
        U = evolve.pack(f, dict(sD=sqrtg * D, sS=sqrtg * S, stau=sqrtg * tau, sB=sqrtg * B))
        R = pb.rhs(U, evolve.gauge_source_k0(g, f))
        # scale: the radial pressure-divergence term d_r(sqrt(gamma) p)
        scale = np.abs(g.d1(sqrtg * p, 0)).max()
        inner = (slice(None), slice(1, -1), slice(1, None))
        s_r.append(np.abs(R[25][inner]).max() / scale)
        s_th.append(np.abs(R[26][inner]).max() / scale)
        for q in (24, 27, 28, 29, 30, 31):
            assert np.abs(R[q]).max() <= 1e-13 * scale
    assert s_r[1] < 1e-10 and s_r[2] < 1e-10
    assert s_th[2] < s_th[0] / 20


@pytest.mark.parametrize("field", [False, True])
def test_flat_space_advection_rate_closed_form(field):
    """Matter right-hand side pinned by an exact solution: a density blob
    carried at uniform velocity through flat space in the solver's spherical
    coordinates (tests/advection_case.py gives the exact rates), without and
    with a magnetic flux tube along the flow.  Without the field D, S_r and
    tau converge spectrally to the exact rates and S_theta geometrically in
    n_theta (the polar truncation of the conformal variables, as for the fluid
    at rest); with the tube the magnetic stresses converge at >= 3x per
    refinement.  S_phi (no azimuthal motion) and the induction rates vanish.
    A dropped or halved geometric source, transposed momentum-flux indices, a
    stress without -b_i b_j or a momentum flux without the b_j B^i / W term
    fail it."""
    from advection_case import advection_errors, flat_advection_state
    sizes = ((32, 32, 48), (40, 40, 64)) if field else ((24, 24, 32), (32, 32, 48))
    errs = []
    for n in sizes:
        g, pb, U, K0, exact = flat_advection_state(*n, field=field)
        e, induction = advection_errors(pb.rhs(U, K0), exact)
        errs.append(e)
        assert induction < 1e-14 and e[3] < 1e-12
    coarse, fine = errs
    if not field:
        for q in (0, 1, 4):  # D, S_r, tau
            assert fine[q] < 1e-3 and fine[q] < coarse[q] / 20, (q, coarse, fine)
        assert fine[2] < 0.1 and fine[2] < coarse[2] / 4, (coarse, fine)
    else:
        assert fine[0] < coarse[0] / 20, (coarse, fine)
        for q, bar in ((1, 1e-2), (2, 0.1), (4, 0.2)):  # S_r, S_theta, tau
            assert fine[q] < bar and fine[q] < coarse[q] / 3, (q, coarse, fine)
