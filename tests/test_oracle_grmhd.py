"""Pins for the oracle's GRMHD pieces against the covariant definitions
(Results: GRMHD Conservative Form, stress-energy tensor of fluid + field,
flux freezing *F = u b - b u; Methods: Primitive Variable Recovery, Conserved
Fluxes and Geometric Source Terms).

The 3+1 closed forms used by the oracle are checked against an independent
route: the 4-metric assembled from (alpha, beta, gamma), u^mu, the projection
b^mu = (delta + u u)^mu_nu F^nu / u^0 of the field F^i = B^i/alpha, and
T^{mu nu} = (rho h + b^2) u u + (p + b^2/2) g^{-1} - b b contracted with the
normal observer n_mu = (-alpha, 0, 0, 0)."""

import numpy as np
import pytest

from oracle import grmhd, kerr_schild as ks


def random_spd(rng, n):
    A = rng.standard_normal((n, 3, 3)) * 0.3
    g = np.einsum('nij,nkj->nik', A, A) + np.eye(3)[None] * rng.uniform(0.5, 3.0, (n, 1, 1))
    return np.moveaxis(g, 0, -1)  # (3, 3, n)


def random_state(rng, n, W_max=10.0, sig_max=100.0, zero_B=False, zero_v=False, gam=None):
    gam = random_spd(rng, n) if gam is None else gam
    rho = 10 ** rng.uniform(-10, 0, n)
    eps = 10 ** rng.uniform(-6, 1, n)
    G = 4.0 / 3.0
    p = (G - 1) * rho * eps
    W = rng.uniform(1.0, W_max, n)
    dirv = rng.standard_normal((3, n))
    vv = np.einsum('i...,i...->...', grmhd.lower(gam, dirv), dirv)
    v = dirv * np.sqrt((1 - 1 / W ** 2) / vv)
    if zero_v:
        v[:] = 0
    dirb = rng.standard_normal((3, n))
    B = dirb
    if zero_B:
        B = np.zeros_like(dirb)
    else:
        _, _, _, b2 = grmhd.magnetic(v, B, gam)
        sig = 10 ** rng.uniform(-4, np.log10(sig_max), n)
        B = B * np.sqrt(sig * rho / b2)
    alpha = rng.uniform(0.3, 1.2, n)
    beta = rng.standard_normal((3, n)) * 0.3
    return dict(gam=gam, rho=rho, p=p, v=v, B=B, alpha=alpha, beta=beta, G=G)


def covariant(s):
    """u^mu, b^mu, 4-metric and T^{mu nu} from the definitions."""
    gam, alpha, beta = s['gam'], s['alpha'], s['beta']
    n = alpha.shape[-1]
    beta_lo = grmhd.lower(gam, beta)
    g4 = np.zeros((4, 4, n))
    g4[0, 0] = -alpha ** 2 + np.einsum('i...,i...->...', beta_lo, beta)
    g4[0, 1:] = beta_lo
    g4[1:, 0] = beta_lo
    g4[1:, 1:] = gam
    g4inv = np.moveaxis(np.linalg.inv(np.moveaxis(g4, (0, 1), (-2, -1))), (-2, -1), (0, 1))
    W = grmhd.lorentz(s['v'], gam)
    u = np.zeros((4, n))
    u[0] = W / alpha
    u[1:] = W * (s['v'] - beta / alpha)
    u_lo = np.einsum('mn...,n...->m...', g4, u)
    F = np.zeros((4, n))
    F[1:] = s['B'] / alpha
    proj = np.eye(4)[:, :, None] + np.einsum('m...,n...->mn...', u, u_lo)
    b = np.einsum('mn...,n...->m...', proj, F) / u[0]
    b2 = np.einsum('mn...,m...,n...->...', g4, b, b)
    G = s['G']
    h = 1 + p_over(s) * G / (G - 1)
    T = (s['rho'] * h + b2) * np.einsum('m...,n...->mn...', u, u) + (s['p'] + 0.5 * b2) * g4inv \
        - np.einsum('m...,n...->mn...', b, b)
    return dict(g4=g4, g4inv=g4inv, u=u, b=b, b2=b2, T=T, W=W)


def p_over(s):
    return s['p'] / s['rho']


def test_conserved_variables_match_covariant_definition():
    rng = np.random.default_rng(11)
    s = random_state(rng, 400)
    c = covariant(s)
    D, S, tau = grmhd.prim_to_cons(s['rho'], s['p'], s['v'], s['B'], s['gam'], s['G'])
    alpha = s['alpha']
    D_cov = s['rho'] * alpha * c['u'][0]
    T0_lo = np.einsum('n...,nj...->j...', c['T'][0], c['g4'][:, 1:])   # T^0_j
    S_cov = alpha * T0_lo
    tau_cov = alpha ** 2 * c['T'][0, 0] - D_cov
    assert np.abs(D / D_cov - 1).max() < 1e-13
    scale = np.abs(S_cov).max(axis=0) + tau_cov + D_cov
    assert (np.abs(S - S_cov).max(axis=0) / scale).max() < 1e-11
    assert (np.abs(tau - tau_cov) / (tau_cov + D_cov)).max() < 1e-10
    # and b^2 / alpha b^0 closed forms
    W, ab0, b_lo, b2 = grmhd.magnetic(s['v'], s['B'], s['gam'])
    assert np.abs(b2 / c['b2'] - 1).max() < 1e-10
    assert np.abs(ab0 - alpha * c['b'][0]).max() < 1e-10 * np.sqrt(c['b2']).max()


def test_fluxes_match_covariant_definition():
    rng = np.random.default_rng(12)
    s = random_state(rng, 300)
    c = covariant(s)
    sqrtg = np.sqrt(np.linalg.det(np.moveaxis(s['gam'], (0, 1), (-2, -1))))
    D, S, tau = grmhd.prim_to_cons(s['rho'], s['p'], s['v'], s['B'], s['gam'], s['G'])
    F = grmhd.fluxes(D, S, tau, s['B'], s['rho'], s['p'], s['v'], s['alpha'], s['beta'], s['gam'], sqrtg)
    sqg4 = s['alpha'] * sqrtg
    u, b, T = c['u'], c['b'], c['T']
    Tmix = np.einsum('in...,nj...->ij...', T[1:], c['g4'][:, 1:])  # T^i_j
    for i in range(3):
        ref = np.zeros((8,) + s['alpha'].shape)
        ref[0] = sqg4 * s['rho'] * u[1 + i]
        ref[1:4] = sqg4 * Tmix[i]
        ref[4] = sqg4 * (s['alpha'] * T[0, 1 + i] - s['rho'] * u[1 + i])
        for k in range(3):
            ref[5 + k] = sqg4 * (u[1 + i] * b[1 + k] - u[1 + k] * b[1 + i])
        scale = np.abs(ref).max(axis=0) + sqg4 * (tau + D)
        assert (np.abs(F[:, i] - ref).max(axis=0) / scale).max() < 1e-10


def _cstep(fun, x, h=1e-40):
    return np.imag(fun(x + 1j * h)) / h


@pytest.mark.parametrize("a", [0.0, 0.5, 0.9375])
def test_3p1_sources_match_christoffel_form_on_stationary_kerr_schild(a):
    """Sbar_{S_j} = (alpha/2) T^{mu nu} d_j g_{mu nu} and
    Sbar_tau = alpha (T^{mu 0} d_mu alpha - alpha T^{mu nu} Gamma^0_{mu nu})
    for the stationary Kerr-Schild metric (d_t g = 0); derivatives by complex
    step of the closed forms; K_ij = L_beta gamma_ij / (2 alpha)."""
    rng = np.random.default_rng(13)
    n = 50
    r = rng.uniform(1.9, 15.0, n)
    th = rng.uniform(0.2, 2.9, n)
    M = 1.0
    alpha, beta, gam = ks.adm(r, th, M, a)
    s = random_state(rng, n, W_max=3.0, sig_max=10.0, gam=gam)
    s.update(alpha=alpha, beta=beta)
    c = covariant(s)
    # derivatives with respect to x^j = (r, theta, phi); phi-derivatives vanish
    d_adm = []
    for j in range(2):
        def f(z, j=j):
            rr, tt = (z, th) if j == 0 else (r, z)
            al, be, ga = ks.adm(rr, tt, M, a)
            return np.concatenate([al[None], be, ga.reshape(9, -1)])
        d_adm.append(_cstep(f, r if j == 0 else th))
    d_adm.append(np.zeros_like(d_adm[0]))
    d_adm = np.array(d_adm)            # [j, 13, n]
    dalpha = d_adm[:, 0]
    dbeta = d_adm[:, 1:4]              # [j, k] = d_j beta^k
    dgam = d_adm[:, 4:].reshape(3, 3, 3, n)
    Kij = (np.einsum('k...,kij...->ij...', beta, dgam) + np.einsum('ik...,jk...->ij...', gam, dbeta)
           + np.einsum('jk...,ik...->ij...', gam, dbeta)) / (2 * alpha)
    D, S, tau = grmhd.prim_to_cons(s['rho'], s['p'], s['v'], s['B'], gam, s['G'])
    E, Sij = grmhd.matter_3p1(s['rho'], s['p'], s['v'], s['B'], D, tau, gam, s['G'])
    gamu = grmhd.inv3(gam)
    srcS, srcT = grmhd.sources_3p1(E, S, Sij, alpha, dalpha, dbeta, dgam, Kij, gamu)
    # 4-metric derivatives
    dg4 = []
    for j in range(2):
        def f4(z, j=j):
            rr, tt = (z, th) if j == 0 else (r, z)
            return ks.metric4(rr, tt, M, a).reshape(16, -1)
        dg4.append(_cstep(f4, r if j == 0 else th).reshape(4, 4, n))
    dg4 = np.array(dg4 + [np.zeros((4, 4, n))])        # [j, mu, nu]
    T = c['T']
    refS = 0.5 * alpha * np.einsum('mn...,jmn...->j...', T, dg4)
    dg4full = np.concatenate([np.zeros((1, 4, 4, n)), dg4])   # d_t g = 0
    # Gamma^0_{mn} = 1/2 g^{0s} (d_m g_sn + d_n g_sm - d_s g_mn), dg4full[c, m, n] = d_c g_mn
    A = (np.einsum('msn...->mns...', dg4full) + np.einsum('nsm...->mns...', dg4full)
         - np.einsum('smn...->mns...', dg4full))
    Gam0 = 0.5 * np.einsum('s...,mns...->mn...', c['g4inv'][0], A)
    dalpha4 = np.concatenate([np.zeros((1, n)), dalpha])
    refT = alpha * (np.einsum('m...,m...->...', T[:, 0], dalpha4) - alpha * np.einsum('mn...,mn...->...', T, Gam0))
    scaleS = np.abs(refS).max(axis=0) + 1e-300
    assert (np.abs(srcS - refS).max(axis=0) / (scaleS + np.abs(E * dalpha).max(axis=0))).max() < 1e-10
    assert (np.abs(srcT - refT) / (np.abs(refT) + np.abs(E) * np.abs(dalpha).max(axis=0))).max() < 1e-9


@pytest.mark.parametrize("W_max,sig_max,tol", [(2.0, 1.0, 1e-12), (10.0, 100.0, 1e-9)])
def test_con2prim_round_trip(W_max, sig_max, tol):
    rng = np.random.default_rng(14)
    s = random_state(rng, 2000, W_max=W_max, sig_max=sig_max)
    gam = s['gam']
    D, S, tau = grmhd.prim_to_cons(s['rho'], s['p'], s['v'], s['B'], gam, s['G'])
    rho, p, v, fail = grmhd.con2prim(D, S, tau, s['B'], gam, grmhd.inv3(gam), s['G'], 0.0, 0.0)
    assert not fail.any()
    W, _, _, b2 = grmhd.magnetic(s['v'], s['B'], gam)
    assert np.abs(rho / s['rho'] - 1).max() < tol
    # p = (Gamma-1)/Gamma (Z/W^2 - rho) cancels when p << rho: error relative to
    # the scale (rho + p + b^2) W^2 of the quantities it is recovered from
    assert (np.abs(p - s['p']) / ((s['rho'] + s['p'] + b2) * W ** 2)).max() < tol
    assert (np.abs(v - s['v']).max(axis=0) / np.sqrt(1 - 1 / W ** 2 + 1e-30)).max() < tol * 10


@pytest.mark.parametrize("case", ["B0", "v0"])
def test_con2prim_special_cases(case):
    rng = np.random.default_rng(15)
    s = random_state(rng, 500, zero_B=(case == "B0"), zero_v=(case == "v0"))
    gam = s['gam']
    D, S, tau = grmhd.prim_to_cons(s['rho'], s['p'], s['v'], s['B'], gam, s['G'])
    rho, p, v, fail = grmhd.con2prim(D, S, tau, s['B'], gam, grmhd.inv3(gam), s['G'], 0.0, 0.0)
    assert not fail.any()
    W, _, _, b2 = grmhd.magnetic(s['v'], s['B'], gam)
    assert np.abs(rho / s['rho'] - 1).max() < 1e-10
    assert (np.abs(p - s['p']) / ((s['rho'] + s['p'] + b2) * W ** 2)).max() < 1e-12
    if case == "v0":
        assert np.abs(v).max() < 1e-12


def test_con2prim_failure_policy():
    rng = np.random.default_rng(16)
    s = random_state(rng, 10)
    gam = s['gam']
    D, S, tau = grmhd.prim_to_cons(s['rho'], s['p'], s['v'], s['B'], gam, s['G'])
    tau = tau.copy()
    D = D.copy()
    tau[3] = -2.0 * D[3]        # tau + D < 0: unphysical
    D[5] = -1.0                 # negative density
    rho, p, v, fail = grmhd.con2prim(D, S, tau, s['B'], gam, grmhd.inv3(gam), s['G'], 1e-15, 1e-17)
    assert fail[3] and fail[5] and fail.sum() == 2
    assert rho[3] == 1e-15 and p[3] == 1e-17 and np.all(v[:, 3] == 0)


def _damped_from(s, rho0, p0, v0, maxit=40):
    gam = s['gam']
    gamu = grmhd.inv3(gam)
    D, S, tau = grmhd.prim_to_cons(s['rho'], s['p'], s['v'], s['B'], gam, s['G'])
    return grmhd.con2prim_damped(D, S, tau, s['B'], gam, gamu, s['G'], 1e-30, 1e-40, rho0, p0, v0,
                                 maxit=maxit)


def _warm_state(seed, n):
    rng = np.random.default_rng(seed)
    s = random_state(rng, n, W_max=2.0, sig_max=1.0)
    eps = 10 ** rng.uniform(-2, 1, n)
    s['p'] = (s['G'] - 1) * s['rho'] * eps
    return s, eps, rng


def test_damped_con2prim_fixed_point_is_the_known_primitives():
    """The paper's damped iteration (reading: predicted values are the
    conserved variables of the current primitives) converges to the known
    primitives of random warm states (eps >= 10^-2, W <= 2, b^2/rho <= 1) from
    a guess 10^-3 away, given enough tries (1000; with the paper's 30-40 most
    points are not there yet: lambda only ever halves, and the scalar Jacobian
    rho h W^2 underestimates dS/dv by up to 1 + 2 W^2 v^2).  A wrong sign or
    index in the update, or a fixed point other than the inverse, fails
    this."""
    s, eps, rng = _warm_state(11, 400)
    d = 1e-3 * rng.uniform(-1, 1, (5, 400))
    rho0, p0, v0 = s['rho'] * (1 + d[0]), s['p'] * (1 + d[1]), s['v'] * (1 + d[2:5])
    rho, p, v, fail, its = _damped_from(s, rho0, p0, v0, maxit=1000)
    assert not fail.any()
    err = np.abs(rho / s['rho'] - 1)
    assert np.mean(err < 1e-10) > 0.99
    good = err < 1e-10
    # p through the cancellation in tau: relative conditioning ~ 1e-16 / eps
    assert np.all(np.abs(p / s["p"] - 1)[good] < 1e-9 * (1 + 1 / eps[good]))
    assert np.all(np.abs(v - s['v']).max(axis=0)[good] < 1e-9)


def test_damped_con2prim_exact_guess_and_unusable_guess():
    """From the exact primitives the result stays there (to the conditioning
    of tau); a state at rest without field from the fallback start (rho0 = 0)
    gets the exact answer (v = 0, eps = tau/D)."""
    s, eps, rng = _warm_state(12, 50)
    rho, p, v, fail, its = _damped_from(s, s['rho'], s['p'], s['v'])
    assert not fail.any()
    assert np.all(np.abs(rho / s['rho'] - 1) < 1e-12) and np.all(np.abs(p / s["p"] - 1) < 1e-12 * (1 + 1 / eps))
    s = random_state(rng, 50, zero_B=True, zero_v=True)
    epsr = s['p'] / ((s['G'] - 1) * s['rho'])
    rho, p, v, fail, its = _damped_from(s, np.zeros(50), np.zeros(50), np.zeros((3, 50)))
    assert not fail.any()
    assert np.all(np.abs(rho / s['rho'] - 1) < 1e-14) and np.all(np.abs(p / s['p'] - 1) < 1e-14 / epsr)
    assert np.abs(v).max() == 0.0


def test_damped_con2prim_halving_keeps_the_state_physical():
    """A poor guess (velocity scaled by 0.1 at W up to 10, strong fields, cold
    and hot gas): the halving keeps every iterate at v^2 < 1; no NaN comes
    out, and what the tries leave unusable is flagged (atmosphere), not
    returned."""
    rng = np.random.default_rng(13)
    s = random_state(rng, 300, W_max=10.0, sig_max=100.0)
    rho, p, v, fail, its = _damped_from(s, s['rho'], s['p'], 0.1 * s['v'])
    assert np.isfinite(rho).all() and np.isfinite(p).all() and np.isfinite(v).all()
    v2 = np.einsum('i...,i...->...', grmhd.lower(s['gam'], v), v)
    assert np.all(v2 < 1.0)
    assert np.all(rho[fail] == 1e-30) and np.all(p[fail] == 1e-40)
    assert np.all(p[~fail] > 0)


def test_con2prim_unresolved_bracket_is_flagged(monkeypatch):
    """A point whose bracket the bisection budget leaves wider than adjacent
    doubles is not a recovered state: with a budget of 5 halvings every point
    takes the atmosphere and is flagged (the GPU's Newton iteration applies
    the same policy to its own budget)."""
    rng = np.random.default_rng(17)
    s = random_state(rng, 50, W_max=2.0, sig_max=1.0)
    gam = s['gam']
    D, S, tau = grmhd.prim_to_cons(s['rho'], s['p'], s['v'], s['B'], gam, s['G'])
    monkeypatch.setattr(grmhd, "C2P_BISECTIONS", 5)
    rho, p, v, fail = grmhd.con2prim(D, S, tau, s['B'], gam, grmhd.inv3(gam), s['G'], 1e-30, 1e-40)
    assert fail.all() and np.all(rho == 1e-30) and np.all(v == 0)
    monkeypatch.setattr(grmhd, "C2P_BISECTIONS", 2000)
    rho, p, v, fail = grmhd.con2prim(D, S, tau, s['B'], gam, grmhd.inv3(gam), s['G'], 1e-30, 1e-40)
    assert not fail.any()
