"""Valencia ideal GRMHD pieces, oracle side (plain NumPy FP64).

Paper: Results, "GRMHD Conservative Form" (conserved variables D, S_j, tau,
B^k; fluxes; Lorentz factor; magnetic four-vector b^mu; source term; magnetic
constraint), Methods, "The Primitive Variable Recovery", "The Conserved Fluxes
and Geometric Source Terms", "Stress-Energy Tensor" and "Ideal-gas EOS".

Readings of the paper taken here (where it is silent or inconsistent):
  * conserved variables: the paper's h* = 1 + eps + p/rho + b^2/rho followed by
    (rho h* + b^2) counts b^2 twice; the standard Valencia form is used:
      D = rho W,  S_j = (rho h W^2 + B^2) v_j - (B.v) B_j,
      tau = rho h W^2 - p + B^2 - (B^2/W^2 + (B.v)^2)/2 - D,
    with h = 1 + eps + p/rho, B^2 = gamma_ij B^i B^j, B.v = gamma_ij B^i v^j.
  * fluxes: the printed fluxes omit lapse and shift; the standard form with
    vt^i = v^i - beta^i/alpha and the conservation law
      d_t(sqrt(gamma) U) + d_i(alpha sqrt(gamma) F^i) = sqrt(gamma) S
    is used; at alpha = 1, beta = 0 it reduces to the printed fluxes.
  * sources: the Christoffel form of the paper is written in the equivalent
    3+1 form (lapse, shift and extrinsic-curvature terms).
  * b^0 in the recovery step means alpha b^0 (only gamma_ij enters).
  * con2prim: the result is the unique primitive state reproducing U; it is
    computed here by bisection on a one-dimensional residual in
    Z = rho h W^2 down to adjacent floating-point numbers (the paper's damped
    iteration is one way to approach the same root).
  * EOS: p = (Gamma - 1) rho eps with the adiabatic index given by the caller.
"""

import numpy as np


def lower(g, v):
    """v_i = g_ij v^j."""
    return np.einsum('ij...,j...->i...', g, v)


def dot(a, b):
    return np.einsum('i...,i...->...', a, b)


def inv3(g):
    """Inverse of a stack of symmetric 3x3 matrices with shape (3, 3, ...)."""
    gm = np.moveaxis(np.moveaxis(g, 0, -1), 0, -1)  # (..., 3, 3)
    inv = np.linalg.inv(gm)
    return np.moveaxis(np.moveaxis(inv, -1, 0), -1, 0)


def det3(g):
    gm = np.moveaxis(np.moveaxis(g, 0, -1), 0, -1)
    return np.linalg.det(gm)


def eos_pressure(rho, eps, Gamma):
    return (Gamma - 1.0) * rho * eps


def eos_eps(rho, p, Gamma):
    return p / ((Gamma - 1.0) * rho)


def lorentz(v_up, gam):
    """W = 1/sqrt(1 - gamma_ij v^i v^j)."""
    return 1.0 / np.sqrt(1.0 - dot(lower(gam, v_up), v_up))


def magnetic(v_up, B_up, gam):
    """Return W, alpha b^0, b_i (lower), b^2 for Eulerian field B^i.

    alpha b^0 = W (B.v); b_i = B_i/W + W (B.v) v_i; b^2 = B^2/W^2 + (B.v)^2."""
    W = lorentz(v_up, gam)
    v_lo = lower(gam, v_up)
    B_lo = lower(gam, B_up)
    Bv = dot(B_up, v_lo)
    B2 = dot(B_up, B_lo)
    ab0 = W * Bv
    b_lo = B_lo / W + W * Bv * v_lo
    b2 = B2 / W ** 2 + Bv ** 2
    return W, ab0, b_lo, b2


def prim_to_cons(rho, p, v_up, B_up, gam, Gamma):
    """Undensitised (D, S_j, tau) from primitives (standard Valencia form)."""
    W = lorentz(v_up, gam)
    eps = eos_eps(rho, p, Gamma)
    h = 1.0 + eps + p / rho
    v_lo = lower(gam, v_up)
    B_lo = lower(gam, B_up)
    Bv = dot(B_up, v_lo)
    B2 = dot(B_up, B_lo)
    Z = rho * h * W * W
    D = rho * W
    S = (Z + B2) * v_lo - Bv * B_lo
    tau = Z - p + B2 - 0.5 * (B2 / W ** 2 + Bv ** 2) - D
    return D, S, tau


# Bisection budget: halving [0, hi] down to adjacent doubles takes at most
# about 1100 steps (the exponent range of a double plus its 53-bit mantissa).
C2P_BISECTIONS = 2000


def _c2p_residual(Z, D, tau, S2, B2, BS, Gamma):
    """f(Z) = Z + B^2 - p - B^2/(2W^2) - (B.S)^2/(2Z^2) - tau - D, with
    v^2(Z) = (Z^2 S^2 + (2Z + B^2)(B.S)^2) / (Z^2 (Z + B^2)^2) and the ideal-gas
    pressure p = (Gamma-1)/Gamma (Z/W^2 - D/W).  Points where v^2 >= 1 are
    reported as f = -inf (Z below the physical range)."""
    with np.errstate(divide='ignore', invalid='ignore'):
        v2 = (Z * Z * S2 + (2.0 * Z + B2) * BS * BS) / (Z * Z * (Z + B2) ** 2)
        ok = (v2 < 1.0) & (Z > 0.0)
        iw2 = np.where(ok, 1.0 - v2, 1.0)
        p = (Gamma - 1.0) / Gamma * (Z * iw2 - D * np.sqrt(iw2))
        f = Z + B2 - p - 0.5 * B2 * iw2 - 0.5 * BS * BS / (Z * Z) - tau - D
    return np.where(ok, f, -np.inf)


def con2prim(D, S_lo, tau, B_up, gam, gamu, Gamma, rho_fl, p_fl):
    """Primitive state (rho, p, v^i) with prim_to_cons(...) == (D, S_j, tau).

    Bisection on f(Z) over (0, Z_hi], Z_hi >= Gamma (tau + D) >= the root,
    halving until the bracket ends are adjacent doubles; then
      v_j = (S_j + (B.S) B_j / Z) / (Z + B^2),  rho = D/W,
      p = (Gamma-1)/Gamma (Z/W^2 - rho).
    Failure policy (both implementations): D <= 0, tau + D <= 0, no sign change,
    a bracket left unresolved by the iteration budget, v^2 >= 1, rho < rho_fl
    or p < p_fl -> atmosphere (rho_fl, p_fl, v = 0) and the point is flagged.
    Returns rho, p, v_up, fail (bool array)."""
    D = np.asarray(D, float)
    shape = D.shape
    S2 = dot(S_lo, np.einsum('ij...,j...->i...', gamu, S_lo))
    B_lo = lower(gam, B_up)
    B2 = dot(B_up, B_lo)
    BS = dot(B_up, S_lo)
    bad = ~((D > 0.0) & (tau + D > 0.0))
    Dc = np.where(bad, 1.0, D)
    tc = np.where(bad, 1.0, tau)
    lo = np.zeros(shape)
    hi = Gamma * (tc + Dc) + B2 + 1e-300
    fhi = _c2p_residual(hi, Dc, tc, S2, B2, BS, Gamma)
    for _ in range(8):  # widen the upper end if needed (not expected)
        need = ~(fhi >= 0.0)
        if not need.any():
            break
        hi = np.where(need, 2.0 * hi, hi)
        fhi = _c2p_residual(hi, Dc, tc, S2, B2, BS, Gamma)
    bad |= ~(fhi >= 0.0)
    for _ in range(C2P_BISECTIONS):
        mid = 0.5 * (lo + hi)
        active = (mid > lo) & (mid < hi)
        if not active.any():
            break
        fm = _c2p_residual(mid, Dc, tc, S2, B2, BS, Gamma)
        up = fm < 0.0
        lo = np.where(active & up, mid, lo)
        hi = np.where(active & ~up, mid, hi)
    # a bracket not yet reduced to adjacent doubles is not a recovered state
    mid = 0.5 * (lo + hi)
    bad |= (mid > lo) & (mid < hi)
    Z = hi
    v_lo = (S_lo + BS * B_lo / Z) / (Z + B2)
    v_up = np.einsum('ij...,j...->i...', gamu, v_lo)
    v2 = dot(v_up, v_lo)
    with np.errstate(invalid='ignore', divide='ignore'):
        W = 1.0 / np.sqrt(1.0 - v2)
        rho = Dc / W
        p = (Gamma - 1.0) / Gamma * (Z / W ** 2 - rho)
    fail = bad | ~(v2 < 1.0) | ~(rho >= rho_fl) | ~(p >= p_fl)
    rho = np.where(fail, rho_fl, rho)
    p = np.where(fail, p_fl, p)
    v_up = np.where(fail[None], 0.0, v_up)
    return rho, p, v_up, fail


def con2prim_damped(D, S_lo, tau, B_up, gam, gamu, Gamma, rho_fl, p_fl, rho0, p0, v0,
                    maxit=40, lam0=0.5, tol=1e-15):
    """The paper's damped iteration for the primitive state (Methods, "The
    Primitive Variable Recovery"), started from a previous primitive state
    (rho0, p0, v0^i).  Readings: the predicted conserved variables are those of
    the current primitives (prim_to_cons, so the fixed point is the exact
    inverse); the velocity update raises Delta S_j with gamma^{ij}; the residual
    is |Delta S|_gamma + |Delta tau| with |Delta S|_gamma^2 =
    gamma^{ij} Delta S_i Delta S_j; one damping factor lambda = 0.5 for v and
    eps, halved (and the step retried from the previous iterate) whenever a
    step does not lower the residual or leaves v^2 < 1, eps > 0; stop once the
    residual is below tol (|S|_gamma + |tau| + D), or after maxit tries; if not
    converged, one Newton step on eps at fixed rho and v (d tau/d eps =
    rho (Gamma W^2 - (Gamma - 1))).  An unusable guess (rho0 or p0 <= 0,
    v0^2 >= 1) starts from v = 0, rho = D, eps = max((tau - B^2/2)/D,
    eps_floor).  Failure policy as con2prim.  Returns rho, p, v_up, fail,
    iterations taken."""
    D = np.asarray(D, float)
    bad = ~((D > 0.0) & (tau + D > 0.0))
    Dc = np.where(bad, 1.0, D)
    tc = np.where(bad, 1.0, tau)
    B_lo = lower(gam, B_up)
    B2 = dot(B_up, B_lo)
    gm1 = Gamma - 1.0
    with np.errstate(invalid='ignore', divide='ignore'):
        v2g = dot(lower(gam, v0), v0)
        ok = (rho0 > 0.0) & (p0 > 0.0) & (v2g < 1.0)
        v = np.where(ok[None], v0, 0.0)
        eps_fl = p_fl / (gm1 * rho_fl)
        eps = np.where(ok, p0 / (gm1 * np.where(ok, rho0, 1.0)), np.maximum((tc - 0.5 * B2) / Dc, eps_fl))
    S_up = np.einsum('ij...,j...->i...', gamu, S_lo)
    scale = np.sqrt(dot(S_lo, S_up)) + np.abs(tc) + Dc

    def lorentz_of(vv):
        return 1.0 / np.sqrt(1.0 - dot(lower(gam, vv), vv))

    def resid(rr, ee, vv):
        _, Sp, tp = prim_to_cons(rr, gm1 * rr * ee, vv, B_up, gam, Gamma)
        dS = S_lo - Sp
        dT = tc - tp
        return np.sqrt(dot(dS, np.einsum('ij...,j...->i...', gamu, dS))) + np.abs(dT), dS, dT

    rho = Dc / lorentz_of(v)
    r, dS, dT = resid(rho, eps, v)
    conv = r <= tol * scale
    lam = np.full(D.shape, lam0)
    its = np.zeros(D.shape, dtype=int)
    for _ in range(maxit):
        act = ~conv
        if not act.any():
            break
        its += act
        W = lorentz_of(v)
        h = 1.0 + Gamma * eps
        vt = v + lam * np.einsum('ij...,j...->i...', gamu, dS) / (rho * h * W * W)
        et = eps + lam * dT / (rho * W * W)
        with np.errstate(invalid='ignore', divide='ignore'):
            v2t = dot(lower(gam, vt), vt)
            phys = (v2t < 1.0) & (et > 0.0)
            vs = np.where(phys[None], vt, v)  # keep the arithmetic finite where rejected
            es = np.where(phys, et, eps)
            rt = Dc / lorentz_of(vs)
            r_t, dS_t, dT_t = resid(rt, es, vs)
        acc = act & phys & (r_t < r)
        lam = np.where(act & ~acc, 0.5 * lam, lam)
        v = np.where(acc[None], vt, v)
        eps = np.where(acc, et, eps)
        rho = np.where(acc, rt, rho)
        r = np.where(acc, r_t, r)
        dS = np.where(acc[None], dS_t, dS)
        dT = np.where(acc, dT_t, dT)
        conv = conv | (acc & (r_t <= tol * scale))
    W = lorentz_of(v)
    eps = np.where(conv, eps, eps + dT / (rho * (Gamma * W * W - gm1)))
    p = gm1 * rho * eps
    v2 = dot(lower(gam, v), v)
    fail = bad | ~(v2 < 1.0) | ~(rho >= rho_fl) | ~(p >= p_fl)
    rho = np.where(fail, rho_fl, rho)
    p = np.where(fail, p_fl, p)
    v = np.where(fail[None], 0.0, v)
    return rho, p, v, fail, its


def fluxes(D, S_lo, tau, B_up, rho, p, v_up, alpha, beta, gam, sqrtg):
    """Densitised fluxes alpha sqrt(gamma) F^i of (D, S_j, tau, B^k).

    Returns an array of shape (8, 3, ...): [variable, direction i, grid]."""
    W, ab0, b_lo, b2 = magnetic(v_up, B_up, gam)
    vt = v_up - beta / alpha
    ps = p + 0.5 * b2
    F = np.zeros((8, 3) + np.shape(D))
    for i in range(3):
        F[0, i] = D * vt[i]
        for j in range(3):
            F[1 + j, i] = S_lo[j] * vt[i] - b_lo[j] * B_up[i] / W + (ps if i == j else 0.0)
        F[4, i] = tau * vt[i] + ps * v_up[i] - ab0 * B_up[i] / W
        for k in range(3):
            F[5 + k, i] = vt[i] * B_up[k] - vt[k] * B_up[i]
    return F * (alpha * sqrtg)


def matter_3p1(rho, p, v_up, B_up, D, tau, gam, Gamma):
    """ADM matter projections of T^{mu nu} = rho h* u u + p* g - b b:
    energy density E = tau + D and spatial stress
    S_ij = (rho h + b^2) W^2 v_i v_j + p* gamma_ij - b_i b_j (lower indices).
    (The momentum density S_j is the conserved momentum itself.)"""
    W, ab0, b_lo, b2 = magnetic(v_up, B_up, gam)
    eps = eos_eps(rho, p, Gamma)
    h = 1.0 + eps + p / rho
    v_lo = lower(gam, v_up)
    ps = p + 0.5 * b2
    E = tau + D
    Sij = (rho * h + b2) * W * W * np.einsum('i...,j...->ij...', v_lo, v_lo) \
        + ps * gam - np.einsum('i...,j...->ij...', b_lo, b_lo)
    return E, Sij


def sources_3p1(E, S_lo, Sij, alpha, dalpha, dbeta, dgam, Kij, gamu):
    """Source vector sqrt(gamma)-free part for S_j and tau (3+1 form):
      Sbar_{S_j} = -E d_j alpha + S_k d_j beta^k + (alpha/2) S^{kl} d_j gamma_kl
      Sbar_tau   = alpha S^{kl} K_kl - S^k d_k alpha
    dalpha[j] = d_j alpha, dbeta[j, k] = d_j beta^k, dgam[j, k, l] = d_j gamma_kl."""
    Sup = np.einsum('ik...,jl...,kl...->ij...', gamu, gamu, Sij)
    S_up = np.einsum('ij...,j...->i...', gamu, S_lo)
    srcS = -E * dalpha + np.einsum('k...,jk...->j...', S_lo, dbeta) \
        + 0.5 * alpha * np.einsum('kl...,jkl...->j...', Sup, dgam)
    srcT = alpha * np.einsum('kl...,kl...->...', Sup, Kij) - dot(S_up, dalpha)
    return srcS, srcT
