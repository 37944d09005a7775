"""Initial data, oracle side: Kerr-Schild BSSN variables, Michel accretion,
monopole magnetic field and the seeded density perturbation.

Paper: Results, "The Kerr-Schild Metric and 3+1 Decomposition"; Methods,
"BSSN Evolution Equations" (variable definitions).  The paper prints no
constants for its matter data; the Michel flow (relativistic Bondi accretion:
conserved mass flux rho u^r r^2 and Bernoulli constant h^2 (1 - 2M/r + u^2),
sonic point u_c^2 = M/(2 r_c), c_s^2 = u_c^2/(1 - 3 u_c^2)) is the standard
closed-form solution; its parameters (r_c, rho(r_c)) and the field strength
(minimum of 2p/b^2 over the nodes) are inputs.

Readings of the paper taken here (where it is silent or inconsistent):
  * K_ij from stationarity of the background: K_ij = L_beta gamma_ij / (2 alpha)
    with spectral derivatives of the nodal gamma_ij and beta^i.
  * Gamma-tilde^i = gt^{jk} Gamma-tilde^i_jk from spectral derivatives of gt_ij;
    B-driver = 0.  The static 1+log source K0 is not part of these data: it
    is K - beta^k d_k alpha / (2 alpha) of the initial slice
    (evolve.gauge_source_k0).
  * Michel radial profile is used for every spin with u^theta = u^phi = 0 in
    Kerr-Schild coordinates and u^t from the normalisation (exactly stationary
    only at a = 0).  Supersonic branch inside r_c, subsonic outside.
  * monopole field: sqrt(gamma) B^r = B0 sin(theta) (nodal values of the
    densitised field), B^theta = B^phi = 0.
  * perturbation: rho -> rho (1 + A (2u - 1)) at node n = (l n_th + k) n_r + j
    with u = top 53 bits of SplitMix64(seed XOR n) times 2^-53; p and v^i kept.
"""

import numpy as np

from . import kerr_schild as ks
from .grmhd import inv3, det3, lower, dot, magnetic, prim_to_cons
from .bssn import conformal_christoffel

MASK64 = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 output for state x (Steele, Lea & Flood 2014): add the golden
    gamma, then the two xor-shift-multiply rounds and a final xor-shift.
    Integer arithmetic modulo 2^64 on Python ints."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def uniform01(seed, n_points):
    """u_n = (SplitMix64(seed ^ n) >> 11) * 2^-53 for n = 0 .. n_points-1."""
    out = np.empty(n_points)
    for n in range(n_points):
        out[n] = (splitmix64((seed ^ n) & MASK64) >> 11) * 2.0 ** -53
    return out


# ---- Kerr-Schild background in BSSN variables --------------------------------

def kerr_schild_bssn(grid, M, a):
    """phi, gt, At, K, Gt, alpha, beta, Bd (dict) on the nodes of `grid`."""
    alpha, beta, gam = ks.adm(grid.R, grid.TH, M, a)
    beta = np.ascontiguousarray(beta)
    gam = np.ascontiguousarray(gam)
    gamu = inv3(gam)
    dgam = np.array([[[grid.d1(gam[i, j], k) for j in range(3)] for i in range(3)] for k in range(3)])
    dbeta = np.array([[grid.d1(beta[i], k) for i in range(3)] for k in range(3)])  # [k, i] = d_k beta^i
    Lg = np.einsum('k...,kij...->ij...', beta, dgam) \
        + np.einsum('ik...,jk...->ij...', gam, dbeta) + np.einsum('jk...,ik...->ij...', gam, dbeta)
    Kij = Lg / (2.0 * alpha)
    phi = np.log(det3(gam)) / 12.0
    gt = np.exp(-4.0 * phi) * gam
    K = np.einsum('ij...,ij...->...', gamu, Kij)
    At = np.exp(-4.0 * phi) * (Kij - gam * K / 3.0)
    dgt = np.array([[[grid.d1(gt[i, j], k) for j in range(3)] for i in range(3)] for k in range(3)])
    gtu = inv3(gt)
    _, Gu = conformal_christoffel(gtu, dgt)
    Gt = np.einsum('jk...,ijk...->i...', gtu, Gu)
    return dict(phi=phi, gt=gt, At=At, K=K, Gt=Gt, alpha=alpha, beta=beta,
                Bd=np.zeros_like(beta))


# ---- Michel accretion ---------------------------------------------------------

class Michel:
    """Polytropic (p = K rho^Gamma) relativistic Bondi flow with sonic radius
    r_c and density rho_c there."""

    def __init__(self, M, Gamma, r_c, rho_c):
        self.M, self.G, self.r_c, self.rho_c = M, Gamma, r_c, rho_c
        self.n = 1.0 / (Gamma - 1.0)
        uc2 = M / (2.0 * r_c)
        cs2 = uc2 / (1.0 - 3.0 * uc2)
        # c_s^2 = Gamma T / h with h = 1 + (n+1) T, T = p/rho
        self.Tc = cs2 / (Gamma - (self.n + 1.0) * cs2)
        self.Kp = self.Tc / rho_c ** (Gamma - 1.0)
        self.uc = np.sqrt(uc2)
        self.C1 = rho_c * self.uc * r_c ** 2
        self.C2 = (1.0 + (self.n + 1.0) * self.Tc) ** 2 * (1.0 - 2.0 * M / r_c + uc2)

    def _F(self, lnT, r):
        T = np.exp(lnT)
        rho = (T / self.Kp) ** self.n
        u = self.C1 / (r * r * rho)
        h = 1.0 + (self.n + 1.0) * T
        return h * h * (1.0 - 2.0 * self.M / r + u * u) - self.C2

    def temperature(self, r):
        """T = p/rho at radius r on the transonic branch."""
        grid = np.linspace(np.log(self.Tc) - 30.0, np.log(self.Tc) + 12.0, 8001)
        F = self._F(grid, r)
        s = np.sign(F)
        idx = np.nonzero(s[:-1] * s[1:] < 0)[0]
        if r < self.r_c:
            cand = [i for i in idx if F[i] > 0]        # first + -> - change
            i0 = cand[0] if cand else None
        else:
            cand = [i for i in idx if F[i] < 0]        # last - -> + change
            i0 = cand[-1] if cand else None
        if i0 is None:
            # double root (r ~ r_c): minimum of F by golden-section search
            i = int(np.argmin(F))
            lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)]
            g = (np.sqrt(5.0) - 1.0) / 2.0
            for _ in range(200):
                m1, m2 = hi - g * (hi - lo), lo + g * (hi - lo)
                if self._F(m1, r) < self._F(m2, r):
                    hi = m2
                else:
                    lo = m1
            return float(np.exp(0.5 * (lo + hi)))
        lo, hi = grid[i0], grid[i0 + 1]
        flo = self._F(lo, r)
        while True:
            mid = 0.5 * (lo + hi)
            if not (lo < mid < hi):
                break
            fm = self._F(mid, r)
            if (fm > 0) == (flo > 0):
                lo, flo = mid, fm
            else:
                hi = mid
        return float(np.exp(0.5 * (lo + hi)))

    def profile(self, r):
        """rho, p, u^r (negative: inflow) at the radii r (1D array)."""
        T = np.array([self.temperature(float(x)) for x in np.ravel(r)]).reshape(np.shape(r))
        rho = (T / self.Kp) ** self.n
        p = rho * T
        ur = -self.C1 / (np.asarray(r) ** 2 * rho)
        return rho, p, ur


def four_velocity_t(r, th, M, a, ur):
    """u^t from g_{mu nu} u^mu u^nu = -1 with u^theta = u^phi = 0 (the root
    continuous across g_tt = 0)."""
    g = ks.metric4(r, th, M, a)
    A = g[0, 0]
    B = g[0, 1] * ur
    C = g[1, 1] * ur * ur + 1.0
    return C / (-B + np.sqrt(B * B - A * C))


def michel_monopole(grid, fields, M, a, Gamma, r_c, rho_c, beta_min, pert_amp, seed):
    """Primitive and densitised conserved matter variables on the nodes.

    Returns dict with rho, p, v (upper), B (upper, undensitised) and the
    densitised conserved arrays sD, sS (lower), stau, sB (upper)."""
    mic = Michel(M, Gamma, r_c, rho_c)
    rho1, p1, ur1 = mic.profile(grid.r)
    shape = grid.shape
    rho = np.broadcast_to(rho1[None, None, :], shape).copy()
    p = np.broadcast_to(p1[None, None, :], shape).copy()
    ur = np.broadcast_to(ur1[None, None, :], shape)
    alpha, beta = fields['alpha'], fields['beta']
    gam = np.exp(4.0 * fields['phi']) * fields['gt']
    sqrtg = np.exp(6.0 * fields['phi']) * np.sqrt(det3(fields['gt']))
    ut = four_velocity_t(grid.R, grid.TH, M, a, ur)
    W = alpha * ut
    v = np.zeros((3,) + shape)
    v[0] = ur / W + beta[0] / alpha
    v[1] = beta[1] / alpha
    v[2] = beta[2] / alpha
    sB = np.zeros((3,) + shape)
    sB[0] = np.sin(grid.TH)
    B1 = sB / sqrtg
    _, _, _, b2 = magnetic(v, B1, gam)
    B0 = np.sqrt(2.0 * np.min(p / b2) / beta_min)
    sB *= B0
    B = sB / sqrtg
    if pert_amp != 0.0:
        u = uniform01(seed, grid.npts).reshape(shape)
        rho = rho * (1.0 + pert_amp * (2.0 * u - 1.0))
    D, S, tau = prim_to_cons(rho, p, v, B, gam, Gamma)
    return dict(rho=rho, p=p, v=v, B=B, sD=sqrtg * D, sS=sqrtg * S, stau=sqrtg * tau, sB=sB, B0=B0)


# ---- Fishbone-Moncrief torus ---------------------------------------------------
#
# Hydrostatic torus of constant ell = u^t u_phi around a Kerr hole (Fishbone &
# Moncrief 1976), isentropic p = K rho^Gamma.  The velocity is purely
# azimuthal, u = u^t (1, 0, 0, Omega); the components g_tt, g_tphi, g_phiphi
# are the same in Boyer-Lindquist and Kerr-Schild coordinates and u^r = 0, so
# u^t and u^phi carry over unchanged.
#
# Derivation used here (restated, not copied): with the ZAMO quantities
# omega = -g_tphi/g_phiphi, alpha_Z^2 = omega^2 g_phiphi - g_tt and the
# azimuthal speed V = sqrt(g_phiphi) (Omega - omega)/alpha_Z measured by the
# ZAMO, ell = u^t u_phi = sqrt(g_phiphi) V / (alpha_Z (1 - V^2)), a quadratic
# c V^2 + V - c = 0 in V with c = ell alpha_Z / sqrt(g_phiphi).  The Euler
# equation of circular flow, d ln h = -d ln(-u_t) + Omega dl / (1 - Omega l)
# with l = -u_phi/u_t, integrates at constant ell (l = ell/(1 + ell Omega)) to
#   ln h = ln(1 + ell Omega) - ln(-u_t) - ell Omega + const,
# the constant fixed by h = 1 at the inner edge (r_in, pi/2).  ell follows
# from r_max: at the pressure maximum the flow is on the prograde circular
# equatorial geodesic (Bardeen, Press & Teukolsky 1972), ell = u^t u_phi of
# that orbit.

class FMTorus:
    def __init__(self, M, a, r_in, r_max, Gamma, rho_max):
        self.M, self.a, self.r_in, self.r_max = M, a, r_in, r_max
        self.Gamma, self.rho_max = Gamma, rho_max
        self.ell = self.ell_circular(r_max)
        self.lnh_in = 0.0
        self.lnh_in = self.lnh(np.array(r_in), np.array(0.5 * np.pi))
        h_max = np.exp(self.lnh(np.array(r_max), np.array(0.5 * np.pi)))
        # rho_max = ((h - 1)(Gamma - 1)/(K Gamma))^(1/(Gamma - 1)) at the maximum
        self.K = (h_max - 1.0) * (Gamma - 1.0) / (Gamma * rho_max ** (Gamma - 1.0))

    def ell_circular(self, r):
        """u^t u_phi of the prograde circular equatorial geodesic at r."""
        M, a = self.M, self.a
        sq = np.sqrt(r ** 1.5 - 3.0 * M * np.sqrt(r) + 2.0 * a * np.sqrt(M))
        ut = (r ** 1.5 + a * np.sqrt(M)) / (r ** 0.75 * sq)
        uphi_lo = np.sqrt(M) * (r * r - 2.0 * a * np.sqrt(M * r) + a * a) / (r ** 0.75 * sq)
        return ut * uphi_lo

    def velocity(self, r, th):
        """u^t, u^phi (upper), Omega and u_t (lower) of the torus flow."""
        g = ks.metric4(r, th, self.M, self.a)
        gtt, gtp, gpp = g[0, 0], g[0, 3], g[3, 3]
        omega = -gtp / gpp
        alz = np.sqrt(omega * omega * gpp - gtt)
        c = self.ell * alz / np.sqrt(gpp)
        V = (np.sqrt(1.0 + 4.0 * c * c) - 1.0) / (2.0 * c)
        ut = 1.0 / (alz * np.sqrt(1.0 - V * V))
        Om = omega + alz * V / np.sqrt(gpp)
        u_t = ut * (gtt + gtp * Om)
        return ut, ut * Om, Om, u_t

    def lnh(self, r, th):
        _, _, Om, u_t = self.velocity(r, th)
        return np.log(1.0 + self.ell * Om) - np.log(-u_t) - self.ell * Om - self.lnh_in

    def density(self, r, th):
        """rho of the torus (0 outside it: ln h <= 0 or r < r_in)."""
        r, th = np.broadcast_arrays(np.asarray(r, dtype=float), np.asarray(th, dtype=float))
        out = np.zeros(r.shape)
        m = r >= self.r_in
        lh = np.full(r.shape, -1.0)
        lh[m] = self.lnh(r[m], th[m])
        inside = lh > 0.0
        hm1 = np.expm1(lh[inside])
        out[inside] = (hm1 * (self.Gamma - 1.0) / (self.K * self.Gamma)) ** (1.0 / (self.Gamma - 1.0))
        return out


def fm_torus(grid, fields, M, a, Gamma, r_in, r_max, rho_max, beta_min, pert_amp, seed, atm=1e-2, a_cut=0.2):
    """Magnetised Fishbone-Moncrief torus on the nodes (same return keys as
    michel_monopole).

    Readings (the paper leaves these open): atmosphere rho = atm rho_max (r/r_max)^-3/2
    at Eulerian rest on the same isentrope, rho = max(rho_torus, rho_atm);
    one poloidal loop A_phi = max(rho_torus/rho_max - a_cut, 0) with the
    densitised field sqrt(gamma) B^r = d_theta A_phi, sqrt(gamma) B^theta =
    -d_r A_phi from the spectral derivatives (discrete div B = 0 because the
    axis operators commute), scaled so that the minimum of 2p/b^2 over the
    nodes where A_phi > 0 equals beta_min; pressure perturbation
    p -> p (1 + A (2u - 1)) with the SplitMix64 stream of the density one."""
    tor = FMTorus(M, a, r_in, r_max, Gamma, rho_max)
    shape = grid.shape
    R, TH = grid.R, grid.TH
    rho_t = tor.density(R, TH)
    rho_a = atm * rho_max * (R / r_max) ** -1.5
    rho = np.maximum(rho_t, rho_a)
    p = tor.K * rho ** Gamma
    alpha, beta = fields['alpha'], fields['beta']
    gam = np.exp(4.0 * fields['phi']) * fields['gt']
    sqrtg = np.exp(6.0 * fields['phi']) * np.sqrt(det3(fields['gt']))
    v = np.zeros((3,) + shape)
    inside = rho_t > 0.0
    ut, uph, _, _ = tor.velocity(R[inside], TH[inside])
    W = alpha[inside] * ut
    v[0][inside] = beta[0][inside] / alpha[inside]
    v[1][inside] = beta[1][inside] / alpha[inside]
    v[2][inside] = uph / W + beta[2][inside] / alpha[inside]
    Aph = np.maximum(rho_t / rho_max - a_cut, 0.0)
    sB = np.zeros((3,) + shape)
    sB[0] = grid.d_th(Aph)
    sB[1] = -grid.d_r(Aph)
    _, _, _, b2 = magnetic(v, sB / sqrtg, gam)
    loop = Aph > 0.0
    B0 = np.sqrt(2.0 * np.min(p[loop] / b2[loop]) / beta_min)
    sB *= B0
    B = sB / sqrtg
    if pert_amp != 0.0:
        u = uniform01(seed, grid.npts).reshape(shape)
        p = p * (1.0 + pert_amp * (2.0 * u - 1.0))
    D, S, tau = prim_to_cons(rho, p, v, B, gam, Gamma)
    return dict(rho=rho, p=p, v=v, B=B, sD=sqrtg * D, sS=sqrtg * S, stau=sqrtg * tau, sB=sB, B0=B0,
                K=tor.K, ell=tor.ell)
