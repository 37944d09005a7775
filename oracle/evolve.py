"""Full right-hand side, boundary treatment, RK4 step, filter and time step,
oracle side.

Paper: Methods, "Time Integration: The Fourth-Order Runge-Kutta" (classic RK4
tableau), "The Stability and Complexity" (CFL condition), "Dealiasing and
Spectral Filtering", Results "GRMHD Conservative Form" (conservation law) and
the coupled-evolution description.

Readings of the paper taken here (where it is silent or inconsistent):
  * coupling: all 32 fields (24 spacetime + 8 densitised GRMHD) are advanced
    together by one unsplit classic RK4 step (the paper's half-step/Euler
    operator split would not give the fourth-order accuracy it claims).
  * state is nodal (equivalent to the paper's coefficient state U_hat).
  * boundary: the right-hand side of every field is set to zero at the outer
    radial nodes (r = r_out) and at both theta end nodes; the inner radial
    boundary lies inside the horizon and is left free; phi is periodic.
  * filter: once per step, on the new state, all 32 fields, along r, theta,
    phi; optional 2/3 dealiasing before it.
  * fixed background (cowling = True, the solver's fixed-background version
    in "Numerical Implementation of Coupled GRMHD-Einstein Evolution"): the
    24 spacetime fields keep their initial values exactly; their right-hand
    sides are zero and neither the filter nor the dealiasing touches them.
  * 1+log source: K0 = K - beta^k d_k alpha/(2 alpha) at t = 0 (stored,
    static), so that the Kerr-Schild slice is stationary with the advection
    term of the printed 1+log equation kept.
  * time step: dt = cfl * min over nodes of min(dr, r dtheta, r sin(theta)
    dphi) with neighbour spacings and characteristic speed bound 1 (light
    speed), fixed for the run.
  * GLM constraint damping (optional, Methods "GLM Constraint Damping
    Source"): a 33rd evolved field psi (undensitised) with
    d_t psi = -c_h^2 D_i B^i - psi / tau, D_i B^i = d_i(sqrt(gamma) B^i) /
    sqrt(gamma), and the induction source sqrt(gamma) S^i with
    S^i = -gamma^{ij} d_j psi.  The paper prints S_{B^i} = d_i psi: the index
    is raised with the spatial metric, and the sign is Dedner's (with the
    printed sign the pair d_t psi, d_t B would give d_tt psi = -c_h^2
    Laplacian psi, which is ill-posed); no lapse factors, as printed.
    Frozen at the same boundary nodes and filtered like the other fields.
  * operator-split coupled step (optional, Methods "Coupled Main Loop" and the
    coupled-evolution description: a GRMHD half-step on the current spacetime,
    primitive recovery and T^{mu nu}, a first-order Euler BSSN step, then the
    gauge update): taken in its symmetric form, classic RK4 over dt/2 of the
    GRMHD fields (and psi) with the spacetime frozen, one forward-Euler step
    dt of the 24 spacetime fields (BSSN and gauge together, their right-hand
    sides evaluated after the first half-step) with the matter frozen, classic
    RK4 over dt/2 of the GRMHD fields on the new spacetime, then the filter.
    The literal loop has one fluid half-step per step, which would advance the
    fluid by dt/2 while the spacetime advances by dt; the symmetric form is the
    one in which both advance by dt.
  * primitive recovery: the exact inverse by default; optionally the paper's
    damped iteration (c2p = "damped", grmhd.con2prim_damped) started from the
    primitives of the previous recovery (the first recovery of a Problem is
    exact), so a Problem carries that chain from call to call.
"""

import numpy as np

from . import spectral
from .grmhd import inv3, det3, con2prim, con2prim_damped, fluxes, matter_3p1, sources_3p1
from .bssn import bssn_rhs, SYM

# State layout: 32 fields, each a (n_phi, n_theta, n_r) array.
FIELDS = (['phi']
          + ['gt_' + a + b for a, b in (('r', 'r'), ('r', 'th'), ('r', 'ph'), ('th', 'th'), ('th', 'ph'), ('ph', 'ph'))]
          + ['At_' + a + b for a, b in (('r', 'r'), ('r', 'th'), ('r', 'ph'), ('th', 'th'), ('th', 'ph'), ('ph', 'ph'))]
          + ['K', 'Gt_r', 'Gt_th', 'Gt_ph', 'alpha', 'beta_r', 'beta_th', 'beta_ph', 'Bd_r', 'Bd_th', 'Bd_ph',
             'sD', 'sS_r', 'sS_th', 'sS_ph', 'stau', 'sB_r', 'sB_th', 'sB_ph'])
NF = len(FIELDS)
assert NF == 32


def _sym(a6):
    """(6, ...) -> (3, 3, ...) symmetric."""
    out = np.empty((3, 3) + a6.shape[1:])
    for c, (i, j) in enumerate(SYM):
        out[i, j] = a6[c]
        out[j, i] = a6[c]
    return out


def _unsym(t):
    return np.array([t[i, j] for i, j in SYM])


def unpack(U):
    f = dict(phi=U[0], gt=_sym(U[1:7]), At=_sym(U[7:13]), K=U[13], Gt=U[14:17], alpha=U[17],
             beta=U[18:21], Bd=U[21:24])
    m = dict(sD=U[24], sS=U[25:28], stau=U[28], sB=U[29:32])
    return f, m


def pack(f, m):
    U = np.empty((NF,) + np.shape(f['phi']))
    U[0] = f['phi']
    U[1:7] = _unsym(f['gt'])
    U[7:13] = _unsym(f['At'])
    U[13] = f['K']
    U[14:17] = f['Gt']
    U[17] = f['alpha']
    U[18:21] = f['beta']
    U[21:24] = f['Bd']
    U[24] = m['sD']
    U[25:28] = m['sS']
    U[28] = m['stau']
    U[29:32] = m['sB']
    return U


class Problem:
    """Grid + physical parameters; the method-of-lines RHS and RK4 step."""

    def __init__(self, grid, M=1.0, a=0.5, Gamma=4.0 / 3.0, eta=2.0, cowling=False,
                 gauge_k0=True, rho_floor=1e-20, p_floor=1e-24, filt_alpha=36.0,
                 filt_order=16, filter_on=True, dealias=False, cfl=0.25, glm=False, glm_ch=1.0,
                 glm_tau=2.0, split=False, c2p="exact"):
        if c2p not in ("exact", "damped"):
            raise ValueError("c2p must be 'exact' or 'damped'")
        self.c2p = c2p
        self.guess = None  # previous primitives (damped recovery)
        if split and cowling:
            raise ValueError("the split step needs the coupled system")
        self.split = split
        self.g = grid
        self.glm, self.glm_ch, self.glm_tau = glm, glm_ch, glm_tau
        self.M, self.a, self.Gamma, self.eta = M, a, Gamma, eta
        self.cowling, self.gauge_k0 = cowling, gauge_k0
        self.rho_fl = rho_floor * grid.R ** -1.5
        self.p_fl = p_floor * grid.R ** -2.5
        self.filt_alpha, self.filt_order, self.filter_on = filt_alpha, filt_order, filter_on
        self.dealias = dealias
        self.cfl = cfl
        self.last_fail = None

    # ---- time step ------------------------------------------------------------
    def dt(self):
        g = self.g
        dr = np.abs(np.diff(g.r))
        dr_node = np.minimum(np.r_[dr, np.inf], np.r_[np.inf, dr])
        dth = np.abs(np.diff(g.th))
        dth_node = np.minimum(np.r_[dth, np.inf], np.r_[np.inf, dth])
        dph = 2.0 * np.pi / g.nph
        h = np.minimum(np.minimum(dr_node[None, None, :], g.r[None, None, :] * dth_node[None, :, None]),
                       g.r[None, None, :] * np.sin(g.th)[None, :, None] * dph)
        return self.cfl * float(np.min(h))

    # ---- pointwise pieces -----------------------------------------------------
    def metric(self, f):
        gam = np.exp(4.0 * f['phi']) * f['gt']
        gamu = inv3(gam)
        sqrtg = np.exp(6.0 * f['phi']) * np.sqrt(det3(f['gt']))
        return gam, gamu, sqrtg

    def primitives(self, U):
        f, m = unpack(U)
        gam, gamu, sqrtg = self.metric(f)
        D, S, tau, B = m['sD'] / sqrtg, m['sS'] / sqrtg, m['stau'] / sqrtg, m['sB'] / sqrtg
        if self.c2p == "damped" and self.guess is not None:
            rho, p, v, fail, _ = con2prim_damped(D, S, tau, B, gam, gamu, self.Gamma, self.rho_fl, self.p_fl,
                                                 *self.guess)
        else:
            rho, p, v, fail = con2prim(D, S, tau, B, gam, gamu, self.Gamma, self.rho_fl, self.p_fl)
        if self.c2p == "damped":
            self.guess = (rho, p, v)
        return dict(rho=rho, p=p, v=v, fail=fail, D=D, S=S, tau=tau, B=B,
                    gam=gam, gamu=gamu, sqrtg=sqrtg)

    # ---- right-hand side ------------------------------------------------------
    def rhs(self, U, K0):
        g = self.g
        f, m = unpack(U)
        P = self.primitives(U)
        self.last_fail = P['fail']
        gam, sqrtg = P['gam'], P['sqrtg']
        F = fluxes(P['D'], P['S'], P['tau'], P['B'], P['rho'], P['p'], P['v'],
                   f['alpha'], f['beta'], gam, sqrtg)
        # first derivatives (derivative index first)
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
        # matter
        E, Sij = matter_3p1(P['rho'], P['p'], P['v'], P['B'], P['D'], P['tau'], gam, self.Gamma)
        rb = bssn_rhs(f, d, dd, E, P['S'], Sij, K0, self.eta, self.gauge_k0)
        # GRMHD: -d_i(alpha sqrt(gamma) F^i) + sqrt(gamma) Sbar
        div = np.array([sum(g.d1(F[v, i], i) for i in range(3)) for v in range(8)])
        e4 = np.exp(4.0 * f['phi'])
        dgam = e4 * (d['gt'] + 4.0 * np.einsum('ij...,k...->kij...', f['gt'], d['phi']))
        Kij = e4 * (f['At'] + f['gt'] * f['K'] / 3.0)
        srcS, srcT = sources_3p1(E, P['S'], Sij, f['alpha'], d['alpha'], d['beta'], dgam, Kij, P['gamu'])
        rm = dict(sD=-div[0], sS=-div[1:4] + sqrtg * srcS, stau=-div[4] + sqrtg * srcT, sB=-div[5:8])
        if self.cowling:
            rb = {k: np.zeros_like(v) for k, v in rb.items()}
        if self.glm:
            psi = U[NF]
            dpsi = np.array([g.d1(psi, k) for k in range(3)])
            divB = sum(g.d1(U[29 + i], i) for i in range(3)) / sqrtg
            rm['sB'] = rm['sB'] - sqrtg * np.einsum('ij...,j...->i...', P['gamu'], dpsi)
            R = np.concatenate([pack(rb, rm), (-self.glm_ch ** 2 * divB - psi / self.glm_tau)[None]])
        else:
            R = pack(rb, rm)
        # freeze: r_out nodes and theta end nodes
        R[:, :, :, 0] = 0.0
        R[:, :, 0, :] = 0.0
        R[:, :, -1, :] = 0.0
        return R

    # ---- RK4 + filter -----------------------------------------------------------
    def apply_filter(self, U):
        # with a fixed background (Cowling) only the GRMHD fields (and psi)
        # are evolved, so only they are dealiased and filtered
        lo = 24 if self.cowling else 0
        out = U[lo:]
        if self.dealias:
            out = self.g.dealias(out)
        if self.filter_on:
            out = self.g.filter(out, self.filt_alpha, self.filt_order)
        return np.concatenate([U[:lo], out]) if lo else out

    def fluid_rk4(self, U, K0, h):
        """Classic RK4 over h of the GRMHD fields (and psi) with the spacetime
        fields held at their values in U (split step)."""
        def L(V):
            R = self.rhs(V, K0)
            R[:24] = 0.0
            return R
        k1 = L(U)
        k2 = L(U + 0.5 * h * k1)
        k3 = L(U + 0.5 * h * k2)
        k4 = L(U + h * k3)
        return U + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)

    def step_split(self, U, K0, dt):
        """Operator-split coupled step (symmetric reading of the coupled main
        loop): fluid dt/2, Euler BSSN + gauge dt with the matter frozen, fluid
        dt/2, filter."""
        V = self.fluid_rk4(U, K0, 0.5 * dt)
        R = self.rhs(V, K0)
        W = V.copy()
        W[:24] = V[:24] + dt * R[:24]
        return self.apply_filter(self.fluid_rk4(W, K0, 0.5 * dt))

    def step(self, U, K0, dt):
        if self.split:
            return self.step_split(U, K0, dt)
        k1 = self.rhs(U, K0)
        k2 = self.rhs(U + 0.5 * dt * k1, K0)
        k3 = self.rhs(U + 0.5 * dt * k2, K0)
        k4 = self.rhs(U + dt * k3, K0)
        Un = U + (dt / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        return self.apply_filter(Un)

    def evolve(self, U, K0, dt, nsteps):
        for _ in range(nsteps):
            U = self.step(U, K0, dt)
        return U


def initial_state(grid, problem, r_c=8.0, rho_c=1e-8, beta_min=100.0, pert_amp=1e-6, seed=1,
                  id_kind="michel", tor_r_in=6.0, tor_r_max=12.0, tor_rho_max=1e-8, tor_atm=1e-2,
                  tor_loop_cut=0.2):
    """Kerr-Schild BSSN data + magnetised Michel flow (id_kind "michel") or a
    magnetised Fishbone-Moncrief torus ("torus"); returns (U, K0, matter)."""
    from .initial_data import kerr_schild_bssn, michel_monopole, fm_torus
    f = kerr_schild_bssn(grid, problem.M, problem.a)
    if id_kind == "torus":
        mat = fm_torus(grid, f, problem.M, problem.a, problem.Gamma, tor_r_in, tor_r_max, tor_rho_max,
                       beta_min, pert_amp, seed, atm=tor_atm, a_cut=tor_loop_cut)
    else:
        mat = michel_monopole(grid, f, problem.M, problem.a, problem.Gamma, r_c, rho_c, beta_min, pert_amp,
                              seed)
    U = pack(f, dict(sD=mat['sD'], sS=mat['sS'], stau=mat['stau'], sB=mat['sB']))
    if problem.glm:
        U = np.concatenate([U, np.zeros((1,) + U.shape[1:])])  # psi = 0
    return U, gauge_source_k0(grid, f), mat


def gauge_source_k0(grid, f):
    """K0 = K - beta^k d_k alpha / (2 alpha) at t = 0: the static source of the
    1+log condition d_t alpha = beta^k d_k alpha - 2 alpha (K - K0) for which
    the initial slice is stationary (reading of the 1+log slicing equation)."""
    adv = sum(f['beta'][k] * grid.d1(f['alpha'], k) for k in range(3))
    return f['K'] - adv / (2.0 * f['alpha'])
