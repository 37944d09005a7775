"""Synthetic workload definitions shared by tests, bench and smoke.

Pure data and seeded input generators: no arithmetic of the method lives here.
The grids, physics parameters and step counts are those of the five
workloads the build is measured on (Kerr-Schild a = 0.5 Michel accretion with
a monopole field at min plasma beta 100 on log-mapped Chebyshev(r) x
Chebyshev(theta) x Fourier(phi) grids)."""

import math

import numpy as np

COMMON_GRID = dict(r_in=1.8, r_out=20.0, th_min=0.05, th_max=math.pi - 0.05,
                   filt_alpha=36.0, filt_order=16, filter_on=True)
COMMON_PHYS = dict(M=1.0, a=0.5, gamma_ad=4.0 / 3.0, cfl=0.25, eta=2.0, cowling=False, gauge_k0=True,
                   r_c=8.0, rho_c=1e-8, beta_min=100.0, pert_amp=1e-6, rho_floor=1e-20, p_floor=1e-24)

# torus workloads: spin 0.9375, inner radius scaled with the horizon
# (r_in(a) = 1.8 r_h(a)/r_h(0.5) = 1.300), outer radius 60; Fishbone-Moncrief
# torus with inner edge 6, pressure maximum 12, Gamma = 13/9, rho_max = 1e-8;
# one poloidal loop at min plasma beta 100 over the loop; +-4 % pressure
# perturbation
def _r_h(a):
    return 1.0 + math.sqrt(1.0 - a * a)


TORUS_SPIN = 0.9375
TORUS_GRID = dict(COMMON_GRID, r_in=1.8 * _r_h(TORUS_SPIN) / _r_h(0.5), r_out=60.0)
TORUS_PHYS = dict(COMMON_PHYS, a=TORUS_SPIN, gamma_ad=13.0 / 9.0, beta_min=100.0, pert_amp=0.04,
                  id_kind="torus", tor_r_in=6.0, tor_r_max=12.0, tor_rho_max=1e-8, tor_atm=1e-2,
                  tor_loop_cut=0.2)

WORKLOADS = {
    # tiny coupled evolution: 16^3, 10 RK4 steps
    "ks_michel_16x16x16": dict(grid=dict(nr=16, nth=16, nph=16, **COMMON_GRID),
                               phys=dict(seed=1, **COMMON_PHYS), steps=10),
    # plain FP64 GPU baseline: 64 x 64 x 128, 100 RK4 steps
    "ks_michel_64x64x128": dict(grid=dict(nr=64, nth=64, nph=128, **COMMON_GRID),
                                phys=dict(seed=2, **COMMON_PHYS), steps=100),
    # magnetised Fishbone-Moncrief torus at high resolution, a = 0.9375:
    # 128 x 96 x 192, r in [r_in(a), 60], 200 RK4 steps
    "ks_torus_128x96x192": dict(grid=dict(nr=128, nth=96, nph=192, **TORUS_GRID),
                                phys=dict(seed=4, **TORUS_PHYS), steps=200),
    # the same physics on a small grid (parity against the oracle)
    "ks_torus_24x20x16": dict(grid=dict(nr=24, nth=20, nph=16, **TORUS_GRID),
                              phys=dict(seed=3, **TORUS_PHYS), steps=10),
}


def oracle_kwargs(w):
    """Split a workload into (grid args, Problem kwargs, initial_state kwargs) for the oracle."""
    g = w["grid"]
    p = w["phys"]
    grid_args = (g["nr"], g["nth"], g["nph"], g["r_in"], g["r_out"], g["th_min"], g["th_max"])
    prob = dict(M=p["M"], a=p["a"], Gamma=p["gamma_ad"], eta=p["eta"], cowling=p["cowling"],
                gauge_k0=p["gauge_k0"], rho_floor=p["rho_floor"], p_floor=p["p_floor"],
                filt_alpha=g["filt_alpha"], filt_order=g["filt_order"], filter_on=g["filter_on"],
                dealias=g.get("dealias", False),
                cfl=p["cfl"])
    init = dict(r_c=p["r_c"], rho_c=p["rho_c"], beta_min=p["beta_min"], pert_amp=p["pert_amp"],
                seed=p["seed"])
    for k in ("id_kind", "tor_r_in", "tor_r_max", "tor_rho_max", "tor_atm", "tor_loop_cut"):
        if k in p:
            init[k] = p[k]
    for k in ("glm", "glm_ch", "glm_tau", "split", "c2p"):
        if k in p:
            prob[k] = p[k]
    return grid_args, prob, init


def grid_nodes(g):
    """(r, theta, phi) node coordinates of a workload grid, each shaped
    (n_phi, n_theta, n_r) for broadcasting: Chebyshev-Gauss-Lobatto in
    ln r and theta (index 0 at the outer / upper end), uniform in phi."""
    nr, nth, nph = g["nr"], g["nth"], g["nph"]
    x = np.cos(np.pi * np.arange(nr) / (nr - 1))
    y = np.cos(np.pi * np.arange(nth) / (nth - 1))
    lc, lh = 0.5 * math.log(g["r_in"] * g["r_out"]), 0.5 * math.log(g["r_out"] / g["r_in"])
    tc, th = 0.5 * (g["th_min"] + g["th_max"]), 0.5 * (g["th_max"] - g["th_min"])
    r = np.exp(lc + lh * x)[None, None, :]
    t = (tc + th * y)[None, :, None]
    p = (2.0 * np.pi * np.arange(nph) / nph)[:, None, None]
    return r, t, p


def divergence_seed(g, U):
    """The divergence-carrying field perturbation of the GLM studies: the
    densitised radial field scaled by 1 + 0.05 exp(-ln(r/5)^2) sin(theta)
    sin(phi) (a monopole's is independent of r, so its divergence vanishes)."""
    r, t, p = grid_nodes(g)
    U = U.copy()
    U[29] = U[29] * (1.0 + 0.05 * np.exp(-np.log(r / 5.0) ** 2) * np.sin(t) * np.sin(p))
    return U


def random_fields(shape, nfields, seed):
    """Seeded standard-normal test fields (float64), for operator tests."""
    return np.random.default_rng(seed).standard_normal((nfields,) + tuple(shape))


def smooth_fields(grid_r, grid_th, grid_ph, nfields, seed):
    """Seeded smooth fields: random low-order products of 1/(r + c), cos/sin of
    theta and low Fourier modes in phi."""
    rng = np.random.default_rng(seed)
    R = grid_r[None, None, :]
    T = grid_th[None, :, None]
    Ph = grid_ph[:, None, None]
    out = []
    for _ in range(nfields):
        c = rng.uniform(0.5, 3.0)
        a, b = rng.uniform(0.5, 2.0, 2)
        m = rng.integers(0, 4)
        out.append((1.0 / (R + c)) * np.cos(a * T + b) * (1.0 + 0.3 * np.cos(m * Ph + rng.uniform(0, 6))))
    return np.array(out)


# ---- served job stream --------------------------------------------------------
SERVED_GRIDS = [(16, 16, 16), (32, 32, 64), (48, 48, 96), (64, 64, 128)]


def served_stream(n_jobs=256, rate=4.0, seed=2508, t_scale=1.0, cowling_frac=0.0):
    """Seeded job stream: Poisson arrivals at `rate` jobs/s; per job spin
    a ~ U[0, 0.95], plasma beta ~ logU[10, 1000], a grid drawn uniformly from
    SERVED_GRIDS, end time T ~ U[10, 100] M times t_scale, and its own
    perturbation seed.  A fraction cowling_frac of the jobs (drawn from a
    generator of their own, so the rest of the stream does not change) evolve
    on the fixed Kerr-Schild background."""
    rng = np.random.default_rng(seed)
    fixed = np.random.default_rng(seed + 1).random(n_jobs) < cowling_frac
    gaps = rng.exponential(1.0 / rate, n_jobs)
    arrivals = np.cumsum(gaps) - gaps[0]
    jobs = []
    for i in range(n_jobs):
        jobs.append(dict(arrival=float(arrivals[i]), a=float(rng.uniform(0.0, 0.95)),
                         beta=float(10 ** rng.uniform(1.0, 3.0)),
                         grid=SERVED_GRIDS[int(rng.integers(0, len(SERVED_GRIDS)))],
                         T=float(rng.uniform(10.0, 100.0) * t_scale), seed=int(rng.integers(1, 2 ** 62)),
                         cowling=bool(fixed[i])))
    return jobs
