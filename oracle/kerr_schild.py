"""Kerr metric in (spherical) Kerr-Schild coordinates and its 3+1 split.

Paper: Results, "The Kerr-Schild Metric and 3+1 Decomposition" (the line
element with Sigma = r^2 + a^2 cos^2 theta, H = M r / Sigma, alpha =
(1+2H)^(-1/2)).  The line element is taken as authoritative.  The printed null
covector l_phi = +a sin^2 theta / Sigma, the flat part diag(-1,1,1,1) and the
appendix table entry beta^r = 2r^2/Sigma disagree with that line element; the
3+1 closed forms below are the ones that follow from it (checked against the
numerical split of `metric4` in the tests).
"""

import numpy as np


def sigma(r, th, a):
    return r * r + a * a * np.cos(th) ** 2


def H_of(r, th, M, a):
    return M * r / sigma(r, th, a)


def metric4(r, th, M, a):
    """g_{mu nu}(t, r, theta, phi) read off the Kerr-Schild line element.
    Returns an array of shape (4, 4) + broadcast shape of (r, th)."""
    r, th = np.broadcast_arrays(np.asarray(r), np.asarray(th))
    S = sigma(r, th, a)
    H = M * r / S
    s2 = np.sin(th) ** 2
    g = np.zeros((4, 4) + r.shape, dtype=np.result_type(r, th, float))
    g[0, 0] = -(1.0 - 2.0 * H)
    g[0, 1] = g[1, 0] = 2.0 * H                      # (4Mr/Sigma) dt dr
    g[1, 1] = 1.0 + 2.0 * H
    g[2, 2] = S
    g[3, 3] = s2 * (S + a * a * s2 * (1.0 + 2.0 * H))
    g[0, 3] = g[3, 0] = -2.0 * a * H * s2            # -(4aMr sin^2/Sigma) dt dphi
    g[1, 3] = g[3, 1] = -a * s2 * (1.0 + 2.0 * H)    # -2a sin^2 (1+2H) dr dphi
    return g


def adm(r, th, M, a):
    """Closed-form lapse, shift (upper index) and spatial metric (lower).

    alpha = (1+2H)^(-1/2); beta^r = 2H/(1+2H), beta^theta = beta^phi = 0;
    gamma_ij = the spatial block of the line element."""
    r, th = np.broadcast_arrays(np.asarray(r), np.asarray(th))
    S = sigma(r, th, a)
    H = M * r / S
    s2 = np.sin(th) ** 2
    dt = np.result_type(r, th, float)
    alpha = 1.0 / np.sqrt(1.0 + 2.0 * H)
    beta = np.zeros((3,) + r.shape, dtype=dt)
    beta[0] = 2.0 * H / (1.0 + 2.0 * H)
    gam = np.zeros((3, 3) + r.shape, dtype=dt)
    gam[0, 0] = 1.0 + 2.0 * H
    gam[0, 2] = gam[2, 0] = -a * s2 * (1.0 + 2.0 * H)
    gam[1, 1] = S
    gam[2, 2] = s2 * (S + a * a * s2 * (1.0 + 2.0 * H))
    return alpha, beta, gam


def sqrt_det_gamma(r, th, M, a):
    """sqrt(det gamma_ij) = Sigma sin(theta) sqrt(1+2H)."""
    S = sigma(r, th, a)
    return S * np.sin(th) * np.sqrt(1.0 + 2.0 * M * r / S)


def horizon_radius(M, a):
    """Outer event horizon r_h = M + sqrt(M^2 - a^2)."""
    return M + np.sqrt(M * M - a * a)
