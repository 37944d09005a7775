"""Pins for the Kerr-Schild background (Results: The Kerr-Schild Metric and
3+1 Decomposition; Appendix table of the ADM split at a = 0.5)."""

import json
import os

import numpy as np
import pytest

from oracle import kerr_schild as ks

GOLD = os.path.join(os.path.dirname(__file__), "golden", "kerr_adm_table.json")


def _points():
    rng = np.random.default_rng(7)
    r = rng.uniform(1.2, 30.0, 200)
    th = rng.uniform(0.05, np.pi - 0.05, 200)
    return r, th


@pytest.mark.parametrize("a", [0.0, 0.5, 0.9375])
def test_closed_form_split_matches_line_element(a):
    """alpha^2 = beta_k beta^k - g_tt, beta^i = gamma^{ij} g_tj, gamma_ij = g_ij
    computed numerically from the 4-metric reproduce the closed forms."""
    r, th = _points()
    g = ks.metric4(r, th, 1.0, a)
    alpha, beta, gam = ks.adm(r, th, 1.0, a)
    gam4 = g[1:, 1:]
    assert np.abs(gam4 - gam).max() < 1e-13 * np.abs(gam).max()
    gmat = np.moveaxis(gam4, (0, 1), (-2, -1))
    beta_num = np.linalg.solve(gmat, np.moveaxis(g[0, 1:], 0, -1)[..., None])[..., 0]
    beta_num = np.moveaxis(beta_num, -1, 0)
    assert np.abs(beta_num - beta).max() < 1e-13
    a2 = np.einsum('i...,i...->...', g[0, 1:], beta_num) - g[0, 0]
    assert np.abs(np.sqrt(a2) - alpha).max() < 1e-14
    det = np.linalg.det(gmat)
    assert np.abs(np.sqrt(det) / ks.sqrt_det_gamma(r, th, 1.0, a) - 1).max() < 1e-13
    # inverse 4-metric: g^{tt} = -1/alpha^2 (3+1 identity)
    g4inv = np.linalg.inv(np.moveaxis(g, (0, 1), (-2, -1)))
    assert np.abs(g4inv[..., 0, 0] * alpha ** 2 + 1).max() < 1e-12


@pytest.mark.parametrize("a", [0.0, 0.5, 0.9])
def test_horizon_is_where_grr_vanishes(a):
    """g^{rr} = Delta/Sigma vanishes at r_h = M + sqrt(M^2 - a^2)."""
    rh = ks.horizon_radius(1.0, a)
    th = np.linspace(0.1, 3.0, 7)
    g4inv = np.linalg.inv(np.moveaxis(ks.metric4(np.full_like(th, rh), th, 1.0, a), (0, 1), (-2, -1)))
    assert np.abs(g4inv[..., 1, 1]).max() < 1e-13
    g4inv_out = np.linalg.inv(np.moveaxis(ks.metric4(np.full_like(th, rh * 1.1), th, 1.0, a), (0, 1), (-2, -1)))
    assert np.all(g4inv_out[..., 1, 1] > 0)


def test_appendix_table_a05():
    tab = json.load(open(GOLD))
    M, a = tab["M"], tab["a"]
    r, th = _points()
    S = r ** 2 + a ** 2 * np.cos(th) ** 2
    env = dict(r=r, th=th, S=S, a=a, sqrt=np.sqrt, sin=np.sin, cos=np.cos)
    ev = {k: eval(v, {"__builtins__": {}}, env) for k, v in tab["entries"].items()}
    alpha, beta, gam = ks.adm(r, th, M, a)
    assert np.abs(ev["alpha"] - alpha).max() < 1e-14
    assert np.abs(ev["g_thth"] - gam[1, 1]).max() < 1e-12
    assert np.abs(ev["g_phph"] - gam[2, 2]).max() < 1e-11 * np.abs(gam[2, 2]).max()
    assert np.abs(ev["g_x1x1"] - r ** 2 * gam[0, 0]).max() < 1e-12 * np.abs(ev["g_x1x1"]).max()
    assert np.all(beta[1] == 0)
    # the printed beta^r row is the garbled one; the line element gives 2r/(Sigma+2r)
    assert np.abs(beta[0] - 2 * r / (S + 2 * r)).max() < 1e-15
    assert np.abs(ev["beta_r_printed"] - beta[0]).max() > 0.1
