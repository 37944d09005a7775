"""BSSN + 1+log slicing + Gamma-driver right-hand side, oracle side.

Paper: Methods, "BSSN Evolution Equations", "Gauge Conditions" (1+log slicing
and Gamma-driver shift) and "Stress-Energy Tensor" (matter coupling).  The paper
cites Alcubierre's textbook for the ADM/BSSN formalism; the Ricci tensor,
D_i D_j alpha and the matter projections it does not print are the textbook
forms written out below.

Readings of the paper taken here (where it is silent or inconsistent):
  * conformal factor phi = (1/12) ln det gamma_ij (the printed (1/4) ln det
    contradicts the printed d_t phi = -alpha K/6 + ...).
  * the Gamma-tilde equation carries the standard +12 alpha A^{ij} d_j phi
    term (2 alpha * 6 A^{ij} d_j phi), and j^i = gamma-tilde^{ij} S_j.
  * Gamma-tilde^i enters as the evolved variable where it is differentiated
    (the Ricci term and the advection term) and as
    Gamma-tilde_d^i = gamma-tilde^{jk} Gamma-tilde^i_{jk} everywhere else.
  * det gamma-tilde = 1 and tr A-tilde = 0 are not enforced.
  * 1+log slicing is taken as d_t alpha = beta^i d_i alpha - 2 alpha (K - K0)
    with a static field K0 chosen at t = 0 so that the initial slice is
    stationary (K0 = K - beta^k d_k alpha/(2 alpha)); the literal
    -2 alpha K is selected by gauge_k0 = False.
  * Gamma-driver: d_t beta^i = (3/4) B^i, d_t B^i = d_t Gamma-tilde^i - eta B^i
    (no advection terms, as printed); the driver field is called Bd here to
    keep it apart from the magnetic field.
"""

import numpy as np

from .grmhd import inv3

PI = np.pi
SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def conformal_christoffel(gtu, dgt):
    """Gamma-tilde_{ijk} = (d_j gt_ik + d_k gt_ij - d_i gt_jk)/2 and
    Gamma-tilde^i_{jk} = gt^{il} Gamma-tilde_{ljk}; dgt[k, i, j] = d_k gt_ij."""
    Gl = 0.5 * (np.einsum('jik...->ijk...', dgt) + np.einsum('kij...->ijk...', dgt) - dgt)
    Gu = np.einsum('il...,ljk...->ijk...', gtu, Gl)
    return Gl, Gu


def ricci(gt, gtu, dgt, ddgt, dGt, dphi, ddphi):
    """R_ij = R-tilde_ij + R^phi_ij (textbook BSSN form).

    R-tilde_ij = -1/2 gt^{lm} d_l d_m gt_ij + gt_k(i d_j) Gt^k + Gd^k Gl_(ij)k
                 + gt^{lm} (2 Gu^k_l(i Gl_j)km + Gu^k_im Gl_klj)
    R^phi_ij   = -2 Dt_i Dt_j phi - 2 gt_ij gt^{lm} Dt_l Dt_m phi
                 + 4 d_i phi d_j phi - 4 gt_ij gt^{lm} d_l phi d_m phi
    dGt[j, k] = d_j Gamma-tilde^k (evolved); ddgt[l, m, i, j] = d_l d_m gt_ij."""
    Gl, Gu = conformal_christoffel(gtu, dgt)
    Gd = np.einsum('jk...,ijk...->i...', gtu, Gu)
    Rt = -0.5 * np.einsum('lm...,lmij...->ij...', gtu, ddgt)
    Rt += 0.5 * (np.einsum('ki...,jk...->ij...', gt, dGt) + np.einsum('kj...,ik...->ij...', gt, dGt))
    Rt += 0.5 * (np.einsum('k...,ijk...->ij...', Gd, Gl) + np.einsum('k...,jik...->ij...', Gd, Gl))
    Rt += np.einsum('lm...,kli...,jkm...->ij...', gtu, Gu, Gl)
    Rt += np.einsum('lm...,klj...,ikm...->ij...', gtu, Gu, Gl)
    Rt += np.einsum('lm...,kim...,klj...->ij...', gtu, Gu, Gl)
    DDphi = ddphi - np.einsum('kij...,k...->ij...', Gu, dphi)
    lap = np.einsum('lm...,lm...->...', gtu, DDphi)
    grad2 = np.einsum('lm...,l...,m...->...', gtu, dphi, dphi)
    Rphi = -2.0 * DDphi - 2.0 * gt * lap + 4.0 * np.einsum('i...,j...->ij...', dphi, dphi) \
        - 4.0 * gt * grad2
    return Rt + Rphi, Gl, Gu, Gd


def bssn_rhs(f, d, dd, E, S_lo, Sij, K0, eta, gauge_k0=True):
    """Right-hand sides of the 24 spacetime variables.

    f  : dict phi, gt[3,3], At[3,3], K, Gt[3], alpha, beta[3], Bd[3]
    d  : dict of first derivatives, derivative index first:
         phi[k], gt[k,i,j], At[k,i,j], K[k], Gt[k,i], alpha[k], beta[k,i]
    dd : dict of second derivatives: phi[k,l], gt[k,l,i,j], alpha[k,l], beta[k,l,i]
    E, S_lo[3], Sij[3,3]: ADM energy density, momentum density, spatial stress.
    Returns a dict with the same keys as f."""
    phi, gt, At, K, alpha, beta, Bd = f['phi'], f['gt'], f['At'], f['K'], f['alpha'], f['beta'], f['Bd']
    dphi, dgt, dAt, dK, dGt, dal, dbeta = d['phi'], d['gt'], d['At'], d['K'], d['Gt'], d['alpha'], d['beta']
    gtu = inv3(gt)
    em4 = np.exp(-4.0 * phi)
    R, Gl, Gu, Gd = ricci(gt, gtu, dgt, dd['gt'], dGt, dphi, dd['phi'])
    dphi_up = np.einsum('kl...,l...->k...', gtu, dphi)
    Gphys = Gu + 2.0 * (np.einsum('ki,j...->kij...', np.eye(3), dphi)
                        + np.einsum('kj,i...->kij...', np.eye(3), dphi)
                        - np.einsum('ij...,k...->kij...', gt, dphi_up))
    DDa = dd['alpha'] - np.einsum('kij...,k...->ij...', Gphys, dal)
    gu = em4 * gtu
    trDDa = np.einsum('ij...,ij...->...', gu, DDa)
    Atu = np.einsum('ik...,jl...,kl...->ij...', gtu, gtu, At)
    AA = np.einsum('ij...,ij...->...', At, Atu)
    Amix = np.einsum('ik...,kl...,lj...->ij...', At, gtu, At)
    divb = np.einsum('kk...->...', dbeta)
    S_tr = np.einsum('ij...,ij...->...', gu, Sij)

    def adv(dfield):
        return np.einsum('k...,k...->...', beta, dfield)

    r = {}
    r['phi'] = -alpha * K / 6.0 + adv(dphi) + divb / 6.0
    r['gt'] = -2.0 * alpha * At + adv(dgt) \
        + np.einsum('ik...,jk...->ij...', gt, dbeta) + np.einsum('jk...,ik...->ij...', gt, dbeta) \
        - (2.0 / 3.0) * gt * divb
    r['K'] = -trDDa + alpha * (AA + K * K / 3.0) + 4.0 * PI * alpha * (E + S_tr) + adv(dK)
    X = -DDa + alpha * (R - 8.0 * PI * Sij)
    XTF = X - gt * np.einsum('kl...,kl...->...', gtu, X) / 3.0
    r['At'] = em4 * XTF + alpha * (K * At - 2.0 * Amix) + adv(dAt) \
        + np.einsum('ik...,jk...->ij...', At, dbeta) + np.einsum('jk...,ik...->ij...', At, dbeta) \
        - (2.0 / 3.0) * At * divb
    ddb = dd['beta']
    r['Gt'] = -2.0 * np.einsum('ij...,j...->i...', Atu, dal) \
        + 2.0 * alpha * (np.einsum('ijk...,jk...->i...', Gu, Atu)
                         + 6.0 * np.einsum('ij...,j...->i...', Atu, dphi)
                         - (2.0 / 3.0) * np.einsum('ij...,j...->i...', gtu, dK)) \
        - 16.0 * PI * alpha * np.einsum('ij...,j...->i...', gtu, S_lo) \
        + np.einsum('jk...,jki...->i...', gtu, ddb) \
        + np.einsum('ij...,jkk...->i...', gtu, ddb) / 3.0 \
        + np.einsum('j...,ji...->i...', beta, dGt) \
        - np.einsum('j...,ji...->i...', Gd, dbeta) \
        + (2.0 / 3.0) * Gd * divb
    Kdrive = (K - K0) if gauge_k0 else K
    r['alpha'] = adv(dal) - 2.0 * alpha * Kdrive
    r['beta'] = 0.75 * Bd
    r['Bd'] = r['Gt'] - eta * Bd
    return r


def hamiltonian(f, d, dd, E):
    """H = e^{-4 phi} gt^{ij} R_ij + (2/3) K^2 - A_ij A^ij - 16 pi E."""
    gt, At, K, phi = f['gt'], f['At'], f['K'], f['phi']
    gtu = inv3(gt)
    R, _, _, _ = ricci(gt, gtu, d['gt'], dd['gt'], d['Gt'], d['phi'], dd['phi'])
    Atu = np.einsum('ik...,jl...,kl...->ij...', gtu, gtu, At)
    return np.exp(-4.0 * phi) * np.einsum('ij...,ij...->...', gtu, R) + (2.0 / 3.0) * K * K \
        - np.einsum('ij...,ij...->...', At, Atu) - 16.0 * PI * E


def momentum(f, d, S_lo):
    """Momentum constraint in covariant components, from the physical form
    D_j (K^j_i - delta^j_i K) = 8 pi S_i written in the BSSN variables:

      M_i = Dt_j At^j_i + 6 At^j_i d_j phi - (2/3) d_i K - 8 pi S_i,

    with At^j_i = gt^{jk} At_ki (the mixed components of the trace-free part
    of K_ij are the same in the physical and the conformal metric), Dt the
    covariant derivative of gt_ij,
      Dt_j At^j_i = d_j At^j_i + Gt^j_jk At^k_i - Gt^k_ji At^j_k,
    and the 6 At^j_i d_j phi term from sqrt(gamma) = e^{6 phi} sqrt(det gt)
    (the other conformal terms of the Christoffel symbols cancel for a
    trace-free mixed tensor).  S_lo[i] is the momentum density S_i seen by
    normal observers (the undensitised Valencia S_j).  Derivative arrays as
    in bssn_rhs (derivative index first)."""
    gt, At = f['gt'], f['At']
    gtu = inv3(gt)
    dgt = d['gt']
    _, Gu = conformal_christoffel(gtu, dgt)
    # d_k gt^{jl} = -gt^{ja} gt^{lb} d_k gt_ab
    dgtu = -np.einsum('ja...,lb...,kab...->kjl...', gtu, gtu, dgt)
    Amix = np.einsum('jk...,ki...->ji...', gtu, At)          # At^j_i
    divA = np.einsum('jjk...,ki...->i...', dgtu, At) + np.einsum('jk...,jki...->i...', gtu, d['At'])
    trG = np.einsum('jjk...->k...', Gu)                       # Gt^j_jk
    DdivA = divA + np.einsum('k...,ki...->i...', trG, Amix) - np.einsum('kji...,jk...->i...', Gu, Amix)
    return DdivA + 6.0 * np.einsum('ji...,j...->i...', Amix, d['phi']) - (2.0 / 3.0) * d['K'] \
        - 8.0 * PI * S_lo


def momentum_norm(f, M_lo):
    """|M| = sqrt(gamma^{ij} M_i M_j), gamma^{ij} = e^{-4 phi} gt^{ij}."""
    gtu = inv3(f['gt'])
    return np.sqrt(np.exp(-4.0 * f['phi']) * np.einsum('ij...,i...,j...->...', gtu, M_lo, M_lo))
