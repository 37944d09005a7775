// Host initial data: Kerr-Schild background in BSSN variables, magnetised
// Michel accretion and the seeded density perturbation.
//
// Paper: Results, "The Kerr-Schild Metric and 3+1 Decomposition" (line
// element, H = M r / Sigma, alpha = (1+2H)^(-1/2)); Methods, "BSSN Evolution
// Equations" (conformal variables).  The matter data are the standard
// relativistic Bondi (Michel) flow: rest-mass flux rho u^r r^2 and Bernoulli
// constant h^2 (1 - 2M/r + (u^r)^2) fixed by the sonic point u_c^2 = M/(2 r_c),
// c_s^2 = u_c^2/(1 - 3 u_c^2) of a polytrope; a monopole field
// sqrt(gamma) B^r = B0 sin(theta) scaled to a minimum plasma beta.
//
// Readings: phi = (1/12) ln det gamma; K_ij = L_beta gamma_ij / (2 alpha)
// (stationary background) and Gamma-tilde^i = gt^jk Gamma-tilde^i_jk with
// spectral derivatives; K0 = K - beta^k d_k alpha / (2 alpha); the Michel
// radial profile is used for every spin with u^theta = u^phi = 0 and u^t from
// the normalisation; supersonic branch inside r_c, subsonic outside.
// The background does not depend on phi, so its derivatives are taken on one
// (theta, r) plane and phi-derivatives are zero.
#include <math.h>
#include <stdio.h>

#include <algorithm>

#include "grmhd_internal.h"

namespace grmhd {

namespace {

struct Bondi {
  double M, G, rc, rhoc, n, Tc, Kp, uc, C1, C2;
  Bondi(double M_, double G_, double rc_, double rhoc_) : M(M_), G(G_), rc(rc_), rhoc(rhoc_) {
    n = 1.0 / (G - 1.0);
    const double uc2 = M / (2.0 * rc);
    const double cs2 = uc2 / (1.0 - 3.0 * uc2);
    Tc = cs2 / (G - (n + 1.0) * cs2);   // c_s^2 = G T / (1 + (n+1) T)
    Kp = Tc / pow(rhoc, G - 1.0);
    uc = sqrt(uc2);
    C1 = rhoc * uc * rc * rc;
    C2 = pow(1.0 + (n + 1.0) * Tc, 2) * (1.0 - 2.0 * M / rc + uc2);
  }
  // Bernoulli residual as a function of ln T at radius r
  double F(double lnT, double r) const {
    const double T = exp(lnT);
    const double rho = pow(T / Kp, n);
    const double u = C1 / (r * r * rho);
    const double h = 1.0 + (n + 1.0) * T;
    return h * h * (1.0 - 2.0 * M / r + u * u) - C2;
  }
  // T = p/rho on the transonic branch: scan ln T, take the first + to - sign
  // change inside r_c (supersonic) or the last - to + outside (subsonic),
  // bisect to adjacent doubles; no sign change (double root at r ~ r_c):
  // golden-section minimum of F.
  double temperature(double r) const {
    const int NS = 8001;
    const double a = log(Tc) - 30.0, b = log(Tc) + 12.0;
    std::vector<double> g(NS), f(NS);
    for (int i = 0; i < NS; ++i) {
      g[i] = a + (b - a) * i / (NS - 1);
      f[i] = F(g[i], r);
    }
    int i0 = -1;
    for (int i = 0; i + 1 < NS; ++i) {
      const bool change = (f[i] > 0 && f[i + 1] < 0) || (f[i] < 0 && f[i + 1] > 0);
      if (!change) continue;
      if (r < rc) {
        if (f[i] > 0) { i0 = i; break; }
      } else if (f[i] < 0) {
        i0 = i;
      }
    }
    if (i0 < 0) {
      int im = (int)(std::min_element(f.begin(), f.end()) - f.begin());
      double lo = g[std::max(im - 1, 0)], hi = g[std::min(im + 1, NS - 1)];
      const double gr = (sqrt(5.0) - 1.0) / 2.0;
      for (int it = 0; it < 200; ++it) {
        const double m1 = hi - gr * (hi - lo), m2 = lo + gr * (hi - lo);
        if (F(m1, r) < F(m2, r)) hi = m2;
        else lo = m1;
      }
      return exp(0.5 * (lo + hi));
    }
    double lo = g[i0], hi = g[i0 + 1];
    const bool lo_pos = F(lo, r) > 0;
    for (;;) {
      const double mid = 0.5 * (lo + hi);
      if (!(lo < mid && mid < hi)) break;
      if ((F(mid, r) > 0) == lo_pos) lo = mid;
      else hi = mid;
    }
    return exp(0.5 * (lo + hi));
  }
};

// 3x3 symmetric helpers on row-major 9-arrays
double det3(const double* g) {
  return g[0] * (g[4] * g[8] - g[5] * g[7]) - g[1] * (g[3] * g[8] - g[5] * g[6]) + g[2] * (g[3] * g[7] - g[4] * g[6]);
}
void inv3(const double* g, double* u) {
  const double d = det3(g);
  u[0] = (g[4] * g[8] - g[5] * g[7]) / d;
  u[1] = (g[2] * g[7] - g[1] * g[8]) / d;
  u[2] = (g[1] * g[5] - g[2] * g[4]) / d;
  u[3] = (g[5] * g[6] - g[3] * g[8]) / d;
  u[4] = (g[0] * g[8] - g[2] * g[6]) / d;
  u[5] = (g[2] * g[3] - g[0] * g[5]) / d;
  u[6] = (g[3] * g[7] - g[4] * g[6]) / d;
  u[7] = (g[1] * g[6] - g[0] * g[7]) / d;
  u[8] = (g[0] * g[4] - g[1] * g[3]) / d;
}
const int SI[6] = {0, 0, 0, 1, 1, 2}, SJ[6] = {0, 1, 2, 1, 2, 2};

}  // namespace

int host_initial_plane(const grmhd_grid& gr, const grmhd_phys& ph, const Operators& ops,
                       std::vector<double>* plane, std::string* err) {
  const int nr = gr.nr, nth = gr.nth;
  const size_t PL = (size_t)nr * nth;
  const double M = ph.M, a = ph.a;
  auto bad = [&](const char* why) {
    if (err) *err = std::string("initial data: ") + why;
    return GRMHD_E_ARG;
  };
  if (!(M > 0.0)) return bad("needs a black hole, M > 0");
  if (!(ph.pert_amp >= 0.0 && ph.pert_amp < 1.0)) return bad("needs 0 <= pert_amp < 1");
  if (ph.id_kind == GRMHD_ID_MICHEL && !(ph.rho_c > 0.0 && ph.beta_min > 0.0))
    return bad("Michel flow needs rho_c > 0 and beta_min > 0");
  // derivative along r / theta of a plane function f[k * nr + j]
  auto dr = [&](const std::vector<double>& f, std::vector<double>& out) {
    const int np = ops.npad[0];
    const std::vector<double>& AT = ops.at[0][OP_D1];
    out.assign(PL, 0.0);
    for (int k = 0; k < nth; ++k)
      for (int i = 0; i < nr; ++i) {
        double s = 0.0;
        for (int m = 0; m < nr; ++m) s += AT[(size_t)m * np + i] * f[(size_t)k * nr + m];
        out[(size_t)k * nr + i] = s;
      }
  };
  auto dth = [&](const std::vector<double>& f, std::vector<double>& out) {
    const int np = ops.npad[1];
    const std::vector<double>& AT = ops.at[1][OP_D1];
    out.assign(PL, 0.0);
    for (int i = 0; i < nth; ++i)
      for (int j = 0; j < nr; ++j) {
        double s = 0.0;
        for (int m = 0; m < nth; ++m) s += AT[(size_t)m * np + i] * f[(size_t)m * nr + j];
        out[(size_t)i * nr + j] = s;
      }
  };

  // ---- Kerr-Schild 3+1 fields on the (theta, r) plane ----
  std::vector<double> alpha(PL), betar(PL), gam[9];
  for (int c = 0; c < 9; ++c) gam[c].assign(PL, 0.0);
  for (int k = 0; k < nth; ++k)
    for (int j = 0; j < nr; ++j) {
      const size_t e = (size_t)k * nr + j;
      const double r = ops.r[j], th = ops.th[k];
      const double S = r * r + a * a * cos(th) * cos(th);
      const double H = M * r / S;
      const double s2 = sin(th) * sin(th);
      alpha[e] = 1.0 / sqrt(1.0 + 2.0 * H);
      betar[e] = 2.0 * H / (1.0 + 2.0 * H);
      gam[0][e] = 1.0 + 2.0 * H;
      gam[2][e] = gam[6][e] = -a * s2 * (1.0 + 2.0 * H);
      gam[4][e] = S;
      gam[8][e] = s2 * (S + a * a * s2 * (1.0 + 2.0 * H));
    }
  // spectral derivatives of gamma_ij and beta^r along r and theta
  std::vector<double> dgam[2][9], dbr[2], tmp;
  for (int c = 0; c < 9; ++c) {
    dr(gam[c], dgam[0][c]);
    dth(gam[c], dgam[1][c]);
  }
  dr(betar, dbr[0]);
  dth(betar, dbr[1]);

  std::vector<double> phi(PL), gt[6], At[6], Kf(PL), Gt[3], K0(PL);
  for (int s = 0; s < 6; ++s) {
    gt[s].assign(PL, 0.0);
    At[s].assign(PL, 0.0);
  }
  for (int i = 0; i < 3; ++i) Gt[i].assign(PL, 0.0);
  for (size_t e = 0; e < PL; ++e) {
    double g[9], gu[9];
    for (int c = 0; c < 9; ++c) g[c] = gam[c][e];
    inv3(g, gu);
    phi[e] = log(det3(g)) / 12.0;
    const double em4 = exp(-4.0 * phi[e]);
    // K_ij = (beta^k d_k gamma_ij + gamma_ik d_j beta^k + gamma_jk d_i beta^k)/(2 alpha);
    // only beta^r is non-zero, phi-derivatives vanish
    double Kij[9];
    for (int i = 0; i < 3; ++i)
      for (int jj = 0; jj < 3; ++jj) {
        double v = betar[e] * dgam[0][i * 3 + jj][e];
        if (jj < 2) v += g[i * 3 + 0] * dbr[jj][e];
        if (i < 2) v += g[jj * 3 + 0] * dbr[i][e];
        Kij[i * 3 + jj] = v / (2.0 * alpha[e]);
      }
    double K = 0.0;
    for (int c = 0; c < 9; ++c) K += gu[c] * Kij[c];
    Kf[e] = K;
    for (int s = 0; s < 6; ++s) {
      const int c = SI[s] * 3 + SJ[s];
      gt[s][e] = em4 * g[c];
      At[s][e] = em4 * (Kij[c] - g[c] * K / 3.0);
    }
  }
  // Gamma-tilde^i = gt^jk Gamma-tilde^i_jk from spectral derivatives of gt_ij
  {
    std::vector<double> dgt[2][6];
    for (int s = 0; s < 6; ++s) {
      dr(gt[s], dgt[0][s]);
      dth(gt[s], dgt[1][s]);
    }
    for (size_t e = 0; e < PL; ++e) {
      double g[9], gu[9], d[3][9];
      for (int s = 0; s < 6; ++s) {
        const int i = SI[s], jj = SJ[s];
        g[i * 3 + jj] = g[jj * 3 + i] = gt[s][e];
        for (int q = 0; q < 2; ++q) d[q][i * 3 + jj] = d[q][jj * 3 + i] = dgt[q][s][e];
        d[2][i * 3 + jj] = d[2][jj * 3 + i] = 0.0;
      }
      inv3(g, gu);
      // Gamma-tilde_ljk = (d_j g_lk + d_k g_lj - d_l g_jk)/2
      for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int l = 0; l < 3; ++l)
          for (int jj = 0; jj < 3; ++jj)
            for (int kk = 0; kk < 3; ++kk) {
              const double Gl = 0.5 * (d[jj][l * 3 + kk] + d[kk][l * 3 + jj] - d[l][jj * 3 + kk]);
              s += gu[i * 3 + l] * gu[jj * 3 + kk] * Gl;
            }
        Gt[i][e] = s;
      }
    }
  }
  // K0 = K - beta^k d_k alpha / (2 alpha)
  {
    std::vector<double> dal;
    dr(alpha, dal);
    for (size_t e = 0; e < PL; ++e) K0[e] = Kf[e] - betar[e] * dal[e] / (2.0 * alpha[e]);
  }

  // ---- matter on the (theta, r) plane: rho, p, v^i (upper), densitised B^i ----
  std::vector<double> rho_pl(PL), p_pl(PL), sqrtg(PL), v_pl[3], sB_pl[3];
  for (int i = 0; i < 3; ++i) {
    v_pl[i].assign(PL, 0.0);
    sB_pl[i].assign(PL, 0.0);
  }
  std::vector<double> gm_pl[9];  // physical metric e^{4 phi} gt_ij
  for (int c = 0; c < 9; ++c) gm_pl[c].assign(PL, 0.0);
  for (size_t e = 0; e < PL; ++e) {
    const double e4 = exp(4.0 * phi[e]);
    double gtm[9];
    for (int s = 0; s < 6; ++s) gtm[SI[s] * 3 + SJ[s]] = gtm[SJ[s] * 3 + SI[s]] = gt[s][e];
    for (int c = 0; c < 9; ++c) gm_pl[c][e] = e4 * gtm[c];
    sqrtg[e] = exp(6.0 * phi[e]) * sqrt(det3(gtm));
  }
  // b^2 of the field sB/sqrt(gamma) carried by velocity v at plane point e
  auto bsq = [&](size_t e, const double* sBe, const double* ve) {
    double vl[3], Bu[3], Bl[3];
    for (int i = 0; i < 3; ++i) Bu[i] = sBe[i] / sqrtg[e];
    for (int i = 0; i < 3; ++i) {
      vl[i] = gm_pl[i * 3 + 0][e] * ve[0] + gm_pl[i * 3 + 1][e] * ve[1] + gm_pl[i * 3 + 2][e] * ve[2];
      Bl[i] = gm_pl[i * 3 + 0][e] * Bu[0] + gm_pl[i * 3 + 1][e] * Bu[1] + gm_pl[i * 3 + 2][e] * Bu[2];
    }
    const double v2 = ve[0] * vl[0] + ve[1] * vl[1] + ve[2] * vl[2];
    const double iW2 = 1.0 - v2;
    const double Bv = Bu[0] * vl[0] + Bu[1] * vl[1] + Bu[2] * vl[2];
    const double B2 = Bu[0] * Bl[0] + Bu[1] * Bl[1] + Bu[2] * Bl[2];
    return B2 * iW2 + Bv * Bv;
  };
  double B0 = NAN;
  const bool torus = ph.id_kind == GRMHD_ID_TORUS;
  if (!torus) {
    // Michel flow + monopole sqrt(gamma) B^r = B0 sin(theta)
    const Bondi mic(M, ph.gamma_ad, ph.r_c, ph.rho_c);
    // a transonic solution needs 0 < T_c, i.e. r_c > M (3 Gamma - 2) / (2 (Gamma - 1))
    if (!(ph.r_c > 0.0 && mic.Tc > 0.0 && std::isfinite(mic.Tc) && std::isfinite(mic.Kp)))
      return bad("no transonic Michel flow for this r_c (need r_c > M (3 Gamma - 2) / (2 (Gamma - 1)))");
    std::vector<double> rho1(nr), p1(nr), ur1(nr);
    for (int j = 0; j < nr; ++j) {
      const double r = ops.r[j];
      const double T = mic.temperature(r);
      rho1[j] = pow(T / mic.Kp, mic.n);
      p1[j] = rho1[j] * T;
      ur1[j] = -mic.C1 / (r * r * rho1[j]);
    }
    double min_pb = INFINITY;
    for (int k = 0; k < nth; ++k)
      for (int j = 0; j < nr; ++j) {
        const size_t e = (size_t)k * nr + j;
        const double r = ops.r[j], th = ops.th[k];
        const double S = r * r + a * a * cos(th) * cos(th);
        const double H = M * r / S;
        // u^t from g_tt (u^t)^2 + 2 g_tr u^t u^r + g_rr (u^r)^2 = -1
        const double gtt = -(1.0 - 2.0 * H), gtr = 2.0 * H, grr = 1.0 + 2.0 * H;
        const double ur = ur1[j];
        const double A = gtt, Bq = gtr * ur, C = grr * ur * ur + 1.0;
        const double ut = C / (-Bq + sqrt(Bq * Bq - A * C));
        const double W = alpha[e] * ut;
        rho_pl[e] = rho1[j];
        p_pl[e] = p1[j];
        v_pl[0][e] = ur / W + betar[e] / alpha[e];
        sB_pl[0][e] = sin(th);
        const double sBe[3] = {sB_pl[0][e], 0.0, 0.0}, ve[3] = {v_pl[0][e], 0.0, 0.0};
        min_pb = std::min(min_pb, p_pl[e] / bsq(e, sBe, ve));
      }
    B0 = sqrt(2.0 * min_pb / ph.beta_min);
  } else {
    // Fishbone-Moncrief torus of constant ell = u^t u_phi, isentropic
    // p = K rho^Gamma, purely azimuthal flow; g_tt, g_tphi, g_phiphi (and
    // hence u^t, u^phi) agree in Boyer-Lindquist and Kerr-Schild coordinates.
    const double G = ph.gamma_ad;
    const double sM = sqrt(M);
    auto ell_of = [&](double r) {  // u^t u_phi, prograde circular equatorial geodesic
      const double q = sqrt(pow(r, 1.5) - 3.0 * M * sqrt(r) + 2.0 * a * sM);
      const double ut = (pow(r, 1.5) + a * sM) / (pow(r, 0.75) * q);
      const double uphi = sM * (r * r - 2.0 * a * sqrt(M * r) + a * a) / (pow(r, 0.75) * q);
      return ut * uphi;
    };
    const double ell = ell_of(ph.tor_r_max);
    struct Flow { double ut, uph, lnh_raw; };
    auto flow = [&](double r, double th) {
      const double S = r * r + a * a * cos(th) * cos(th);
      const double H = M * r / S;
      const double s2 = sin(th) * sin(th);
      const double gtt = -(1.0 - 2.0 * H), gtp = -2.0 * a * H * s2;
      const double gpp = s2 * (S + a * a * s2 * (1.0 + 2.0 * H));
      const double omega = -gtp / gpp;
      const double alz = sqrt(omega * omega * gpp - gtt);          // ZAMO lapse
      const double c = ell * alz / sqrt(gpp);
      const double V = (sqrt(1.0 + 4.0 * c * c) - 1.0) / (2.0 * c);  // ZAMO azimuthal speed
      const double ut = 1.0 / (alz * sqrt(1.0 - V * V));
      const double Om = omega + alz * V / sqrt(gpp);
      const double u_t = ut * (gtt + gtp * Om);
      // integral of the circular-flow Euler equation at constant ell
      return Flow{ut, ut * Om, log(1.0 + ell * Om) - log(-u_t) - ell * Om};
    };
    const double lnh_in = flow(ph.tor_r_in, 0.5 * M_PI).lnh_raw;
    const double h_max = exp(flow(ph.tor_r_max, 0.5 * M_PI).lnh_raw - lnh_in);
    const double Kp = (h_max - 1.0) * (G - 1.0) / (G * pow(ph.tor_rho_max, G - 1.0));
    std::vector<double> rho_t(PL, 0.0), Aph(PL, 0.0);
    for (int k = 0; k < nth; ++k)
      for (int j = 0; j < nr; ++j) {
        const size_t e = (size_t)k * nr + j;
        const double r = ops.r[j], th = ops.th[k];
        double ut = 0.0, uph = 0.0;
        if (r >= ph.tor_r_in) {
          const Flow f = flow(r, th);
          const double lnh = f.lnh_raw - lnh_in;
          if (lnh > 0.0) {
            rho_t[e] = pow(expm1(lnh) * (G - 1.0) / (Kp * G), 1.0 / (G - 1.0));
            ut = f.ut;
            uph = f.uph;
          }
        }
        const double rho_a = ph.tor_atm * ph.tor_rho_max * pow(r / ph.tor_r_max, -1.5);
        rho_pl[e] = std::max(rho_t[e], rho_a);
        p_pl[e] = Kp * pow(rho_pl[e], G);
        if (rho_t[e] > 0.0) {
          v_pl[0][e] = betar[e] / alpha[e];
          v_pl[2][e] = uph / (alpha[e] * ut);
        }
        Aph[e] = std::max(rho_t[e] / ph.tor_rho_max - ph.tor_loop_cut, 0.0);
      }
    // one poloidal loop: sqrt(gamma) B^r = d_theta A_phi, sqrt(gamma) B^theta = -d_r A_phi
    std::vector<double> dA;
    dth(Aph, dA);
    sB_pl[0] = dA;
    dr(Aph, dA);
    for (size_t e = 0; e < PL; ++e) sB_pl[1][e] = -dA[e];
    double min_pb = INFINITY;
    for (size_t e = 0; e < PL; ++e) {
      if (!(Aph[e] > 0.0)) continue;
      const double sBe[3] = {sB_pl[0][e], sB_pl[1][e], 0.0};
      const double ve[3] = {v_pl[0][e], v_pl[1][e], v_pl[2][e]};
      min_pb = std::min(min_pb, p_pl[e] / bsq(e, sBe, ve));
    }
    B0 = sqrt(2.0 * min_pb / ph.beta_min);
  }
  for (int i = 0; i < 3; ++i)
    for (size_t e = 0; e < PL; ++e) sB_pl[i][e] *= B0;
  if (!(B0 > 0.0) || !std::isfinite(B0)) {
    if (err) *err = "initial data: field normalisation failed";
    return GRMHD_E_ARG;
  }

  // ---- the plane fields, in the order of the PL_* indices ----
  plane->assign((size_t)PL_NFIELDS * PL, 0.0);
  double* out = plane->data();
  auto put = [&](int f, const std::vector<double>& v) { std::copy(v.begin(), v.end(), out + (size_t)f * PL); };
  put(PL_PHI, phi);
  for (int s = 0; s < 6; ++s) {
    put(PL_GT + s, gt[s]);
    put(PL_AT + s, At[s]);
  }
  put(PL_K, Kf);
  for (int i = 0; i < 3; ++i) put(PL_GAMT + i, Gt[i]);
  put(PL_ALPHA, alpha);
  put(PL_BETAR, betar);
  put(PL_K0, K0);
  put(PL_RHO, rho_pl);
  put(PL_P, p_pl);
  for (int i = 0; i < 3; ++i) {
    put(PL_V + i, v_pl[i]);
    put(PL_SB + i, sB_pl[i]);
  }
  put(PL_SQRTG, sqrtg);
  for (int c = 0; c < 9; ++c) put(PL_GM + c, gm_pl[c]);
  for (const double v : *plane)
    if (!std::isfinite(v)) return bad("a plane field is not finite (excision radius or parameters out of range)");
  return GRMHD_OK;
}

}  // namespace grmhd
