// Pointwise kernels of the RHS evaluation (one thread per grid point,
// structure-of-arrays FP64 streaming from HBM):
//   k_c2p_flux  : metric reconstruction, primitive recovery (safeguarded
//                 Newton, or the paper's damped iteration), densitised fluxes
//   k_rhs_rk    : BSSN + gauge RHS (Ricci tensor included) with matter
//                 sources, Valencia RHS
//                 (-div + sqrt(gamma) S, GLM terms), boundary freeze, RK4 stage
//                 update (or the split step's Euler update of the spacetime)
//   k_rhs_fixed : the Valencia RHS and RK4 stage on a fixed background
//   k_ham, k_k0 : Hamiltonian and momentum constraints; static 1+log source
//                 K0 = K - beta^k d_k alpha/(2 alpha)
//   k_diag      : per-block partial sums / extrema for diagnostics
//                 (wavefront swizzle reductions)
//
// Paper: Results, "GRMHD Conservative Form" (conserved variables, fluxes,
// Lorentz factor, magnetic four-vector, source term); Methods, "The Primitive
// Variable Recovery", "The Conserved Fluxes and Geometric Source Terms",
// "Stress-Energy Tensor", "BSSN Evolution Equations", "Gauge Conditions",
// "Time Integration".  Forms used where the printed equations are garbled:
// standard Valencia conserved variables and fluxes with lapse and shift
// (vt^i = v^i - beta^i/alpha, conservation law for sqrt(gamma) U with flux
// alpha sqrt(gamma) F^i), 3+1 source terms, textbook BSSN Ricci tensor with
// phi = (1/12) ln det gamma, the +12 alpha A^ij d_j phi term in the
// Gamma-tilde equation, Gamma-tilde from the conformal metric wherever it is
// not differentiated.
#include <math.h>

#include <type_traits>

#include "grmhd_internal.h"

namespace grmhd {

namespace {

constexpr double PI = 3.14159265358979323846;

// symmetric 3x3 storage: xx xy xz yy yz zz
__device__ __forceinline__ int S6(int i, int j) {
  const int t[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
  return t[i][j];
}

struct Sym {
  double m[6];
  __device__ __forceinline__ double operator()(int i, int j) const { return m[S6(i, j)]; }
};

__device__ __forceinline__ double det_sym(const Sym& g) {
  return g.m[0] * (g.m[3] * g.m[5] - g.m[4] * g.m[4]) - g.m[1] * (g.m[1] * g.m[5] - g.m[4] * g.m[2]) +
         g.m[2] * (g.m[1] * g.m[4] - g.m[3] * g.m[2]);
}

__device__ __forceinline__ Sym inv_sym(const Sym& g, double det) {
  const double id = 1.0 / det;
  Sym u;
  u.m[0] = (g.m[3] * g.m[5] - g.m[4] * g.m[4]) * id;
  u.m[1] = (g.m[2] * g.m[4] - g.m[1] * g.m[5]) * id;
  u.m[2] = (g.m[1] * g.m[4] - g.m[2] * g.m[3]) * id;
  u.m[3] = (g.m[0] * g.m[5] - g.m[2] * g.m[2]) * id;
  u.m[4] = (g.m[1] * g.m[2] - g.m[0] * g.m[4]) * id;
  u.m[5] = (g.m[0] * g.m[3] - g.m[1] * g.m[1]) * id;
  return u;
}

__device__ __forceinline__ void mv(const Sym& g, const double* v, double* out) {
#pragma unroll
  for (int i = 0; i < 3; ++i) out[i] = g(i, 0) * v[0] + g(i, 1) * v[1] + g(i, 2) * v[2];
}

__device__ __forceinline__ double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// ---- primitive recovery ------------------------------------------------------
// Unknown Z = rho h W^2.  From S_j = (Z + B^2) v_j - (B.v) B_j and B.S = Z B.v:
//   v^2(Z) = (Z^2 S^2 + (2Z + B^2)(B.S)^2) / (Z^2 (Z + B^2)^2)
// and tau + D = Z + B^2 - p - B^2/(2W^2) - (B.S)^2/(2 Z^2) with the ideal-gas
// p = (Gamma-1)/Gamma (Z/W^2 - D/W).  Newton iteration on the residual with
// analytic derivative, kept inside a bracket [lo, hi] that shrinks with the
// sign of the residual (bisection whenever a step leaves it or v^2 >= 1);
// converged once a Newton step is below 1e-12 relative.
struct C2POut {
  double rho, p, v[3];
  int fail;
};

// Iteration budget of the safeguarded Newton recovery.  From a warm start
// Newton converges in a handful of steps; each step that leaves the bracket
// is replaced by a bisection.  A point neither converged nor reduced to a
// bracket of adjacent doubles after this many iterations is flagged and
// takes the atmosphere (the same policy as the oracle's bisection, which
// flags a point left unresolved by its own budget).
constexpr int C2P_MAXIT = 200;

__device__ C2POut con2prim(double D, const double* S, double tau, const double* B, const Sym& gam,
                           const Sym& gamu, double G, double gm1g, double rho_fl, double p_fl,
                           double zguess) {
  C2POut o;
  double Su[3], Bl[3];
  mv(gamu, S, Su);
  mv(gam, B, Bl);
  const double S2 = dot3(S, Su), B2 = dot3(B, Bl), BS = dot3(B, S), BS2 = BS * BS;
  const double gf = gm1g;
  bool bad = !(D > 0.0 && tau + D > 0.0);
  const double Dc = bad ? 1.0 : D, Ec = bad ? 2.0 : tau + D;
  double lo = 0.0, hi = G * Ec + B2 + 1e-300;
  // residual f and derivative; returns false where v^2 >= 1 (Z below range)
  auto resid = [&](double Z, double& f, double& fp) -> bool {
    const double iZ = 1.0 / Z, ia = 1.0 / (Z + B2);
    const double iZ2 = iZ * iZ, ia2 = ia * ia;
    const double v2 = (S2 + (2.0 * Z + B2) * BS2 * iZ2) * ia2;
    if (!(v2 < 1.0) || !(Z > 0.0)) return false;
    const double iw2 = 1.0 - v2, sq = sqrt(iw2);
    const double dv2 = -2.0 * ia2 * ia * (S2 + BS2 * (3.0 * Z * Z + 3.0 * Z * B2 + B2 * B2) * iZ2 * iZ);
    const double p = gf * (Z * iw2 - Dc * sq);
    const double dp = gf * (iw2 - Z * dv2 + 0.5 * Dc * dv2 / sq);
    f = Z + B2 - p - 0.5 * B2 * iw2 - 0.5 * BS2 * iZ2 - Ec;
    fp = 1.0 - dp + 0.5 * B2 * dv2 + BS2 * iZ2 * iZ;
    return true;
  };
  double f, fp;
  bool upper = false;
  for (int w = 0; w <= 8; ++w) {  // make sure the upper end has f >= 0 (up to 8 doublings)
    upper = resid(hi, f, fp) && f >= 0.0;
    if (upper || w == 8) break;
    hi *= 2.0;
  }
  if (!upper) bad = true;
  double Z = (zguess > lo && zguess < hi) ? zguess : 0.5 * (lo + hi);
  if (!bad) {
    // a point that neither converges nor collapses its bracket within the
    // iteration budget is not a recovered state: it takes the failure policy
    bool done = false;
    for (int it = 0; it < C2P_MAXIT && !done; ++it) {
      double zn;
      if (!resid(Z, f, fp)) {
        lo = Z;
        zn = 0.5 * (lo + hi);
      } else {
        if (f < 0.0) lo = Z;
        else hi = Z;
        zn = Z - f / fp;
        // a Newton step this small leaves an error of the order of its square:
        // accept it before the bracket test (the converged step may land on a
        // bracket end, which must not trigger a bisection)
        if (fabs(zn - Z) <= 1e-12 * zn) {
          Z = zn;
          done = true;
          break;
        }
        if (!(zn > lo && zn < hi)) zn = 0.5 * (lo + hi);
      }
      if (!(zn > lo && zn < hi)) {  // bracket collapsed onto adjacent doubles
        Z = hi;
        done = true;
        break;
      }
      Z = zn;
    }
    if (!done) bad = true;
  }
  double vl[3];
  const double iZ = 1.0 / Z, ia = 1.0 / (Z + B2);
#pragma unroll
  for (int i = 0; i < 3; ++i) vl[i] = (S[i] + BS * Bl[i] * iZ) * ia;
  mv(gamu, vl, o.v);
  const double v2 = dot3(o.v, vl);
  const double iw2 = 1.0 - v2;  // 1/W^2
  o.rho = Dc * sqrt(iw2);
  o.p = gf * (Z * iw2 - o.rho);
  o.fail = bad || !(v2 < 1.0) || !(o.rho >= rho_fl) || !(o.p >= p_fl);
  if (o.fail) {
    o.rho = rho_fl;
    o.p = p_fl;
    o.v[0] = o.v[1] = o.v[2] = 0.0;
  }
  return o;
}

// The paper's damped iteration for the primitive state (Methods, "The
// Primitive Variable Recovery"), from the previous primitives (rho0, p0, v0^i).
// Readings: predicted values are the conserved variables of the current
// primitives (so the fixed point is the exact inverse); the velocity update
// raises Delta S_j with gamma^{ij}; residual |Delta S|_gamma + |Delta tau|; one
// damping factor lambda = 0.5, halved (step retried from the previous iterate)
// when a step does not lower the residual or leaves v^2 < 1, eps > 0; stop
// below 1e-15 (|S|_gamma + |tau| + D) or after 40 tries; if not converged one
// Newton step on eps at fixed rho, v.  An unusable guess starts from v = 0,
// eps = max((tau - B^2/2)/D, eps_floor).  Failure policy as con2prim.
struct DampedState {
  double rho, eps, v[3];
};

__device__ __forceinline__ double damped_resid(const DampedState& x, const double* S, double tau,
                                               const double* B, const double* Bl, double B2, const Sym& gam,
                                               const Sym& gamu, double G, double* dS, double& dT) {
  double vl[3];
  mv(gam, x.v, vl);
  const double v2 = dot3(x.v, vl);
  const double W2 = 1.0 / (1.0 - v2), W = sqrt(W2);
  const double p = (G - 1.0) * x.rho * x.eps;
  const double h = 1.0 + x.eps + p / x.rho;
  const double Z = x.rho * h * W2;
  const double Bv = dot3(B, vl);
#pragma unroll
  for (int i = 0; i < 3; ++i) dS[i] = S[i] - ((Z + B2) * vl[i] - Bv * Bl[i]);
  dT = tau - (Z - p + B2 - 0.5 * (B2 / W2 + Bv * Bv) - x.rho * W);
  double dSu[3];
  mv(gamu, dS, dSu);
  return sqrt(dot3(dS, dSu)) + fabs(dT);
}

__device__ C2POut con2prim_damped(double D, const double* S, double tau, const double* B, const Sym& gam,
                                  const Sym& gamu, double G, double rho_fl, double p_fl, double rho0, double p0,
                                  const double* v0) {
  C2POut o;
  const bool bad = !(D > 0.0 && tau + D > 0.0);
  const double Dc = bad ? 1.0 : D, tc = bad ? 1.0 : tau;
  double Bl[3];
  mv(gam, B, Bl);
  const double B2 = dot3(B, Bl);
  const double gm1 = G - 1.0;
  DampedState x;
  {
    double v0l[3];
    mv(gam, v0, v0l);
    const bool ok = rho0 > 0.0 && p0 > 0.0 && dot3(v0, v0l) < 1.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) x.v[i] = ok ? v0[i] : 0.0;
    x.eps = ok ? p0 / (gm1 * rho0) : fmax((tc - 0.5 * B2) / Dc, p_fl / (gm1 * rho_fl));
    double vl[3];
    mv(gam, x.v, vl);
    x.rho = Dc / (1.0 / sqrt(1.0 - dot3(x.v, vl)));
  }
  double Su[3];
  mv(gamu, S, Su);
  const double scale = sqrt(dot3(S, Su)) + fabs(tc) + Dc;
  double dS[3], dT;
  double r = damped_resid(x, S, tc, B, Bl, B2, gam, gamu, G, dS, dT);
  bool conv = r <= 1e-15 * scale;
  double lam = 0.5;
  for (int it = 0; it < 40 && !conv; ++it) {
    double vl[3];
    mv(gam, x.v, vl);
    const double W2 = 1.0 / (1.0 - dot3(x.v, vl));
    const double h = 1.0 + G * x.eps;
    double dSu[3];
    mv(gamu, dS, dSu);
    DampedState t;
#pragma unroll
    for (int i = 0; i < 3; ++i) t.v[i] = x.v[i] + lam * dSu[i] / (x.rho * h * W2);
    t.eps = x.eps + lam * dT / (x.rho * W2);
    double tl[3];
    mv(gam, t.v, tl);
    const double v2t = dot3(t.v, tl);
    bool acc = v2t < 1.0 && t.eps > 0.0;
    double dSt[3], dTt, rt = 0.0;
    if (acc) {
      t.rho = Dc / (1.0 / sqrt(1.0 - v2t));
      rt = damped_resid(t, S, tc, B, Bl, B2, gam, gamu, G, dSt, dTt);
      acc = rt < r;
    }
    if (acc) {
      x = t;
      r = rt;
#pragma unroll
      for (int i = 0; i < 3; ++i) dS[i] = dSt[i];
      dT = dTt;
      conv = rt <= 1e-15 * scale;
    } else {
      lam *= 0.5;
    }
  }
  double vl[3];
  mv(gam, x.v, vl);
  const double v2 = dot3(x.v, vl);
  if (!conv) {
    const double W2 = 1.0 / (1.0 - v2);
    x.eps += dT / (x.rho * (G * W2 - gm1));
  }
  o.rho = x.rho;
  o.p = gm1 * x.rho * x.eps;
#pragma unroll
  for (int i = 0; i < 3; ++i) o.v[i] = x.v[i];
  o.fail = bad || !(v2 < 1.0) || !(o.rho >= rho_fl) || !(o.p >= p_fl);
  if (o.fail) {
    o.rho = rho_fl;
    o.p = p_fl;
    o.v[0] = o.v[1] = o.v[2] = 0.0;
  }
  return o;
}

// Magnetic quantities for Eulerian field B^i and velocity v^i:
// W, alpha b^0 = W (B.v), b_i = B_i/W + W (B.v) v_i, b^2 = B^2/W^2 + (B.v)^2.
struct Mag {
  double W, iW, ab0, bl[3], b2, vl[3];
};

__device__ __forceinline__ Mag magnetic(const double* v, const double* B, const Sym& gam) {
  Mag m;
  double Bl[3];
  mv(gam, v, m.vl);
  mv(gam, B, Bl);
  const double iw2 = 1.0 - dot3(v, m.vl);  // 1/W^2
  m.iW = sqrt(iw2);
  m.W = 1.0 / m.iW;
  const double Bv = dot3(B, m.vl), B2 = dot3(B, Bl);
  m.ab0 = m.W * Bv;
#pragma unroll
  for (int i = 0; i < 3; ++i) m.bl[i] = Bl[i] * m.iW + m.W * Bv * m.vl[i];
  m.b2 = B2 * iw2 + Bv * Bv;
  return m;
}

// Conformal Christoffels from dgt[a][s] = d_a gt_s:
// Gl_ijk = (d_j gt_ik + d_k gt_ij - d_i gt_jk)/2, Gu^i_jk = gt^il Gl_ljk,
// Gd^i = gt^jk Gu^i_jk.
__device__ __forceinline__ void christoffel(const Sym& gtu, const double dgt[3][6], double Gl[3][6],
                                            double Gu[3][6], double Gd[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj)
#pragma unroll
      for (int kk = jj; kk < 3; ++kk)
        Gl[i][S6(jj, kk)] = 0.5 * (dgt[jj][S6(i, kk)] + dgt[kk][S6(i, jj)] - dgt[i][S6(jj, kk)]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int s = 0; s < 6; ++s) Gu[i][s] = gtu(i, 0) * Gl[0][s] + gtu(i, 1) * Gl[1][s] + gtu(i, 2) * Gl[2][s];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double t = 0.0;
#pragma unroll
    for (int jj = 0; jj < 3; ++jj)
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) t += gtu(jj, kk) * Gu[i][S6(jj, kk)];
    Gd[i] = t;
  }
}

// Ricci tensor of the conformal decomposition, R_ij = Rt_ij + Rphi_ij:
//   Rt_ij = -1/2 gt^lm d_l d_m gt_ij + gt_k(i d_j) Gt^k + Gd^k Gl_(ij)k
//           + gt^lm (Gu^k_li Gl_jkm + Gu^k_lj Gl_ikm + Gu^k_im Gl_klj)
//   Rphi_ij = -2 Dt_i Dt_j phi - 2 gt_ij Dt^l Dt_l phi + 4 d_i phi d_j phi
//             - 4 gt_ij d^l phi d_l phi
// DD(a, b, s): d_a d_b of second-derivative field s (phi 0, gt 1..6).
template <typename Acc>
__device__ __forceinline__ void ricci(const Sym& gt, const Sym& gtu, const double Gl[3][6],
                                      const double Gu[3][6], const double Gd[3], const double dGt[3][3],
                                      const double dphi[3], Acc DD, Sym& R) {
#pragma unroll
  for (int s = 0; s < 6; ++s) R.m[s] = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int m = l; m < 3; ++m) {
      const double w = (l == m ? -0.5 : -1.0) * gtu(l, m);  // symmetric in l, m
#pragma unroll
      for (int s = 0; s < 6; ++s) R.m[s] += w * DD(l, m, 1 + s);
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = i; jj < 3; ++jj) {
      double t = 0.0;
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        t += 0.5 * (gt(kk, i) * dGt[jj][kk] + gt(kk, jj) * dGt[i][kk]);
        t += 0.5 * Gd[kk] * (Gl[i][S6(jj, kk)] + Gl[jj][S6(i, kk)]);
      }
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          double q = 0.0;
#pragma unroll
          for (int kk = 0; kk < 3; ++kk)
            q += Gu[kk][S6(l, i)] * Gl[jj][S6(kk, m)] + Gu[kk][S6(l, jj)] * Gl[i][S6(kk, m)] +
                 Gu[kk][S6(i, m)] * Gl[kk][S6(l, jj)];
          t += gtu(l, m) * q;
        }
      R.m[S6(i, jj)] += t;
    }
  double DDphi[6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = i; jj < 3; ++jj)
      DDphi[S6(i, jj)] = DD(i, jj, 0) - (Gu[0][S6(i, jj)] * dphi[0] + Gu[1][S6(i, jj)] * dphi[1] +
                                         Gu[2][S6(i, jj)] * dphi[2]);
  double lap = 0.0, grad2 = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      lap += gtu(l, m) * DDphi[S6(l, m)];
      grad2 += gtu(l, m) * dphi[l] * dphi[m];
    }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = i; jj < 3; ++jj) {
      const int s = S6(i, jj);
      R.m[s] += -2.0 * DDphi[s] - 2.0 * gt.m[s] * lap + 4.0 * dphi[i] * dphi[jj] - 4.0 * gt.m[s] * grad2;
    }
}

// derivative array offsets relative to the first-derivative block
constexpr int O_D2 = SC_D2 - SC_D1, O_MX = SC_MX - SC_D1, O_DF = SC_DF - SC_D1, O_GLM = SC_GLM - SC_D1;

// Loads of arrays that a launch reads once: non-temporal, so the streams pass
// the caches without evicting each other (the RHS kernels read 80-240 such
// arrays per point).
template <typename T>
__device__ __forceinline__ T ldnt(const T* p) {
  return __builtin_nontemporal_load(p);
}

}  // namespace

// ---------------------------------------------------------------------------
// DAMPED: the paper's damped iteration in place of the safeguarded Newton
// (its own instantiation, so the default kernel keeps its register budget).
template <bool DAMPED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DAMPED ? 2 : 4))) void k_c2p_flux(const double* __restrict__ U,
                                                  const double* __restrict__ Ug,
                                                  double* __restrict__ prim,
                                                  double* __restrict__ fail,
                                                  double* __restrict__ flux,
                                                  const double* __restrict__ floors, PointParams pp,
                                                  JobSet js) {
  const long long P = pp.P;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= P) return;
  {  // this job's buffers
    const long long jd = js.d[blockIdx.y];
    U = shift_ptr(U, jd);
    Ug = shift_ptr(Ug, jd);
    prim = shift_ptr(prim, jd);
    fail = shift_ptr(fail, jd);
    floors = shift_ptr(floors, jd);
    if (flux != nullptr) flux = shift_ptr(flux, jd);
  }
  const int j = (int)(idx % pp.nr);
#define LD(f) ldnt(&U[(size_t)(f) * P + idx])
#define LG(f) ldnt(&Ug[(size_t)(f) * P + idx])
  const double phi = LG(0);
  Sym gt;
#pragma unroll
  for (int s = 0; s < 6; ++s) gt.m[s] = LG(1 + s);
  const double alpha = LG(17);
  double beta[3] = {LG(18), LG(19), LG(20)};
  const double e2 = exp(2.0 * phi), e4 = e2 * e2;
  const double detgt = det_sym(gt);
  const double sqrtg = e4 * e2 * sqrt(detgt);
  Sym gam;
#pragma unroll
  for (int s = 0; s < 6; ++s) gam.m[s] = e4 * gt.m[s];
  const Sym gamu = inv_sym(gam, e4 * e4 * e4 * detgt);
  const double isg = 1.0 / sqrtg;
  const double D = LD(24) * isg, tau = LD(28) * isg;
  double S[3] = {LD(25) * isg, LD(26) * isg, LD(27) * isg};
  double B[3] = {LD(29) * isg, LD(30) * isg, LD(31) * isg};
#undef LG
#undef LD
  const double rho_fl = floors[j], p_fl = floors[pp.nr + j];
  C2POut c;
  if (DAMPED) {  // the paper's iteration from the last recovered primitives
    const double vg[3] = {ldnt(&prim[2 * (size_t)P + idx]), ldnt(&prim[3 * (size_t)P + idx]),
                          ldnt(&prim[4 * (size_t)P + idx])};
    c = con2prim_damped(D, S, tau, B, gam, gamu, pp.gamma_ad, rho_fl, p_fl, ldnt(&prim[idx]),
                        ldnt(&prim[(size_t)P + idx]), vg);
  } else {
  // warm start Z = rho h W^2 from the last recovered primitives
  double zg = -1.0;
  {
    const double rg = ldnt(&prim[idx]), pg = ldnt(&prim[(size_t)P + idx]);
    double vg[3] = {ldnt(&prim[2 * (size_t)P + idx]), ldnt(&prim[3 * (size_t)P + idx]),
                    ldnt(&prim[4 * (size_t)P + idx])};
    double vgl[3];
    mv(gam, vg, vgl);
    const double v2 = dot3(vg, vgl);
    if (rg > 0.0 && pg > 0.0 && v2 < 1.0)
      zg = (rg + pg * pp.gfac) / (1.0 - v2);
  }
  c = con2prim(D, S, tau, B, gam, gamu, pp.gamma_ad, pp.gm1g, rho_fl, p_fl, zg);
  }
  prim[idx] = c.rho;
  prim[(size_t)P + idx] = c.p;
  prim[2 * (size_t)P + idx] = c.v[0];
  prim[3 * (size_t)P + idx] = c.v[1];
  prim[4 * (size_t)P + idx] = c.v[2];
  fail[idx] = c.fail ? 1.0 : 0.0;
  if (flux == nullptr) return;
  const Mag m = magnetic(c.v, B, gam);
  const double ps = c.p + 0.5 * m.b2;
  const double asg = alpha * sqrtg;
  const double iW = m.iW, ial = 1.0 / alpha;
  const double vt[3] = {c.v[0] - beta[0] * ial, c.v[1] - beta[1] * ial, c.v[2] - beta[2] * ial};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double vta = vt[a];
    double* F = flux + (size_t)(8 * a) * P + idx;
    F[0] = asg * D * vta;
#pragma unroll
    for (int jj = 0; jj < 3; ++jj)
      F[(size_t)(1 + jj) * P] = asg * (S[jj] * vta - m.bl[jj] * B[a] * iW + (a == jj ? ps : 0.0));
    F[(size_t)4 * P] = asg * (tau * vta + ps * c.v[a] - m.ab0 * B[a] * iW);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double vtk = vt[k];
      F[(size_t)(5 + k) * P] = asg * (vta * B[k] - vtk * B[a]);
    }
  }
}

// ---------------------------------------------------------------------------
// Second-derivative field index s: phi 0, gt 1..6, alpha 7, beta 8..10.
//
// The kernel finishes one group of right-hand sides at a time and applies the
// RK4 stage update to it at once (phi, gt, gauge; Valencia; then the
// conformal Ricci tensor; K and A-tilde; Gamma-tilde and the driver), with
// compiler scheduling barriers between the phases so that each phase's loads
// are issued where they are consumed and the live register set stays small.
//
// Us, Un, acc and out never share a location that the launch writes: the RK4
// stages alternate between two stage buffers (stage 4 writes U^n, which it
// does not read), the accumulator is read and written through acc alone, and
// a right-hand side (mode 0) goes to a buffer apart from its input.  Declared
// __restrict__, the loads of Un and the accumulator for one field then need
// not wait for the stores of the fields before it.  The split step's forward
// Euler update of the spacetime in place (mode 5, Us = Un = out) is the one
// instantiation without the qualifier.
#define PHASE() __asm__ __volatile__("" ::: "memory")

template <bool R, typename T>
using maybe_restrict = typename std::conditional<R, T* __restrict__, T*>::type;

// Matter terms of one point that the BSSN right-hand sides use: E, S_i,
// S_ij and the trace of S^i_j.
struct Matter {
  double Em, Sl[3], Str;
  Sym Sij;
};

// Valencia right-hand sides of one point: minus the divergence of the
// densitised fluxes (their derivative arrays at O_DF) plus sqrt(gamma) times the
// geometric sources of S_j and tau; with GLM the induction source
// -sqrt(gamma) gamma^{ij} d_j psi and the psi equation.  Geometry: sqrt(gamma),
// e^{+-4 phi}, gt_ij and its inverse, A-tilde_ij, K, alpha and the first
// derivatives of alpha, beta^i, gt_ij and phi ([a][..] = d_a).  Each result goes
// to emit(f, value, U_f) (f = 24..31, and 32 with GLM; U_f the stage value of
// the field, which stage 1 takes as U^n).
template <typename DT, typename Emit>
__device__ __forceinline__ Matter valencia_rhs(const double* Us, const DT* __restrict__ der,
                                               const double* __restrict__ prim, long long idx, long long P,
                                               const PointParams& pp, double sqrtg, double e4, double em4,
                                               const Sym& gt, const Sym& gtu, const Sym& At, double K,
                                               double alpha, const double* dal, const double (*dbeta)[3],
                                               const double (*dgt)[6], const double* dphi, Emit& emit) {
#define LU(f) Us[(size_t)(f) * P + idx]
#define LS(g) ((double)ldnt(&der[(size_t)(g) * P + idx]))
  Matter mt;
  double u[8];  // D, S_j, tau, B^i (densitised)
#pragma unroll
  for (int v = 0; v < 8; ++v) u[v] = LU(24 + v);
  const double isg = 1.0 / sqrtg;
  mt.Em = (u[4] + u[0]) * isg;
  const double Em = mt.Em;
  double* Sl = mt.Sl;
  Sl[0] = u[1] * isg;
  Sl[1] = u[2] * isg;
  Sl[2] = u[3] * isg;
  Sym gam, gamu;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    gam.m[s] = e4 * gt.m[s];
    gamu.m[s] = em4 * gtu.m[s];
  }
  Sym& Sij = mt.Sij;
  {
    const double rho = ldnt(&prim[idx]), p = ldnt(&prim[(size_t)P + idx]);
    const double v[3] = {ldnt(&prim[2 * (size_t)P + idx]), ldnt(&prim[3 * (size_t)P + idx]),
                         ldnt(&prim[4 * (size_t)P + idx])};
    const double B[3] = {u[5] * isg, u[6] * isg, u[7] * isg};
    const Mag m = magnetic(v, B, gam);
    const double h = 1.0 + p / rho * pp.gfac;
    const double cw = (rho * h + m.b2) * m.W * m.W;
    const double ps = p + 0.5 * m.b2;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int jj = i; jj < 3; ++jj)
        Sij.m[S6(i, jj)] = cw * m.vl[i] * m.vl[jj] + ps * gam.m[S6(i, jj)] - m.bl[i] * m.bl[jj];
  }
  double Str = 0.0;
  {
    double Sup[3][3];  // S^{kl} = gamma^{ki} gamma^{lj} S_ij
    double t[3][3];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int jj = 0; jj < 3; ++jj)
        t[kk][jj] = gamu(kk, 0) * Sij(0, jj) + gamu(kk, 1) * Sij(1, jj) + gamu(kk, 2) * Sij(2, jj);
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int l = 0; l < 3; ++l) Sup[kk][l] = t[kk][0] * gamu(l, 0) + t[kk][1] * gamu(l, 1) + t[kk][2] * gamu(l, 2);
#pragma unroll
    for (int i = 0; i < 3; ++i) Str += t[i][i];
    // Sbar_{S_j} = -E d_j alpha + S_k d_j beta^k + (alpha/2) S^{kl} d_j gamma_kl,
    // d_j gamma_kl = e^{4 phi} (d_j gt_kl + 4 gt_kl d_j phi)
    double src[3];
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      double tt = -Em * dal[jj];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) tt += Sl[kk] * dbeta[jj][kk];
      double q = 0.0;
#pragma unroll
      for (int kk = 0; kk < 3; ++kk)
#pragma unroll
        for (int l = 0; l < 3; ++l) q += Sup[kk][l] * e4 * (dgt[jj][S6(kk, l)] + 4.0 * gt(kk, l) * dphi[jj]);
      src[jj] = tt + 0.5 * alpha * q;
    }
    // Sbar_tau = alpha S^{kl} K_kl - S^k d_k alpha, K_kl = e^{4 phi} (A_kl + gt_kl K/3)
    double srcT = 0.0;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int l = 0; l < 3; ++l) srcT += Sup[kk][l] * e4 * (At(kk, l) + gt(kk, l) * K / 3.0);
    srcT *= alpha;
    double Su[3];
    mv(gamu, Sl, Su);
    srcT -= dot3(Su, dal);
    PHASE();
    // GLM: induction source -sqrt(gamma) gamma^{ij} d_j psi
    double sb[3] = {0.0, 0.0, 0.0};
    if (pp.glm) {
      const double dpsi[3] = {LS(O_GLM + 3), LS(O_GLM + 4), LS(O_GLM + 5)};
      mv(gamu, dpsi, sb);
    }
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      double r = -(LS(O_DF + v) + LS(O_DF + 8 + v) + LS(O_DF + 16 + v));
      if (v >= 1 && v <= 3) r += sqrtg * src[v - 1];
      if (v == 4) r += sqrtg * srcT;
      if (v >= 5) r -= sqrtg * sb[v - 5];
      emit(24 + v, r, u[v]);
    }
    if (pp.glm) {  // d_t psi = -c_h^2 d_i(sqrt(gamma) B^i) / sqrt(gamma) - psi / tau
      const double divB = (LS(O_GLM) + LS(O_GLM + 1) + LS(O_GLM + 2)) * isg;
      const double psi = LU(32);
      emit(32, -pp.ch2 * divB - psi * pp.itau, psi);
    }
  }
  mt.Str = Str;
  return mt;
#undef LS
#undef LU
}

// LDS slots per thread of the RHS kernel (values parked across the Ricci
// tensor): E, trace of S^i_j, S_j (3), S_ij (6), beta^i (3), d_a alpha (3),
// d_a K (3), d_a beta^i (9).
constexpr int RHS_PARK = 29;

// MODE: the stage mode as a compile-time constant, so that every update is
// straight-line code and the loads of Un and the accumulator can issue early.
template <typename DT, int MODE, bool NA = (MODE != 5)>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_rhs_rk(
                                                maybe_restrict<NA, const double> Us,
                                                const DT* __restrict__ der,
                                                const double* __restrict__ prim,
                                                const double* __restrict__ K0p,
                                                maybe_restrict<NA, const double> Un,
                                                maybe_restrict<NA, double> acc, maybe_restrict<NA, double> out,
                                                PointParams pp, JobSet js) {
  constexpr int mode = MODE;
  const long long P = pp.P;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= P) return;
  const double dt = js.dt[blockIdx.y];
  {  // this job's buffers
    const long long jd = js.d[blockIdx.y];
    Us = shift_ptr(Us, jd);
    der = shift_ptr(der, jd);
    prim = shift_ptr(prim, jd);
    K0p = shift_ptr(K0p, jd);
    Un = shift_ptr(Un, jd);
    acc = shift_ptr(acc, jd);
    out = shift_ptr(out, jd);
  }
  const int j = (int)(idx % pp.nr);
  const int k = (int)((idx / pp.nr) % pp.nth);
  const bool frozen = (j == 0 || k == 0 || k == pp.nth - 1);
#define LU(f) Us[(size_t)(f) * P + idx]
#define LS(g) ((double)ldnt(&der[(size_t)(g) * P + idx]))
#define D1(a, f) LS(21 * (a) + (f))
  auto DD = [&](int a, int b, int s) -> double {
    if (a == b) return LS(O_D2 + 11 * a + s);
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const int m = (lo == 0) ? (hi == 1 ? 0 : 1) : 2;
    return LS(O_MX + 11 * m + s);
  };
  // classic RK4 stage update of field f with right-hand side kf; the
  // accumulator holds Un + dt sum_s b_s k_s, so the last stage does not read Un
  // mode 0: out = k; 1 (Us is Un, read once): acc = Un + dt/6 k, out = Un + dt/2 k;
  // 2: acc += dt/3 k, out = Un + dt/2 k; 3: acc += dt/3 k, out = Un + dt k;
  // 4: out = acc + dt/6 k; 5 (split step): forward Euler out = Un + dt k of the
  // 24 spacetime fields only, the matter fields are not written
  // us: the stage value of field f (held in a register where the right-hand
  // side already read it; stage 1 takes it as U^n instead of reading U^n again)
  auto emit = [&](int f, double kf, double us) {
    // kf is formed on every lane: otherwise the compiler moves its loads
    // into a branch over the non-frozen lanes, behind the stores before it
    __asm__ __volatile__("" : "+v"(kf));
    if (frozen || (pp.cowling && f < 24)) kf = 0.0;  // Cowling: fixed spacetime
    const size_t e = (size_t)f * P + idx;
    if (mode == 0) {
      out[e] = kf;
    } else if (mode == 5) {
      if (f < 24) out[e] = ldnt(&Un[e]) + dt * kf;
    } else if (mode == 1) {
      const double un = us;  // stage 1 is evaluated at U^n
      acc[e] = un + (dt / 6.0) * kf;
      out[e] = un + 0.5 * dt * kf;
    } else if (mode == 2) {
      acc[e] = ldnt(&acc[e]) + (dt / 3.0) * kf;
      out[e] = ldnt(&Un[e]) + 0.5 * dt * kf;
    } else if (mode == 3) {
      acc[e] = ldnt(&acc[e]) + (dt / 3.0) * kf;
      out[e] = ldnt(&Un[e]) + dt * kf;
    } else {
      out[e] = ldnt(&acc[e]) + (dt / 6.0) * kf;
    }
  };

  // ---- phase 1: conformal metric, gauge, first derivatives ---------------------
  const double phi = LU(0);
  Sym gt, At;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    gt.m[s] = LU(1 + s);
    At.m[s] = LU(7 + s);
  }
  const double K = LU(13);
  const double alpha = LU(17);
  double beta[3] = {LU(18), LU(19), LU(20)};
  const double K0 = K0p[idx];
  const double detgt = det_sym(gt);
  const Sym gtu = inv_sym(gt, detgt);
  const double e4 = exp(4.0 * phi), em4 = 1.0 / e4;
  const double sqrtg = e4 * exp(2.0 * phi) * sqrt(detgt);
  double dphi[3], dal[3], dK[3], dbeta[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dphi[a] = D1(a, 0);
    dal[a] = D1(a, 17);
    dK[a] = D1(a, 13);
#pragma unroll
    for (int i = 0; i < 3; ++i) dbeta[a][i] = D1(a, 18 + i);
  }
  const double divb = dbeta[0][0] + dbeta[1][1] + dbeta[2][2];
  PHASE();

  // ---- phase 2: Christoffels; phi, gt_ij, alpha, beta right-hand sides ---------
  double Gl[3][6], Gu[3][6], Gd[3];
  double dgt[3][6];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int s = 0; s < 6; ++s) dgt[a][s] = D1(a, 1 + s);
  christoffel(gtu, dgt, Gl, Gu, Gd);
  emit(0, -alpha * K / 6.0 + dot3(beta, dphi) + divb / 6.0, phi);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = i; jj < 3; ++jj) {
      const int s = S6(i, jj);
      double lie = 0.0;
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) lie += gt(i, kk) * dbeta[jj][kk] + gt(jj, kk) * dbeta[i][kk];
      const double adv = beta[0] * dgt[0][s] + beta[1] * dgt[1][s] + beta[2] * dgt[2][s];
      emit(1 + s, -2.0 * alpha * At.m[s] + adv + lie - (2.0 / 3.0) * gt.m[s] * divb, gt.m[s]);
    }
  emit(17, dot3(beta, dal) - 2.0 * alpha * (pp.gauge_k0 ? (K - K0) : K), alpha);
  {
    const double Bd[3] = {LU(21), LU(22), LU(23)};
#pragma unroll
    for (int i = 0; i < 3; ++i) emit(18 + i, 0.75 * Bd[i], beta[i]);
  }
  PHASE();

  // ---- phase 3: matter; Valencia right-hand sides ------------------------------
  // Values needed after the Ricci tensor wait in LDS (one slot per thread)
  // while it is formed: the matter terms and the shift and lapse and K
  // derivatives.  In registers they would make the kernel spill at two waves
  // per SIMD; the LDS is otherwise unused.
  __shared__ double park[RHS_PARK][256];
  double* const pk = &park[0][threadIdx.x];  // slot q at pk[256 q]
  {
    const Matter m3 = valencia_rhs(Us, der, prim, idx, P, pp, sqrtg, e4, em4, gt, gtu, At, K, alpha, dal, dbeta,
                                   dgt, dphi, emit);
    pk[0] = m3.Em;
    pk[256] = m3.Str;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      pk[256 * (2 + q)] = m3.Sl[q];
      pk[256 * (11 + q)] = beta[q];
      pk[256 * (14 + q)] = dal[q];
      pk[256 * (17 + q)] = dK[q];
#pragma unroll
      for (int r = 0; r < 3; ++r) pk[256 * (20 + 3 * q + r)] = dbeta[q][r];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) pk[256 * (5 + q)] = m3.Sij.m[q];
  }
  PHASE();

  // ---- phase 4: conformal Ricci tensor -------------------------------------------
  double dGt[3][3];  // [a][i] = d_a Gt^i
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int i = 0; i < 3; ++i) dGt[a][i] = D1(a, 14 + i);
  Sym R;
  ricci(gt, gtu, Gl, Gu, Gd, dGt, dphi, DD, R);
  PHASE();
  Matter mt;
  mt.Em = pk[0];
  mt.Str = pk[256];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    mt.Sl[q] = pk[256 * (2 + q)];
    beta[q] = pk[256 * (11 + q)];
    dal[q] = pk[256 * (14 + q)];
    dK[q] = pk[256 * (17 + q)];
#pragma unroll
    for (int r = 0; r < 3; ++r) dbeta[q][r] = pk[256 * (20 + 3 * q + r)];
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) mt.Sij.m[q] = pk[256 * (5 + q)];
  const double Em = mt.Em;
  const double* Sl = mt.Sl;
  const Sym& Sij = mt.Sij;
  const double Str = mt.Str;

  // ---- phase 5: D_i D_j alpha, A-tilde contractions, K and A-tilde -------------
  double DDa[6];
  {
    double dphiu[3];
    mv(gtu, dphi, dphiu);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int jj = i; jj < 3; ++jj) {
        const int s = S6(i, jj);
        double t = DD(i, jj, 7);
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          const double Gp = Gu[kk][s] + 2.0 * ((kk == i ? dphi[jj] : 0.0) + (kk == jj ? dphi[i] : 0.0) -
                                               gt.m[s] * dphiu[kk]);
          t -= Gp * dal[kk];
        }
        DDa[s] = t;
      }
  }
  double trDDa = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int m = 0; m < 3; ++m) trDDa += gtu(l, m) * DDa[S6(l, m)];
  trDDa *= em4;
  double Amix[3][3];  // A_ik gt^kl
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int l = 0; l < 3; ++l) Amix[i][l] = At(i, 0) * gtu(0, l) + At(i, 1) * gtu(1, l) + At(i, 2) * gtu(2, l);
  Sym Atu;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = i; jj < 3; ++jj)
      Atu.m[S6(i, jj)] = gtu(i, 0) * Amix[0][jj] + gtu(i, 1) * Amix[1][jj] + gtu(i, 2) * Amix[2][jj];
  double AA = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) AA += At(i, jj) * Atu(i, jj);
  emit(13, -trDDa + alpha * (AA + K * K / 3.0) + 4.0 * PI * alpha * (Em + Str) + dot3(beta, dK), K);
  {
    double X[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) X[s] = -DDa[s] + alpha * (R.m[s] - 8.0 * PI * Sij.m[s]);
    double trX = 0.0;
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
      for (int m = 0; m < 3; ++m) trX += gtu(l, m) * X[S6(l, m)];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int jj = i; jj < 3; ++jj) {
        const int s = S6(i, jj);
        const double AAij = At(i, 0) * Amix[jj][0] + At(i, 1) * Amix[jj][1] + At(i, 2) * Amix[jj][2];
        double lie = 0.0, adv = 0.0;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          lie += At(i, kk) * dbeta[jj][kk] + At(jj, kk) * dbeta[i][kk];
          adv += beta[kk] * D1(kk, 7 + s);
        }
        emit(7 + s, em4 * (X[s] - gt.m[s] * trX / 3.0) + alpha * (K * At.m[s] - 2.0 * AAij) + adv + lie -
                        (2.0 / 3.0) * At.m[s] * divb,
             At.m[s]);
      }
  }
  PHASE();

  // ---- phase 6: Gamma-tilde and the Gamma-driver ---------------------------------
  // d_j d_k beta^i (symmetric pair S6(j, k)), each array read once, and
  // d_j d_k beta^k
  double ddb[3][6], ddivb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj)
#pragma unroll
      for (int kk = jj; kk < 3; ++kk) ddb[i][S6(jj, kk)] = DD(jj, kk, 8 + i);
#pragma unroll
  for (int jj = 0; jj < 3; ++jj) ddivb[jj] = ddb[0][S6(jj, 0)] + ddb[1][S6(jj, 1)] + ddb[2][S6(jj, 2)];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double t = 0.0;
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      t += -2.0 * Atu(i, jj) * dal[jj];
      t += 2.0 * alpha * (6.0 * Atu(i, jj) * dphi[jj] - (2.0 / 3.0) * gtu(i, jj) * dK[jj]);
      t += -16.0 * PI * alpha * gtu(i, jj) * Sl[jj];
      t += beta[jj] * dGt[jj][i] - Gd[jj] * dbeta[jj][i];
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        t += 2.0 * alpha * Gu[i][S6(jj, kk)] * Atu(jj, kk);
        t += gtu(jj, kk) * ddb[i][S6(jj, kk)];
      }
      t += gtu(i, jj) * ddivb[jj] / 3.0;
    }
    const double rGt = t + (2.0 / 3.0) * Gd[i] * divb;
    emit(14 + i, rGt, LU(14 + i));
    const double bd = LU(21 + i);
    emit(21 + i, rGt - pp.eta * bd, bd);
  }
#undef D1
#undef LS
#undef LU
}
#undef PHASE

// ---------------------------------------------------------------------------
// Fixed-background (Cowling) form: right-hand sides and RK4 stage update of
// the GRMHD fields (and psi) only.  The geometry comes from the fixed
// background state Ug (phi, gt_ij, A-tilde_ij, K, alpha) and its first
// derivatives bg (d_a of background field s at 11 a + s, s = phi, gt_ij, alpha,
// beta^i); the fluid from the stage state Us.  Mode 0 also writes zero
// right-hand sides for the 24 spacetime fields.  Stage modes as in k_rhs_rk,
// with the same promise on the buffers (Ug may be U^n: the background fields
// it supplies are never written here).
template <typename DT, int MODE>
__global__ __launch_bounds__(256) void k_rhs_fixed(const double* __restrict__ Us,
                                                   const double* __restrict__ Ug, const double* __restrict__ bg,
                                                   const DT* __restrict__ der, const double* __restrict__ prim,
                                                   const double* __restrict__ Un, double* __restrict__ acc,
                                                   double* __restrict__ out, PointParams pp, JobSet js) {
  const long long P = pp.P;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= P) return;
  const double dt = js.dt[blockIdx.y];
  {  // this job's buffers
    const long long jd = js.d[blockIdx.y];
    Us = shift_ptr(Us, jd);
    Ug = shift_ptr(Ug, jd);
    bg = shift_ptr(bg, jd);
    der = shift_ptr(der, jd);
    prim = shift_ptr(prim, jd);
    Un = shift_ptr(Un, jd);
    acc = shift_ptr(acc, jd);
    out = shift_ptr(out, jd);
  }
  const int j = (int)(idx % pp.nr);
  const int k = (int)((idx / pp.nr) % pp.nth);
  const bool frozen = (j == 0 || k == 0 || k == pp.nth - 1);
  constexpr int mode = MODE;
  auto emit = [&](int f, double kf, double us) {
    __asm__ __volatile__("" : "+v"(kf));  // formed on every lane, as in k_rhs_rk
    if (frozen) kf = 0.0;
    const size_t e = (size_t)f * P + idx;
    if (mode == 0) {
      out[e] = kf;
    } else if (mode == 1) {
      const double un = us;  // stage 1 is evaluated at U^n
      acc[e] = un + (dt / 6.0) * kf;
      out[e] = un + 0.5 * dt * kf;
    } else if (mode == 2) {
      acc[e] = ldnt(&acc[e]) + (dt / 3.0) * kf;
      out[e] = ldnt(&Un[e]) + 0.5 * dt * kf;
    } else if (mode == 3) {
      acc[e] = ldnt(&acc[e]) + (dt / 3.0) * kf;
      out[e] = ldnt(&Un[e]) + dt * kf;
    } else {
      out[e] = ldnt(&acc[e]) + (dt / 6.0) * kf;
    }
  };
  if (mode == 0)
    for (int f = 0; f < 24; ++f) out[(size_t)f * P + idx] = 0.0;
#define LG(f) ldnt(&Ug[(size_t)(f) * P + idx])
#define BG(a, s) ldnt(&bg[(size_t)(11 * (a) + (s)) * P + idx])
  const double phi = LG(0);
  Sym gt, At;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    gt.m[s] = LG(1 + s);
    At.m[s] = LG(7 + s);
  }
  const double K = LG(13);
  const double alpha = LG(17);
  const double detgt = det_sym(gt);
  const Sym gtu = inv_sym(gt, detgt);
  const double e4 = exp(4.0 * phi), em4 = 1.0 / e4;
  const double sqrtg = e4 * exp(2.0 * phi) * sqrt(detgt);
  double dphi[3], dal[3], dbeta[3][3], dgt[3][6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dphi[a] = BG(a, 0);
#pragma unroll
    for (int q = 0; q < 6; ++q) dgt[a][q] = BG(a, 1 + q);
    dal[a] = BG(a, 7);
#pragma unroll
    for (int i = 0; i < 3; ++i) dbeta[a][i] = BG(a, 8 + i);
  }
#undef BG
#undef LG
  (void)valencia_rhs(Us, der, prim, idx, P, pp, sqrtg, e4, em4, gt, gtu, At, K, alpha, dal, dbeta, dgt, dphi,
                     emit);
}

// ---------------------------------------------------------------------------
// Constraints from FP64 derivative arrays:
//   Hamiltonian H = e^{-4 phi} gt^ij R_ij + 2/3 K^2 - A_ij A^ij - 16 pi E, E = tau + D;
//   momentum    M_i = Dt_j A^j_i + 6 A^j_i d_j phi - 2/3 d_i K - 8 pi S_i
//               (A^j_i = gt^jk At_ki, Dt the covariant derivative of gt,
//               S_i the undensitised momentum), written as its norm
//               |M| = sqrt(e^{-4 phi} gt^ij M_i M_j).
__global__ __launch_bounds__(256) void k_ham(const double* __restrict__ U, const double* __restrict__ der,
                                             double* __restrict__ H, double* __restrict__ Mn, PointParams pp) {
  const long long P = pp.P;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= P) return;
#define LU(f) U[(size_t)(f) * P + idx]
#define LS(g) der[(size_t)(g) * P + idx]
  auto DD = [&](int a, int b, int s) -> double {
    if (a == b) return LS(O_D2 + 11 * a + s);
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const int m = (lo == 0) ? (hi == 1 ? 0 : 1) : 2;
    return LS(O_MX + 11 * m + s);
  };
  const double phi = LU(0);
  Sym gt, At;
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    gt.m[s] = LU(1 + s);
    At.m[s] = LU(7 + s);
  }
  const double K = LU(13);
  const double detgt = det_sym(gt);
  const Sym gtu = inv_sym(gt, detgt);
  const double em4 = exp(-4.0 * phi);
  const double sqrtg = exp(6.0 * phi) * sqrt(detgt);
  double dgt[3][6], dphi[3], dGt[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dphi[a] = LS(21 * a);
#pragma unroll
    for (int s2 = 0; s2 < 6; ++s2) dgt[a][s2] = LS(21 * a + 1 + s2);
#pragma unroll
    for (int i = 0; i < 3; ++i) dGt[a][i] = LS(21 * a + 14 + i);
  }
  double Gl[3][6], Gu[3][6], Gd[3];
  christoffel(gtu, dgt, Gl, Gu, Gd);
  Sym R;
  ricci(gt, gtu, Gl, Gu, Gd, dGt, dphi, DD, R);
  double trR = 0.0, AA = 0.0;
  double Amix[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int l = 0; l < 3; ++l) Amix[i][l] = At(i, 0) * gtu(0, l) + At(i, 1) * gtu(1, l) + At(i, 2) * gtu(2, l);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int jj = 0; jj < 3; ++jj) {
      trR += gtu(i, jj) * R(i, jj);
      AA += Amix[i][jj] * Amix[jj][i];
    }
  const double E = (LU(28) + LU(24)) / sqrtg;
  H[idx] = em4 * trR + (2.0 / 3.0) * K * K - AA - 16.0 * PI * E;
  // momentum constraint: d_j A^j_i = (d_j gt^jk) At_ki + gt^jk d_j At_ki with
  // d_j gt^jk = -gt^kb (gt^ja d_j gt_ab)
  double w[3], v[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int a = 0; a < 3; ++a) t += gtu(j, a) * dgt[j][S6(a, b)];
    w[b] = t;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = -(gtu(k, 0) * w[0] + gtu(k, 1) * w[1] + gtu(k, 2) * w[2]);
  double trG[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) trG[k] = Gu[0][S6(0, k)] + Gu[1][S6(1, k)] + Gu[2][S6(2, k)];
  // A^j_i = Amix[i][j] (At and gt^-1 symmetric)
  double Mi[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) m += v[k] * At(k, i) + trG[k] * Amix[i][k];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
#pragma unroll
      for (int k = 0; k < 3; ++k) m += gtu(j, k) * LS(21 * j + 7 + S6(k, i)) - Gu[k][S6(j, i)] * Amix[k][j];
      m += 6.0 * Amix[i][j] * dphi[j];
    }
    Mi[i] = m - (2.0 / 3.0) * LS(21 * i + 13) - 8.0 * PI * LU(25 + i) / sqrtg;
  }
  double mm = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) mm += gtu(i, j) * Mi[i] * Mi[j];
  Mn[idx] = sqrt(em4 * mm);
#undef LS
#undef LU
}

// ---------------------------------------------------------------------------
// Initial state from the (theta, r) plane fields (see launch_init_expand).
__device__ __forceinline__ uint64_t splitmix64_dev(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_init_expand(const double* __restrict__ pl, int torus, uint64_t seed,
                                                     double amp, double G, PointParams pp, double* __restrict__ U,
                                                     double* __restrict__ K0) {
  const long long P = pp.P;
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= P) return;
  const long long PL = (long long)pp.nr * pp.nth;
  const long long e = n % PL;
#define PLF(f) pl[(size_t)(f) * PL + e]
  U[n] = PLF(PL_PHI);
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    U[(size_t)(1 + s) * P + n] = PLF(PL_GT + s);
    U[(size_t)(7 + s) * P + n] = PLF(PL_AT + s);
  }
  U[(size_t)13 * P + n] = PLF(PL_K);
#pragma unroll
  for (int i = 0; i < 3; ++i) U[(size_t)(14 + i) * P + n] = PLF(PL_GAMT + i);
  U[(size_t)17 * P + n] = PLF(PL_ALPHA);
  U[(size_t)18 * P + n] = PLF(PL_BETAR);
#pragma unroll
  for (int f = 19; f < 24; ++f) U[(size_t)f * P + n] = 0.0;
  K0[n] = PLF(PL_K0);
  double rho = PLF(PL_RHO), p = PLF(PL_P);
  if (amp != 0.0) {
    const double u = (double)(splitmix64_dev(seed ^ (uint64_t)n) >> 11) * 0x1.0p-53;
    if (torus)
      p = p * (1.0 + amp * (2.0 * u - 1.0));
    else
      rho = rho * (1.0 + amp * (2.0 * u - 1.0));
  }
  const double sg = PLF(PL_SQRTG);
  double gm[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) gm[c] = PLF(PL_GM + c);
  const double v[3] = {PLF(PL_V), PLF(PL_V + 1), PLF(PL_V + 2)};
  const double sB[3] = {PLF(PL_SB), PLF(PL_SB + 1), PLF(PL_SB + 2)};
#undef PLF
  const double Bu[3] = {sB[0] / sg, sB[1] / sg, sB[2] / sg};
  double vl[3], Bl[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    vl[i] = gm[i * 3 + 0] * v[0] + gm[i * 3 + 1] * v[1] + gm[i * 3 + 2] * v[2];
    Bl[i] = gm[i * 3 + 0] * Bu[0] + gm[i * 3 + 1] * Bu[1] + gm[i * 3 + 2] * Bu[2];
  }
  const double v2 = v[0] * vl[0] + v[1] * vl[1] + v[2] * vl[2];
  const double W = 1.0 / sqrt(1.0 - v2);
  const double Bv = Bu[0] * vl[0] + Bu[1] * vl[1] + Bu[2] * vl[2];
  const double B2 = Bu[0] * Bl[0] + Bu[1] * Bl[1] + Bu[2] * Bl[2];
  const double h = 1.0 + p / rho * G / (G - 1.0);
  const double Z = rho * h * W * W;
  const double D = rho * W;
  const double tau = Z - p + B2 - 0.5 * (B2 / (W * W) + Bv * Bv) - D;
  U[(size_t)24 * P + n] = sg * D;
#pragma unroll
  for (int i = 0; i < 3; ++i) U[(size_t)(25 + i) * P + n] = sg * ((Z + B2) * vl[i] - Bv * Bl[i]);
  U[(size_t)28 * P + n] = sg * tau;
#pragma unroll
  for (int i = 0; i < 3; ++i) U[(size_t)(29 + i) * P + n] = sB[i];
}

__global__ __launch_bounds__(256) void k_k0(const double* __restrict__ U, const double* __restrict__ scr,
                                            double* __restrict__ K0, long long P) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= P) return;
  const double alpha = U[17 * (size_t)P + idx];
  double adv = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) adv += U[(size_t)(18 + a) * P + idx] * scr[(size_t)(SC_D1 + 21 * a + 17) * P + idx];
  K0[idx] = U[13 * (size_t)P + idx] - adv / (2.0 * alpha);
}

// ---------------------------------------------------------------------------
// Diagnostics partials per block, DIAG_Q values per block: [0] sum sqrt(g) D w,
// [1] sum rho s sqrt(g) w, [2] fails, [3] non-finite count, [4] max |div B|
// (scratch first-derivative slots of sqrt(g) B^a), [5] min alpha, [6] max W,
// [7] sum H^2 w, [8] max |H|, [9] sum w, [10] sum |M|^2 w, [11] max |M|.
// Each thread accumulates a grid-stride set of points; each wavefront then
// reduces its 64 lanes with cross-lane swizzles (xor butterfly within each
// half-wave, then the two halves read from lanes 0 and 32), the four
// wavefronts of a block are combined in a fixed order by one thread, and the
// host adds the block partials in block order.  No floating-point atomics: the
// result is the same on every run and for a job alone or in a batch.
constexpr int DIAG_THREADS = 256;

// Max / min that keep a NaN operand (fmax/fmin drop it), so that a state gone
// non-finite never reports a finite extremum.
__device__ __forceinline__ double nan_max(double a, double b) { return (a != a || a > b) ? a : b; }
__device__ __forceinline__ double nan_min(double a, double b) { return (a != a || a < b) ? a : b; }

// The value of lane (l xor MASK) within each 32-lane half (ds_swizzle bit
// mode: and-mask 0x1f, or-mask 0, xor-mask MASK).
template <int MASK>
__device__ __forceinline__ double swizzle_xor(double v) {
  static_assert(MASK > 0 && MASK < 32, "xor mask within a half-wave");
  constexpr int pattern = (MASK << 10) | 0x1f;
  const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), pattern);
  const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), pattern);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Reduction of one value over the 64 lanes of a wavefront (all lanes
// active); op is commutative, so both lanes of a pair hold the same value.
template <class Op>
__device__ __forceinline__ double wave_reduce(double v, Op op) {
  v = op(v, swizzle_xor<1>(v));
  v = op(v, swizzle_xor<2>(v));
  v = op(v, swizzle_xor<4>(v));
  v = op(v, swizzle_xor<8>(v));
  v = op(v, swizzle_xor<16>(v));
  return op(read_lane(v, 0), read_lane(v, 32));
}

__global__ __launch_bounds__(DIAG_THREADS) void k_diag(const double* __restrict__ U,
                                                       const double* __restrict__ prim,
                                                       const double* __restrict__ fail,
                                                       const double* __restrict__ scr,
                                                       const double* __restrict__ H,
                                                       const double* __restrict__ Mn,
                                                       const double* __restrict__ wr,
                                                       const double* __restrict__ wth, double G,
                                                       PointParams pp, double* __restrict__ partials) {
  constexpr int NW = DIAG_THREADS / 64;
  __shared__ double sh[NW][DIAG_Q];
  const long long P = pp.P;
  double v[DIAG_Q] = {0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long idx = (long long)blockIdx.x * DIAG_THREADS + threadIdx.x; idx < P;
       idx += (long long)gridDim.x * DIAG_THREADS) {
    const int j = (int)(idx % pp.nr), k = (int)((idx / pp.nr) % pp.nth);
    const double w = wr[j] * wth[k] * (2.0 * PI / pp.nph);
    Sym gt;
    for (int s = 0; s < 6; ++s) gt.m[s] = U[(size_t)(1 + s) * P + idx];
    const double phi = U[idx];
    const double sqrtg = exp(6.0 * phi) * sqrt(det_sym(gt));
    const double rho = prim[idx], p = prim[(size_t)P + idx];
    v[0] += U[(size_t)24 * P + idx] * w;
    v[1] += rho * log(p / pow(rho, G)) / (G - 1.0) * sqrtg * w;
    v[2] += fail[idx];
    int nf = 0;
    for (int f = 0; f < (pp.glm ? NFA : 32); ++f) nf += !isfinite(U[(size_t)f * P + idx]);
    v[3] += nf;
    const double dB = scr[(size_t)(SC_D1 + 0) * P + idx] + scr[(size_t)(SC_D1 + 21 + 1) * P + idx] +
                      scr[(size_t)(SC_D1 + 42 + 2) * P + idx];
    v[4] = nan_max(v[4], fabs(dB));
    v[5] = nan_min(v[5], U[(size_t)17 * P + idx]);
    const double e4 = exp(4.0 * phi);
    Sym gam;
    for (int s = 0; s < 6; ++s) gam.m[s] = e4 * gt.m[s];
    double vv[3] = {prim[2 * (size_t)P + idx], prim[3 * (size_t)P + idx], prim[4 * (size_t)P + idx]}, vl[3];
    mv(gam, vv, vl);
    v[6] = nan_max(v[6], 1.0 / sqrt(1.0 - dot3(vv, vl)));
    const double h = H[idx];
    v[7] += h * h * w;
    v[8] = nan_max(v[8], fabs(h));
    v[9] += w;
    const double m = Mn[idx];
    v[10] += m * m * w;
    v[11] = nan_max(v[11], m);
  }
  auto add = [](double a, double b) { return a + b; };
  auto mx = [](double a, double b) { return nan_max(a, b); };
  auto mn = [](double a, double b) { return nan_min(a, b); };
  double r[DIAG_Q];
#pragma unroll
  for (int q = 0; q < DIAG_Q; ++q) {
    if (q == 5) r[q] = wave_reduce(v[q], mn);
    else if (q == 4 || q == 6 || q == 8 || q == 11) r[q] = wave_reduce(v[q], mx);
    else r[q] = wave_reduce(v[q], add);
  }
  const int wave = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < DIAG_Q; ++q) sh[wave][q] = r[q];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < DIAG_Q; ++q) {
      double t = sh[0][q];
      for (int w2 = 1; w2 < NW; ++w2) {
        const double u = sh[w2][q];
        t = (q == 5) ? nan_min(t, u) : (q == 4 || q == 6 || q == 8 || q == 11) ? nan_max(t, u) : t + u;
      }
      partials[(size_t)blockIdx.x * DIAG_Q + q] = t;
    }
}

// ---------------------------------------------------------------------------
static inline unsigned nblk(long long P) { return (unsigned)((P + 255) / 256); }

hipError_t launch_c2p_flux(const double* U, const double* Ug, double* prim, double* fail, double* flux,
                           const double* floors, const PointParams& pp, const JobSet& js, hipStream_t s) {
  if (js.n < 1 || js.n > MAXB) return hipErrorInvalidValue;
  if (pp.c2p_damped)
    hipLaunchKernelGGL(k_c2p_flux<true>, dim3(nblk(pp.P), js.n), dim3(256), 0, s, U, Ug, prim, fail, flux, floors,
                       pp, js);
  else
    hipLaunchKernelGGL(k_c2p_flux<false>, dim3(nblk(pp.P), js.n), dim3(256), 0, s, U, Ug, prim, fail, flux, floors,
                       pp, js);
  return hipGetLastError();
}

hipError_t launch_rhs_rk(int mode, bool der_f32, const double* Us, const void* der, const double* prim,
                         const double* K0, const double* Un, double* acc, double* out, const PointParams& pp,
                         const JobSet& js, hipStream_t s) {
  if (mode < 0 || mode > 5 || js.n < 1 || js.n > MAXB) return hipErrorInvalidValue;
#define RKM(T, M)                                                                                          \
  hipLaunchKernelGGL((k_rhs_rk<T, M>), dim3(nblk(pp.P), js.n), dim3(256), 0, s, Us, (const T*)der, prim, K0, \
                     Un, acc, out, pp, js)
#define RKT(T)                  \
  switch (mode) {               \
    case 0: RKM(T, 0); break;   \
    case 1: RKM(T, 1); break;   \
    case 2: RKM(T, 2); break;   \
    case 3: RKM(T, 3); break;   \
    case 4: RKM(T, 4); break;   \
    default: RKM(T, 5); break;  \
  }
  if (der_f32) {
    RKT(float)
  } else {
    RKT(double)
  }
#undef RKT
#undef RKM
  return hipGetLastError();
}

hipError_t launch_rhs_fixed(int mode, bool der_f32, const double* Us, const double* Ug, const double* bg,
                            const void* der, const double* prim, const double* Un, double* acc, double* out,
                            const PointParams& pp, const JobSet& js, hipStream_t s) {
  if (mode < 0 || mode > 4 || js.n < 1 || js.n > MAXB) return hipErrorInvalidValue;
#define RFM(T, M)                                                                                        \
  hipLaunchKernelGGL((k_rhs_fixed<T, M>), dim3(nblk(pp.P), js.n), dim3(256), 0, s, Us, Ug, bg, (const T*)der, \
                     prim, Un, acc, out, pp, js)
#define RFT(T)                 \
  switch (mode) {              \
    case 0: RFM(T, 0); break;  \
    case 1: RFM(T, 1); break;  \
    case 2: RFM(T, 2); break;  \
    case 3: RFM(T, 3); break;  \
    default: RFM(T, 4); break; \
  }
  if (der_f32) {
    RFT(float)
  } else {
    RFT(double)
  }
#undef RFT
#undef RFM
  return hipGetLastError();
}

hipError_t launch_ham(const double* U, const double* der, double* H, double* Mn, const PointParams& pp,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_ham, dim3(nblk(pp.P)), dim3(256), 0, s, U, der, H, Mn, pp);
  return hipGetLastError();
}

hipError_t launch_k0(const double* U, const double* scr, double* K0, const PointParams& pp,
                     hipStream_t s) {
  hipLaunchKernelGGL(k_k0, dim3(nblk(pp.P)), dim3(256), 0, s, U, scr, K0, pp.P);
  return hipGetLastError();
}

hipError_t launch_init_expand(const double* plane, int torus, uint64_t seed, double amp, double gamma_ad,
                              const PointParams& pp, double* U, double* K0, hipStream_t s) {
  hipLaunchKernelGGL(k_init_expand, dim3(nblk(pp.P)), dim3(256), 0, s, plane, torus, seed, amp, gamma_ad, pp, U,
                     K0);
  return hipGetLastError();
}

int diag_partials_blocks(long long P) {
  long long b = (P + DIAG_THREADS - 1) / DIAG_THREADS;
  return (int)(b < 1024 ? b : 1024);
}

hipError_t launch_diag_partials(const double* U, const double* prim, const double* fail,
                                const double* scr, const double* H, const double* Mn, const double* wr,
                                const double* wth, double gamma_ad, const PointParams& pp, double* partials,
                                int* nblocks, hipStream_t s) {
  const int nb = diag_partials_blocks(pp.P);
  *nblocks = nb;
  hipLaunchKernelGGL(k_diag, dim3(nb), dim3(DIAG_THREADS), 0, s, U, prim, fail, scr, H, Mn, wr, wth, gamma_ad,
                     pp, partials);
  return hipGetLastError();
}

}  // namespace grmhd
