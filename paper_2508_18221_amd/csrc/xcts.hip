// Conformally flat, time-symmetric initial data (Methods, "Initial Data:
// Approximate XCTS Solution"): the conformal factor psi of gamma_ij = psi^4 f_ij
// (f flat, A_ij = 0, K = 0) from the Hamiltonian constraint
//     Lap psi = -2 pi E psi^5,
// by fixed-point relaxation: each iteration solves the linear problem
// Lap psi_{k+1} = -2 pi E psi_k^5 with the boundary values of the initial
// guess held (Dirichlet on the r ends and the theta ends, phi periodic).
//
// The linear solve is a fast diagonalisation.  Multiplied by r^2 the flat
// Laplacian on the log-mapped Chebyshev(r) x Chebyshev(theta) x Fourier(phi)
// grid separates:
//     r^2 Lap = A_r (x) 1 + 1 (x) B_m,
//     A_r = (D_xx + Lh D_x) / Lh^2                          (radial, constant coefficients)
//     B_m = D_yy / Th^2 + cot(theta) D_y / Th - m^2 / sin^2(theta)   (polar, per Fourier mode m)
// after a real discrete Fourier transform along phi (cos / sin pairs; the
// collocation phi-phi derivative is -m^2 on mode m, the Nyquist mode
// included).  With A_r = V_r L_r V_r^{-1} and B_m = V_m L_m V_m^{-1} on the
// interior nodes (host eigen-decompositions, eig.h), the interior solution of
// r^2 Lap u = q, u = 0 on the boundary, is
//     u = V_m V_r [(V_m^{-1} V_r^{-1} q) / (lam_r + lam_m)],
// a sequence of dense transforms along grid lines and one pointwise division.
// With u = psi_{k+1} - psi_0 and g_0 = r^2 Lap psi_0 (once per solve), each
// iteration takes q = -2 pi r^2 E psi_k^5 - g_0 through: the forward phi
// transform, the polar and radial inverse eigenvector transforms, the
// division, the radial and polar eigenvector transforms, the inverse phi
// transform, then psi_{k+1} = psi_0 + u and the largest change (block maxima,
// host maximum) for the stopping test.
//
// The line transforms run as one thread per output node (a dot product over
// the line, operators from L2): this is set-up work, not the timed stage.
#include <math.h>

#include <string>
#include <vector>

#include "eig.h"
#include "grmhd_internal.h"

namespace grmhd {

namespace {

constexpr double PI = 3.14159265358979323846;
constexpr int XT = 256;  // threads per block

// A dense operator along one axis of the [phi][theta][r] grid, applied on the
// index range [lo, lo + n) of that axis (input and output); outputs outside
// the range are set to zero, or left alone when accumulating.  On the theta
// axis the operator may depend on the Fourier slot l of a phi-transformed
// array: slot l holds mode m = (l + 1) / 2 (0; cos 1, sin 1; cos 2, ...;
// the Nyquist cosine last) and its operator is M + m * mstride.
struct LineOp {
  int axis;
  int lo, n;
  const double* M;     // n x n, row-major: out[i] = sum_t M[i][t] in[lo + t]
  long long mstride;   // theta axis: operator stride per Fourier mode (0: one operator)
  int accumulate;      // 1: out += result (outside the range: unchanged)
};

__global__ __launch_bounds__(XT) void k_line(const double* __restrict__ in, double* __restrict__ out, LineOp op,
                                             int nr, int nth, int nph) {
  const long long P = (long long)nr * nth * nph;
  const long long idx = (long long)blockIdx.x * XT + threadIdx.x;
  if (idx >= P) return;
  const int j = (int)(idx % nr), k = (int)((idx / nr) % nth), l = (int)(idx / ((long long)nr * nth));
  int a;
  long long stride, base;
  const double* M = op.M;
  if (op.axis == 0) {
    a = j;
    stride = 1;
    base = idx - j;
  } else if (op.axis == 1) {
    a = k;
    stride = nr;
    base = idx - (long long)k * nr;
    M += (long long)((l + 1) / 2) * op.mstride;
  } else {
    a = l;
    stride = (long long)nr * nth;
    base = idx - (long long)l * nr * nth;
  }
  const int i = a - op.lo;
  if (i < 0 || i >= op.n) {
    if (!op.accumulate) out[idx] = 0.0;
    return;
  }
  const double* row = M + (long long)i * op.n;
  const double* src = in + base + (long long)op.lo * stride;
  double s = 0.0;
  for (int t = 0; t < op.n; ++t) s += row[t] * src[(long long)t * stride];
  out[idx] = op.accumulate ? out[idx] + s : s;
}

// q = -2 pi r^2 E psi^5 - g0 is formed in two steps: this kernel writes the
// nodal source; g0 (modal) is subtracted after the forward phi transform.
__global__ __launch_bounds__(XT) void k_source(const double* __restrict__ E, const double* __restrict__ psi,
                                               const double* __restrict__ r2, double* __restrict__ q, int nr,
                                               long long P) {
  const long long idx = (long long)blockIdx.x * XT + threadIdx.x;
  if (idx >= P) return;
  const double p = psi[idx], p2 = p * p;
  q[idx] = -2.0 * PI * r2[idx % nr] * E[idx] * (p2 * p2 * p);
}

__global__ __launch_bounds__(XT) void k_sub(double* __restrict__ a, const double* __restrict__ b, long long P) {
  const long long idx = (long long)blockIdx.x * XT + threadIdx.x;
  if (idx < P) a[idx] -= b[idx];
}

// Interior nodes: w /= lam_r[j - 1] + lam_t[m][k - 1]; the boundary nodes are
// zero already.
__global__ __launch_bounds__(XT) void k_divide(double* __restrict__ w, const double* __restrict__ lam_r,
                                               const double* __restrict__ lam_t, int nr, int nth, int nph) {
  const long long P = (long long)nr * nth * nph;
  const long long idx = (long long)blockIdx.x * XT + threadIdx.x;
  if (idx >= P) return;
  const int j = (int)(idx % nr), k = (int)((idx / nr) % nth), l = (int)(idx / ((long long)nr * nth));
  if (j < 1 || j > nr - 2 || k < 1 || k > nth - 2) return;
  const int m = (l + 1) / 2;
  w[idx] /= lam_r[j - 1] + lam_t[(long long)m * (nth - 2) + (k - 1)];
}

// psi_new = psi0 + u; per block: max |psi_new - psi_prev| and max |psi_new|
// (fixed-order tree in LDS; the host takes the maximum over the blocks).
__global__ __launch_bounds__(XT) void k_update(const double* __restrict__ psi0, const double* __restrict__ u,
                                               const double* __restrict__ prev, double* __restrict__ psi,
                                               double* __restrict__ partials, long long P) {
  __shared__ double sd[XT], sp[XT];
  double d = 0.0, m = 0.0;
  for (long long idx = (long long)blockIdx.x * XT + threadIdx.x; idx < P; idx += (long long)gridDim.x * XT) {
    const double v = psi0[idx] + u[idx];
    psi[idx] = v;
    const double dv = fabs(v - prev[idx]);
    d = (dv != dv || dv > d) ? dv : d;
    m = fmax(m, fabs(v));
  }
  sd[threadIdx.x] = d;
  sp[threadIdx.x] = m;
  __syncthreads();
  for (int h = XT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const double o = sd[threadIdx.x + h];
      sd[threadIdx.x] = (o != o || o > sd[threadIdx.x]) ? o : sd[threadIdx.x];
      sp[threadIdx.x] = fmax(sp[threadIdx.x], sp[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = sd[0];
    partials[2 * blockIdx.x + 1] = sp[0];
  }
}

inline unsigned blocks(long long P) { return (unsigned)((P + XT - 1) / XT); }

hipError_t line(const double* in, double* out, int axis, int lo, int n, const double* M, long long mstride,
                int accumulate, int nr, int nth, int nph, hipStream_t s) {
  LineOp op{axis, lo, n, M, mstride, accumulate};
  const long long P = (long long)nr * nth * nph;
  hipLaunchKernelGGL(k_line, dim3(blocks(P)), dim3(XT), 0, s, in, out, op, nr, nth, nph);
  return hipGetLastError();
}

}  // namespace

size_t xcts_operator_doubles(int nr, int nth, int nph) {
  const size_t ni = (size_t)(nr - 2), nt = (size_t)(nth - 2), nm = (size_t)(nph / 2 + 1);
  return 2 * (size_t)nph * nph + (size_t)nr * nr + 2 * ni * ni + ni + nm * ((size_t)nth * nth + 2 * nt * nt + nt) +
         (size_t)nr;
}

int xcts_solve(const XctsGrid& g, double* work, double* partials, int partial_blocks, hipStream_t s,
               const double* E, double* psi, int max_iter, double tol, int* iters, double* change,
               std::string* err) {
  const int nr = g.nr, nth = g.nth, nph = g.nph;
  const long long P = (long long)nr * nth * nph;
  const int ni = nr - 2, nt = nth - 2, nm = nph / 2 + 1;
  auto fail = [&](const std::string& m) {
    if (err) *err = m;
    return GRMHD_E_ARG;
  };
  if (ni < 1 || nt < 1 || nph < 2 || (nph & 1)) return fail("XCTS needs n_r, n_theta >= 3 and an even n_phi");
  // ---- host operators ----------------------------------------------------
  std::vector<double> D1, D2, lam, V, Vi;
  std::string why;
  // radial: A = (D_xx + Lh D_x) / Lh^2
  cheb_reference_matrices(nr, &D1, &D2);
  std::vector<double> Afull((size_t)nr * nr), Aint((size_t)ni * ni);
  for (int i = 0; i < nr; ++i)
    for (int k = 0; k < nr; ++k)
      Afull[(size_t)i * nr + k] = (D2[(size_t)i * nr + k] + g.Lh * D1[(size_t)i * nr + k]) / (g.Lh * g.Lh);
  for (int i = 0; i < ni; ++i)
    for (int k = 0; k < ni; ++k) Aint[(size_t)i * ni + k] = Afull[(size_t)(i + 1) * nr + (k + 1)];
  std::vector<double> Vr, Vri, lam_r;
  if (!eig_real(ni, Aint, &lam_r, &Vr, &Vri, &why)) return fail("XCTS radial operator: " + why);
  // polar, per Fourier mode m
  cheb_reference_matrices(nth, &D1, &D2);
  std::vector<double> Bfull((size_t)nm * nth * nth), Vt((size_t)nm * nt * nt), Vti((size_t)nm * nt * nt),
      lam_t((size_t)nm * nt);
  std::vector<double> Bint((size_t)nt * nt);
  for (int m = 0; m < nm; ++m) {
    double* B = &Bfull[(size_t)m * nth * nth];
    for (int i = 0; i < nth; ++i) {
      const double th = g.th[i], ct = cos(th) / sin(th), is2 = 1.0 / (sin(th) * sin(th));
      for (int k = 0; k < nth; ++k)
        B[(size_t)i * nth + k] = D2[(size_t)i * nth + k] / (g.Th * g.Th) + ct * D1[(size_t)i * nth + k] / g.Th;
      B[(size_t)i * nth + i] -= (double)m * m * is2;
    }
    for (int i = 0; i < nt; ++i)
      for (int k = 0; k < nt; ++k) Bint[(size_t)i * nt + k] = B[(size_t)(i + 1) * nth + (k + 1)];
    if (!eig_real(nt, Bint, &lam, &V, &Vi, &why)) return fail("XCTS polar operator: " + why);
    std::copy(V.begin(), V.end(), Vt.begin() + (size_t)m * nt * nt);
    std::copy(Vi.begin(), Vi.end(), Vti.begin() + (size_t)m * nt * nt);
    std::copy(lam.begin(), lam.end(), lam_t.begin() + (size_t)m * nt);
  }
  // real DFT along phi: slot 0 the mean, 2m-1 / 2m the cos / sin of mode m,
  // the last slot the Nyquist cosine; Fw: nodal -> slots, Bw: slots -> nodal
  std::vector<double> Fw((size_t)nph * nph), Bw((size_t)nph * nph);
  for (int sl = 0; sl < nph; ++sl) {
    const int m = (sl + 1) / 2;
    const bool sine = sl > 0 && sl < nph - 1 && (sl % 2 == 0);
    for (int l = 0; l < nph; ++l) {
      const double ph = 2.0 * PI * l / nph;
      const double basis = sine ? sin(m * ph) : cos(m * ph);
      const double w = (sl == 0 || sl == nph - 1) ? 1.0 / nph : 2.0 / nph;
      Fw[(size_t)sl * nph + l] = w * basis;
      Bw[(size_t)l * nph + sl] = basis;
    }
  }
  std::vector<double> r2(nr);
  for (int j = 0; j < nr; ++j) r2[j] = g.r[j] * g.r[j];
  // ---- device layout in the work buffer ------------------------------------
  double* W0 = work;
  double* W1 = work + P;
  double* G0 = work + 2 * P;
  double* PSI0 = work + 3 * P;
  double* PREV = work + 4 * P;
  double* o = work + 5 * P;
  auto put = [&](const std::vector<double>& h) {
    double* d = o;
    o += h.size();
    return std::make_pair(d, &h);
  };
  const auto dFw = put(Fw), dBw = put(Bw), dA = put(Afull), dVr = put(Vr), dVri = put(Vri), dlr = put(lam_r),
             dB = put(Bfull), dVt = put(Vt), dVti = put(Vti), dlt = put(lam_t), dr2 = put(r2);
#define XCHK(e)                                                              \
  do {                                                                       \
    hipError_t e_ = (e);                                                     \
    if (e_ != hipSuccess) {                                                  \
      if (err) *err = std::string("XCTS: ") + hipGetErrorString(e_);         \
      return GRMHD_E_DEVICE;                                                 \
    }                                                                        \
  } while (0)
  for (auto pr : {dFw, dBw, dA, dVr, dVri, dlr, dB, dVt, dVti, dlt, dr2})
    XCHK(hipMemcpyAsync(pr.first, pr.second->data(), pr.second->size() * sizeof(double), hipMemcpyHostToDevice, s));
  XCHK(hipMemcpyAsync(PSI0, psi, P * sizeof(double), hipMemcpyDeviceToDevice, s));
  XCHK(hipMemcpyAsync(PREV, psi, P * sizeof(double), hipMemcpyDeviceToDevice, s));
  // g0 = r^2 Lap psi0 in phi slots: A_r along r plus B_m along theta of the
  // phi transform of psi0
  XCHK(line(PSI0, W0, 2, 0, nph, dFw.first, 0, 0, nr, nth, nph, s));
  XCHK(line(W0, G0, 0, 0, nr, dA.first, 0, 0, nr, nth, nph, s));
  XCHK(line(W0, G0, 1, 0, nth, dB.first, (long long)nth * nth, 1, nr, nth, nph, s));
  const int nb = std::min(partial_blocks, (int)blocks(P));
  std::vector<double> host(2 * (size_t)nb);
  double ch = INFINITY;
  int k = 0;
  for (k = 1; k <= max_iter; ++k) {
    hipLaunchKernelGGL(k_source, dim3(blocks(P)), dim3(XT), 0, s, E, PREV, dr2.first, W0, nr, P);
    XCHK(hipGetLastError());
    XCHK(line(W0, W1, 2, 0, nph, dFw.first, 0, 0, nr, nth, nph, s));
    hipLaunchKernelGGL(k_sub, dim3(blocks(P)), dim3(XT), 0, s, W1, G0, P);
    XCHK(hipGetLastError());
    XCHK(line(W1, W0, 1, 1, nt, dVti.first, (long long)nt * nt, 0, nr, nth, nph, s));
    XCHK(line(W0, W1, 0, 1, ni, dVri.first, 0, 0, nr, nth, nph, s));
    hipLaunchKernelGGL(k_divide, dim3(blocks(P)), dim3(XT), 0, s, W1, dlr.first, dlt.first, nr, nth, nph);
    XCHK(hipGetLastError());
    XCHK(line(W1, W0, 0, 1, ni, dVr.first, 0, 0, nr, nth, nph, s));
    XCHK(line(W0, W1, 1, 1, nt, dVt.first, (long long)nt * nt, 0, nr, nth, nph, s));
    XCHK(line(W1, W0, 2, 0, nph, dBw.first, 0, 0, nr, nth, nph, s));
    hipLaunchKernelGGL(k_update, dim3(nb), dim3(XT), 0, s, PSI0, W0, PREV, psi, partials, P);
    XCHK(hipGetLastError());
    XCHK(hipMemcpyAsync(PREV, psi, P * sizeof(double), hipMemcpyDeviceToDevice, s));
    XCHK(hipMemcpyAsync(host.data(), partials, host.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    XCHK(hipStreamSynchronize(s));
    double dmax = 0.0, pmax = 0.0;
    for (int b = 0; b < nb; ++b) {
      const double d = host[2 * b], p = host[2 * b + 1];
      dmax = (d != d || d > dmax) ? d : dmax;
      pmax = std::max(pmax, p);
    }
    ch = pmax > 0 ? dmax / pmax : dmax;
    if (!(ch == ch)) break;  // non-finite: stop and report
    if (ch <= tol) break;
  }
#undef XCHK
  if (iters) *iters = k > max_iter ? max_iter : k;
  if (change) *change = ch;
  return GRMHD_OK;
}

}  // namespace grmhd
