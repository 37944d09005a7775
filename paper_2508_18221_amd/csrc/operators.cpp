// Grid nodes, spectral operators, quadrature weights and the time step.
//
// Methods, "Grid Discretization": Chebyshev-Gauss-Lobatto nodes
// x_j = cos(j pi/(N-1)) (index 0 is x = +1) mapped logarithmically in r
// (ln r = Lc + Lh x) and affinely in theta (theta = Tc + Th y); uniform phi.
// Methods, "The Spectral Derivative Operators": the derivative of the degree
// N-1 Chebyshev interpolant, and the Fourier derivative (ik)^d with
// k = -N/2+1 .. N/2 keeping the real part at the nodes (the Nyquist mode
// drops out of odd derivatives and gives -(N/2)^2 in the second).
// Methods, "Dealiasing and Spectral Filtering": sigma(k) = exp(-alpha
// (|k|/k_max)^p), k_max = N-1 (Chebyshev), N/2 (Fourier).
//
// All operators are dense N x N matrices built in long double and rounded
// once to double; they are stored transposed (AT[k][i] = A[i][k]) and
// zero-padded to a multiple of 16 for the MFMA contraction kernels.
#include <math.h>

#include <string.h>

#include <algorithm>

#include "grmhd_internal.h"

namespace grmhd {

namespace {

typedef long double ld;
const ld PI_L = 3.141592653589793238462643383279502884L;

// Chebyshev first-derivative matrix on CGL nodes (reference coordinate):
// D_ij = (c_i/c_j) (-1)^(i+j) / (x_i - x_j), x_i - x_j written with the
// product-of-sines identity; diagonal = minus the off-diagonal row sum.
std::vector<ld> cheb_d1(int n) {
  const int n1 = n - 1;
  std::vector<ld> D((size_t)n * n, 0.0L);
  for (int i = 0; i < n; ++i) {
    ld ci = (i == 0 || i == n1) ? 2.0L : 1.0L;
    ld rowsum = 0.0L;
    for (int j = 0; j < n; ++j) {
      if (i == j) continue;
      ld cj = (j == 0 || j == n1) ? 2.0L : 1.0L;
      ld dx = -2.0L * sinl((ld)(i + j) * PI_L / (2.0L * n1)) * sinl((ld)(i - j) * PI_L / (2.0L * n1));
      ld v = (ci / cj) * (((i + j) & 1) ? -1.0L : 1.0L) / dx;
      D[(size_t)i * n + j] = v;
      rowsum += v;
    }
    D[(size_t)i * n + i] = -rowsum;
  }
  return D;
}

std::vector<ld> matmul(const std::vector<ld>& A, const std::vector<ld>& B, int n) {
  std::vector<ld> C((size_t)n * n, 0.0L);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      ld a = A[(size_t)i * n + k];
      for (int j = 0; j < n; ++j) C[(size_t)i * n + j] += a * B[(size_t)k * n + j];
    }
  return C;
}

void zero_row_sums(std::vector<ld>& D, int n) {
  for (int i = 0; i < n; ++i) {
    ld s = 0.0L;
    for (int j = 0; j < n; ++j)
      if (j != i) s += D[(size_t)i * n + j];
    D[(size_t)i * n + i] = -s;
  }
}

// Chebyshev modal filter: F = V diag(m) V^{-1} with V_jk = T_k(x_j) =
// cos(k j pi/(N-1)) and the discrete inverse c_k = 2/((N-1) cb_k) sum_l
// f_l T_k(x_l)/cb_l (cb = 2 at the end indices, 1 otherwise).  The modal
// factor m_k is sigma(k) when sig_on, times the 2/3 truncation mask
// (k <= 2(N-1)/3) when trunc: both act diagonally on the modes, so the
// truncation followed by the filter is this one matrix.
std::vector<ld> cheb_filter(int n, ld alpha, int order, bool sig_on, bool trunc) {
  const int n1 = n - 1;
  std::vector<ld> T((size_t)n * n);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j) T[(size_t)k * n + j] = cosl((ld)k * j * PI_L / n1);
  std::vector<ld> F((size_t)n * n, 0.0L);
  for (int k = 0; k < n; ++k) {
    ld sig = sig_on ? expl(-alpha * powl((ld)k / (ld)n1, (ld)order)) : 1.0L;
    if (trunc && 3 * k > 2 * n1) sig = 0.0L;
    ld cbk = (k == 0 || k == n1) ? 2.0L : 1.0L;
    for (int j = 0; j < n; ++j) {
      ld a = sig * T[(size_t)k * n + j] * 2.0L / (n1 * cbk);
      for (int l = 0; l < n; ++l) {
        ld cbl = (l == 0 || l == n1) ? 2.0L : 1.0L;
        F[(size_t)j * n + l] += a * T[(size_t)k * n + l] / cbl;
      }
    }
  }
  return F;
}

// Fourier operators at the nodes: (1/N) sum_k Re[m(k) e^{i k (phi_j - phi_l)}]
// over k = -N/2+1 .. N/2.  kind 1: m = ik; 2: m = -k^2; 3: m = sigma(|k|)
// (1 unless sig_on), times the 2/3 truncation mask |k| <= N/3 when trunc.
std::vector<ld> fourier_op(int n, int kind, ld alpha, int order, bool sig_on = true, bool trunc = false) {
  // the entries depend on (j - l) mod n only
  const ld h = 2.0L * PI_L / n;
  std::vector<ld> c(n, 0.0L);
  for (int d = 0; d < n; ++d) {
    ld s = 0.0L;
    for (int k = -n / 2 + 1; k <= n / 2; ++k) {
      int m = ((k * d) % n + n) % n;  // k (j - l) h reduced mod 2 pi
      ld arg = (ld)m * h;
      if (kind == 1) s += -(ld)k * sinl(arg);
      else if (kind == 2) s += -(ld)k * k * cosl(arg);
      else if (!(trunc && 3 * (k < 0 ? -k : k) > n))
        s += (sig_on ? expl(-alpha * powl(fabsl((ld)k) / (ld)(n / 2), (ld)order)) : 1.0L) * cosl(arg);
    }
    c[d] = s / n;
  }
  std::vector<ld> A((size_t)n * n);
  for (int j = 0; j < n; ++j)
    for (int l = 0; l < n; ++l) A[(size_t)j * n + l] = c[((j - l) % n + n) % n];
  return A;
}

// Clenshaw-Curtis weights on the CGL nodes for the integral over [-1, 1]:
// w = V^{-T} m with the moments m_k = 2/(1-k^2) (even k), 0 (odd k).
std::vector<ld> cc_weights(int n) {
  const int n1 = n - 1;
  std::vector<ld> w(n, 0.0L);
  for (int l = 0; l < n; ++l) {
    ld cbl = (l == 0 || l == n1) ? 2.0L : 1.0L;
    ld s = 0.0L;
    for (int k = 0; k < n; k += 2) {
      ld cbk = (k == 0 || k == n1) ? 2.0L : 1.0L;
      s += (2.0L / (1.0L - (ld)k * k)) * 2.0L * cosl((ld)k * l * PI_L / n1) / (n1 * cbk * cbl);
    }
    w[l] = s;
  }
  return w;
}

void store_transposed(const std::vector<ld>& A, int n, int npad, std::vector<double>* out) {
  out->assign((size_t)npad * npad, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) (*out)[(size_t)k * npad + i] = (double)A[(size_t)i * n + k];
}

// bf16 (1 sign, 8 exponent, 7 mantissa bits) by round-to-nearest-even of a float
uint16_t to_bf16(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
double from_bf16(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float x;
  memcpy(&x, &u, 4);
  return (double)x;
}

// Reduced-precision copies: FP32 transposed AT[k][i] and the BF16 split
// A = hi + lo (hi = bf16(A), lo = bf16(A - hi)), row-major, k padded to kpad.
void store_mixed(const std::vector<ld>& A, int n, int npad, int kpad, std::vector<float>* at32,
                 std::vector<uint16_t>* bhi, std::vector<uint16_t>* blo) {
  at32->assign((size_t)npad * npad, 0.0f);
  bhi->assign((size_t)npad * kpad, 0);
  blo->assign((size_t)npad * kpad, 0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      const double a = (double)A[(size_t)i * n + k];
      (*at32)[(size_t)k * npad + i] = (float)a;
      const uint16_t h = to_bf16((float)a);
      (*bhi)[(size_t)i * kpad + k] = h;
      (*blo)[(size_t)i * kpad + k] = to_bf16((float)(a - from_bf16(h)));
    }
}

// Even/odd fold of a centro-symmetric operator (even n): rows i < n/2,
// E_ik = (A_ik + A_i,n-1-k)/2, O_ik = (A_ik - A_i,n-1-k)/2, stored transposed
// and zero padded to hpad x hpad, E^T first.
void store_fold(const std::vector<ld>& A, int n, int hpad, std::vector<double>* out) {
  const int h = n / 2;
  const size_t hh = (size_t)hpad * hpad;
  out->assign(2 * hh, 0.0);
  for (int i = 0; i < h; ++i)
    for (int k = 0; k < h; ++k) {
      const ld a = A[(size_t)i * n + k], b = A[(size_t)i * n + (n - 1 - k)];
      (*out)[(size_t)k * hpad + i] = (double)(0.5L * (a + b));
      (*out)[hh + (size_t)k * hpad + i] = (double)(0.5L * (a - b));
    }
}

}  // namespace

void cheb_reference_matrices(int n, std::vector<double>* D1, std::vector<double>* D2) {
  std::vector<ld> A = cheb_d1(n);
  std::vector<ld> B = matmul(A, A, n);
  zero_row_sums(B, n);
  D1->resize(A.size());
  D2->resize(B.size());
  for (size_t e = 0; e < A.size(); ++e) {
    (*D1)[e] = (double)A[e];
    (*D2)[e] = (double)B[e];
  }
}

void build_operators(const grmhd_grid& g, double cfl, Operators* ops) {
  const int n[3] = {g.nr, g.nth, g.nph};
  for (int a = 0; a < 3; ++a) {
    ops->n[a] = n[a];
    ops->npad[a] = round_up(n[a], 16);
    ops->kpad[a] = round_up(n[a], 32);
    ops->fold[a] = (n[a] % 2 == 0);
    ops->hpad[a] = round_up(n[a] / 2, 16);
  }
  // nodes, computed in double exactly as x_j = cos(j pi/(N-1)), r = exp(Lc + Lh x)
  ops->Lc = 0.5 * (log(g.r_in) + log(g.r_out));
  ops->Lh = 0.5 * (log(g.r_out) - log(g.r_in));
  ops->Tc = 0.5 * (g.th_min + g.th_max);
  ops->Th = 0.5 * (g.th_max - g.th_min);
  ops->r.resize(g.nr);
  ops->th.resize(g.nth);
  ops->ph.resize(g.nph);
  for (int j = 0; j < g.nr; ++j) ops->r[j] = exp(ops->Lc + ops->Lh * cos(j * M_PI / (g.nr - 1)));
  for (int k = 0; k < g.nth; ++k) ops->th[k] = ops->Tc + ops->Th * cos(k * M_PI / (g.nth - 1));
  for (int l = 0; l < g.nph; ++l) ops->ph[l] = 2.0 * M_PI * l / g.nph;

  const ld Lh = (ld)ops->Lh, Th = (ld)ops->Th;
  // radial: chain rule of the log map
  {
    int nn = g.nr;
    std::vector<ld> D1 = cheb_d1(nn);
    std::vector<ld> D2 = matmul(D1, D1, nn);
    zero_row_sums(D2, nn);
    std::vector<ld> R1(D1.size()), R2(D1.size());
    for (int i = 0; i < nn; ++i) {
      ld ri = (ld)ops->r[i];
      for (int k = 0; k < nn; ++k) {
        size_t e = (size_t)i * nn + k;
        R1[e] = D1[e] / (ri * Lh);
        R2[e] = (D2[e] - Lh * D1[e]) / (ri * ri * Lh * Lh);
      }
    }
    store_transposed(R1, nn, ops->npad[0], &ops->at[0][OP_D1]);
    store_transposed(R2, nn, ops->npad[0], &ops->at[0][OP_D2]);
    store_mixed(R1, nn, ops->npad[0], ops->kpad[0], &ops->at32[0][0], &ops->bhi[0][0], &ops->blo[0][0]);
    store_mixed(R2, nn, ops->npad[0], ops->kpad[0], &ops->at32[0][1], &ops->bhi[0][1], &ops->blo[0][1]);
    const std::vector<ld> Fr = cheb_filter(nn, g.filt_alpha, g.filt_order, g.filter_on, g.dealias);
    store_transposed(Fr, nn, ops->npad[0], &ops->at[0][OP_FILT]);
    if (ops->fold[0]) {
      // folded forms act with the unmapped D1, D2; the map enters as row
      // scales: R1 u = g1 . D1 u, R2 u = g2 . D2 u + g21 . D1 u
      store_fold(D1, nn, ops->hpad[0], &ops->fmat[0][OP_D1]);
      store_fold(D2, nn, ops->hpad[0], &ops->fmat[0][OP_D2]);
      store_fold(Fr, nn, ops->hpad[0], &ops->fmat[0][OP_FILT]);
      ops->gr.resize(3 * (size_t)nn);
      for (int i = 0; i < nn; ++i) {
        const ld ri = (ld)ops->r[i];
        ops->gr[i] = (double)(1.0L / (ri * Lh));
        ops->gr[nn + i] = (double)(1.0L / (ri * ri * Lh * Lh));
        ops->gr[2 * nn + i] = (double)(-1.0L / (ri * ri * Lh));
      }
    }
  }
  // polar: affine map
  {
    int nn = g.nth;
    std::vector<ld> D1 = cheb_d1(nn);
    std::vector<ld> D2 = matmul(D1, D1, nn);
    zero_row_sums(D2, nn);
    for (auto& v : D1) v /= Th;
    for (auto& v : D2) v /= Th * Th;
    store_transposed(D1, nn, ops->npad[1], &ops->at[1][OP_D1]);
    store_transposed(D2, nn, ops->npad[1], &ops->at[1][OP_D2]);
    store_mixed(D1, nn, ops->npad[1], ops->kpad[1], &ops->at32[1][0], &ops->bhi[1][0], &ops->blo[1][0]);
    store_mixed(D2, nn, ops->npad[1], ops->kpad[1], &ops->at32[1][1], &ops->bhi[1][1], &ops->blo[1][1]);
    const std::vector<ld> Ft = cheb_filter(nn, g.filt_alpha, g.filt_order, g.filter_on, g.dealias);
    store_transposed(Ft, nn, ops->npad[1], &ops->at[1][OP_FILT]);
    if (ops->fold[1]) {
      store_fold(D1, nn, ops->hpad[1], &ops->fmat[1][OP_D1]);
      store_fold(D2, nn, ops->hpad[1], &ops->fmat[1][OP_D2]);
      store_fold(Ft, nn, ops->hpad[1], &ops->fmat[1][OP_FILT]);
    }
  }
  // azimuthal: Fourier
  {
    int nn = g.nph;
    const std::vector<ld> F1 = fourier_op(nn, 1, 0, 0), F2 = fourier_op(nn, 2, 0, 0);
    store_transposed(F1, nn, ops->npad[2], &ops->at[2][OP_D1]);
    store_transposed(F2, nn, ops->npad[2], &ops->at[2][OP_D2]);
    store_mixed(F1, nn, ops->npad[2], ops->kpad[2], &ops->at32[2][0], &ops->bhi[2][0], &ops->blo[2][0]);
    store_mixed(F2, nn, ops->npad[2], ops->kpad[2], &ops->at32[2][1], &ops->bhi[2][1], &ops->blo[2][1]);
    const std::vector<ld> Fp = fourier_op(nn, 3, g.filt_alpha, g.filt_order, g.filter_on, g.dealias);
    store_transposed(Fp, nn, ops->npad[2], &ops->at[2][OP_FILT]);
    if (ops->fold[2]) {
      store_fold(F1, nn, ops->hpad[2], &ops->fmat[2][OP_D1]);
      store_fold(F2, nn, ops->hpad[2], &ops->fmat[2][OP_D2]);
      store_fold(Fp, nn, ops->hpad[2], &ops->fmat[2][OP_FILT]);
    }
  }
  // FP32 copies of the folded derivative operators (mixed-precision form)
  for (int a = 0; a < 3; ++a)
    if (ops->fold[a])
      for (int o = 0; o < 2; ++o) {
        const std::vector<double>& src = ops->fmat[a][o];
        ops->fmat32[a][o].assign(src.begin(), src.end());
      }
  // quadrature weights for dr and dtheta
  {
    std::vector<ld> w = cc_weights(g.nr);
    ops->wr.resize(g.nr);
    for (int j = 0; j < g.nr; ++j) ops->wr[j] = (double)(w[j] * (ld)ops->r[j] * Lh);
    w = cc_weights(g.nth);
    ops->wth.resize(g.nth);
    for (int k = 0; k < g.nth; ++k) ops->wth[k] = (double)(w[k] * Th);
  }
  // time step: cfl * min over nodes of min(dr, r dtheta, r sin(theta) dphi),
  // with the smaller neighbour spacing at each node and speed bound 1
  {
    double h = INFINITY;
    const double dph = 2.0 * M_PI / g.nph;
    for (int j = 0; j < g.nr; ++j) {
      double drj = INFINITY;
      if (j > 0) drj = std::min(drj, fabs(ops->r[j] - ops->r[j - 1]));
      if (j + 1 < g.nr) drj = std::min(drj, fabs(ops->r[j + 1] - ops->r[j]));
      for (int k = 0; k < g.nth; ++k) {
        double dtk = INFINITY;
        if (k > 0) dtk = std::min(dtk, fabs(ops->th[k] - ops->th[k - 1]));
        if (k + 1 < g.nth) dtk = std::min(dtk, fabs(ops->th[k + 1] - ops->th[k]));
        double hk = std::min(std::min(drj, ops->r[j] * dtk), ops->r[j] * sin(ops->th[k]) * dph);
        h = std::min(h, hk);
      }
    }
    ops->dt = cfl * h;
  }
}

}  // namespace grmhd
