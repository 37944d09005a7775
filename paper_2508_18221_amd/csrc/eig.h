// Host eigen-decomposition of a real square matrix whose eigenvalues are real
// (the one-dimensional collocation operators of the conformal-factor
// equation: the radial operator of r^2 times the flat Laplacian and, per
// Fourier mode, the polar one, both with Dirichlet ends).
//
// Method (textbook, e.g. Golub & Van Loan, "Matrix Computations", ch. 7):
// Householder reduction to upper Hessenberg form H = Q^T A Q; explicitly
// shifted QR steps on the active window of H, each a sweep of Givens
// rotations (Wilkinson shift from the trailing 2 x 2 block, an exceptional
// shift after 10 steps without deflation), with the rotations accumulated into
// Z, until H is upper triangular T = Z^T A Z; eigenvectors of T by back
// substitution, mapped back as V = Z Y; V^{-1} by Gaussian elimination with
// partial pivoting.  A trailing 2 x 2 block with complex eigenvalues, or a
// window that does not deflate, ends the decomposition with an error.
#pragma once

#include <math.h>

#include <algorithm>
#include <string>
#include <vector>

namespace grmhd {

// A = V diag(lam) V^{-1}, matrices row-major n x n.  Returns false (with a
// message) if the eigenvalues are not all real or QR does not converge.
inline bool eig_real(int n, const std::vector<double>& A, std::vector<double>* lam, std::vector<double>* V,
                     std::vector<double>* Vinv, std::string* err) {
  auto at = [n](std::vector<double>& M, int i, int j) -> double& { return M[(size_t)i * n + j]; };
  std::vector<double> H = A, Z((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) at(Z, i, i) = 1.0;
  // ---- Householder reduction to Hessenberg form, accumulated into Z ----
  std::vector<double> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    double alpha = 0.0;
    for (int i = k + 1; i < n; ++i) alpha += at(H, i, k) * at(H, i, k);
    alpha = sqrt(alpha);
    if (alpha == 0.0) continue;
    if (at(H, k + 1, k) > 0) alpha = -alpha;
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    v[k + 1] = at(H, k + 1, k) - alpha;
    for (int i = k + 2; i < n; ++i) v[i] = at(H, i, k);
    double vv = 0.0;
    for (int i = k + 1; i < n; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    // H <- P H P with P = I - 2 v v^T / (v^T v); Z <- Z P
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int i = k + 1; i < n; ++i) s += v[i] * at(H, i, j);
      s *= 2.0 / vv;
      for (int i = k + 1; i < n; ++i) at(H, i, j) -= s * v[i];
    }
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = k + 1; j < n; ++j) s += at(H, i, j) * v[j];
      s *= 2.0 / vv;
      for (int j = k + 1; j < n; ++j) at(H, i, j) -= s * v[j];
      double t = 0.0;
      for (int j = k + 1; j < n; ++j) t += at(Z, i, j) * v[j];
      t *= 2.0 / vv;
      for (int j = k + 1; j < n; ++j) at(Z, i, j) -= t * v[j];
    }
    for (int i = k + 2; i < n; ++i) at(H, i, k) = 0.0;
  }
  // ---- shifted QR on the active window [lo, hi] ----
  const double eps = 2.220446049250313e-16;
  std::vector<double> cs(n), sn(n);
  int hi = n - 1, iter = 0, total = 0;
  while (hi > 0) {
    // deflation: the largest lo with a negligible subdiagonal entry
    int lo = hi;
    while (lo > 0) {
      const double s = fabs(at(H, lo - 1, lo - 1)) + fabs(at(H, lo, lo));
      if (fabs(at(H, lo, lo - 1)) <= eps * (s > 0 ? s : 1.0)) {
        at(H, lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {  // one eigenvalue converged
      --hi;
      iter = 0;
      continue;
    }
    if (++iter > 60 || ++total > 60 * n) {
      if (err) *err = "QR iteration did not converge";
      return false;
    }
    // Wilkinson shift from the trailing 2 x 2 block of the window
    const double a = at(H, hi - 1, hi - 1), b = at(H, hi - 1, hi), c = at(H, hi, hi - 1), d = at(H, hi, hi);
    const double tr = a + d, det = a * d - b * c, disc = 0.25 * tr * tr - det;
    if (disc < 0.0 && hi - lo == 1) {
      if (err) *err = "complex eigenvalue pair";
      return false;
    }
    double mu;
    if (disc >= 0.0) {
      const double r = sqrt(disc), m1 = 0.5 * tr + r, m2 = 0.5 * tr - r;
      mu = fabs(m1 - d) < fabs(m2 - d) ? m1 : m2;
    } else {
      mu = d;
    }
    if (iter % 11 == 10) mu = d + fabs(at(H, hi, hi - 1));  // exceptional shift
    // H - mu I = Q R on the window: rotations G_k acting on rows k, k+1
    for (int k = lo; k <= hi; ++k) at(H, k, k) -= mu;
    for (int k = lo; k < hi; ++k) {
      const double x = at(H, k, k), y = at(H, k + 1, k);
      const double r = hypot(x, y);
      const double cc = r == 0.0 ? 1.0 : x / r, ss = r == 0.0 ? 0.0 : y / r;
      cs[k] = cc;
      sn[k] = ss;
      for (int j = k; j < n; ++j) {  // rows of the whole matrix (columns right of the window too)
        const double h1 = at(H, k, j), h2 = at(H, k + 1, j);
        at(H, k, j) = cc * h1 + ss * h2;
        at(H, k + 1, j) = -ss * h1 + cc * h2;
      }
    }
    // R Q + mu I: the transposed rotations on columns k, k+1 (rows above the
    // window too), accumulated into Z
    for (int k = lo; k < hi; ++k) {
      const double cc = cs[k], ss = sn[k];
      const int imax = std::min(k + 2, hi);
      for (int i = 0; i <= imax; ++i) {
        const double h1 = at(H, i, k), h2 = at(H, i, k + 1);
        at(H, i, k) = cc * h1 + ss * h2;
        at(H, i, k + 1) = -ss * h1 + cc * h2;
      }
      for (int i = 0; i < n; ++i) {
        const double z1 = at(Z, i, k), z2 = at(Z, i, k + 1);
        at(Z, i, k) = cc * z1 + ss * z2;
        at(Z, i, k + 1) = -ss * z1 + cc * z2;
      }
    }
    for (int k = lo; k <= hi; ++k) at(H, k, k) += mu;
  }
  // ---- eigenvectors of the triangular T = H by back substitution ----
  lam->resize(n);
  for (int k = 0; k < n; ++k) (*lam)[k] = at(H, k, k);
  std::vector<double> Y((size_t)n * n, 0.0);
  double tnorm = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) tnorm = std::max(tnorm, fabs(at(H, i, j)));
  for (int k = 0; k < n; ++k) {
    at(Y, k, k) = 1.0;
    for (int j = k - 1; j >= 0; --j) {
      double s = 0.0;
      for (int l = j + 1; l <= k; ++l) s += at(H, j, l) * at(Y, l, k);
      double den = at(H, j, j) - at(H, k, k);
      if (fabs(den) < eps * tnorm) den = (den < 0 ? -1.0 : 1.0) * eps * tnorm;  // near-equal eigenvalues
      at(Y, j, k) = -s / den;
    }
  }
  // V = Z Y, columns normalised to unit 2-norm
  V->assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) {
      double s = 0.0;
      for (int l = 0; l <= k; ++l) s += at(Z, i, l) * at(Y, l, k);
      at(*V, i, k) = s;
    }
  for (int k = 0; k < n; ++k) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += at(*V, i, k) * at(*V, i, k);
    s = 1.0 / sqrt(s);
    for (int i = 0; i < n; ++i) at(*V, i, k) *= s;
  }
  // ---- V^{-1}: Gauss-Jordan elimination with partial pivoting ----
  std::vector<double> M = *V, Inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) at(Inv, i, i) = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int i = c + 1; i < n; ++i)
      if (fabs(at(M, i, c)) > fabs(at(M, p, c))) p = i;
    if (at(M, p, c) == 0.0) {
      if (err) *err = "singular eigenvector matrix";
      return false;
    }
    if (p != c)
      for (int j = 0; j < n; ++j) {
        std::swap(at(M, p, j), at(M, c, j));
        std::swap(at(Inv, p, j), at(Inv, c, j));
      }
    const double piv = 1.0 / at(M, c, c);
    for (int j = 0; j < n; ++j) {
      at(M, c, j) *= piv;
      at(Inv, c, j) *= piv;
    }
    for (int i = 0; i < n; ++i) {
      if (i == c) continue;
      const double f = at(M, i, c);
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        at(M, i, j) -= f * at(M, c, j);
        at(Inv, i, j) -= f * at(Inv, c, j);
      }
    }
  }
  *Vinv = Inv;
  return true;
}

}  // namespace grmhd
