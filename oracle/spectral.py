"""Grid and spectral operators, oracle side (plain NumPy FP64).

Paper: Methods, "Grid Discretization" (Chebyshev-Gauss-Lobatto radial nodes
x_j = cos(j pi/(N-1)), uniform azimuthal nodes), "The Spectral Derivative
Operators" (Chebyshev expansion -> chebder -> evaluation; Fourier (ik)^d with
k = -N/2+1 .. N/2) and "Dealiasing and Spectral Filtering" (2/3 rule and the
exponential filter sigma(k) = exp(-alpha (|k|/k_max)^p)).

Readings of the paper taken here (where it is silent or inconsistent):
  * radial coordinate: CGL nodes in x, with ln r = Lc + Lh x (logarithmic map;
    the paper's contour figure uses x1 = ln r).  Index 0 is r_out.
  * polar coordinate: CGL nodes y in [-1, 1], theta = Tc + Th y on
    [th_min, th_max] (the paper's uniform Fourier theta grid is not periodic
    on [0, pi]).  Index 0 is th_max.
  * Fourier Nyquist mode (k = N/2): the real part of the inverse transform is
    kept, so it drops out of odd derivatives and contributes -(N/2)^2 to the
    second derivative.
  * filter: sigma(k) with alpha = 36 and order p given by the caller (16 for the
    workloads here); k_max = N-1 for Chebyshev, N/2 for Fourier.

Arrays of grid functions have shape (..., n_phi, n_theta, n_r): r is the last
(fastest) axis, theta the one before, phi the one before that.
"""

import numpy as np
from numpy.polynomial import chebyshev as npcheb

AX_R, AX_TH, AX_PH = -1, -2, -3


def cgl_nodes(n):
    """Chebyshev-Gauss-Lobatto nodes x_j = cos(j pi / (n-1)), j = 0..n-1."""
    j = np.arange(n, dtype=np.float64)
    return np.cos(j * np.pi / (n - 1))


class Grid:
    """Mapped Chebyshev(r) x Chebyshev(theta) x Fourier(phi) grid."""

    def __init__(self, nr, nth, nph, r_in, r_out, th_min, th_max):
        if nph % 2:
            raise ValueError("n_phi must be even (Fourier Nyquist rule)")
        self.nr, self.nth, self.nph = int(nr), int(nth), int(nph)
        self.r_in, self.r_out = float(r_in), float(r_out)
        self.th_min, self.th_max = float(th_min), float(th_max)
        self.x = cgl_nodes(nr)
        self.Lc = 0.5 * (np.log(r_in) + np.log(r_out))
        self.Lh = 0.5 * (np.log(r_out) - np.log(r_in))
        self.r = np.exp(self.Lc + self.Lh * self.x)
        self.y = cgl_nodes(nth)
        self.Tc = 0.5 * (th_min + th_max)
        self.Th = 0.5 * (th_max - th_min)
        self.th = self.Tc + self.Th * self.y
        self.ph = 2.0 * np.pi * np.arange(nph, dtype=np.float64) / nph
        self.shape = (self.nph, self.nth, self.nr)
        self.npts = self.nph * self.nth * self.nr
        # broadcastable 3D coordinate arrays
        self.R = np.broadcast_to(self.r[None, None, :], self.shape)
        self.TH = np.broadcast_to(self.th[None, :, None], self.shape)
        self.PH = np.broadcast_to(self.ph[:, None, None], self.shape)

    # ---- derivatives (paper's route) -------------------------------------
    def d_r(self, f):
        """dr f = (1/(r Lh)) dx f  (chain rule of ln r = Lc + Lh x)."""
        return cheb_deriv(f, AX_R, 1) / (self.r * self.Lh)

    def d_rr(self, f):
        """drr f = (dxx f - Lh dx f) / (r Lh)^2."""
        fx = cheb_deriv(f, AX_R, 1)
        fxx = cheb_deriv(f, AX_R, 2)
        return (fxx - self.Lh * fx) / (self.r * self.Lh) ** 2

    def d_th(self, f):
        return cheb_deriv(f, AX_TH, 1) / self.Th

    def d_thth(self, f):
        return cheb_deriv(f, AX_TH, 2) / self.Th ** 2

    def d_ph(self, f):
        return fourier_deriv(f, AX_PH, 1)

    def d_phph(self, f):
        return fourier_deriv(f, AX_PH, 2)

    def d1(self, f, axis):
        """First derivative along coordinate 0 = r, 1 = theta, 2 = phi."""
        return (self.d_r, self.d_th, self.d_ph)[axis](f)

    def d2(self, f, a, b):
        """Second derivative d_a d_b f.  Pure ones use the m = 2 route; mixed
        ones apply first-derivative operators in sequence, the lower
        coordinate index first (d_r then d_theta, d_r then d_phi, d_theta then
        d_phi)."""
        if a == b:
            return (self.d_rr, self.d_thth, self.d_phph)[a](f)
        lo, hi = min(a, b), max(a, b)
        return self.d1(self.d1(f, lo), hi)

    # ---- filter ------------------------------------------------------------
    def filter(self, f, alpha, order):
        """Exponential filter along r, then theta, then phi."""
        g = cheb_filter(f, AX_R, alpha, order)
        g = cheb_filter(g, AX_TH, alpha, order)
        return fourier_filter(g, AX_PH, alpha, order)

    def dealias(self, f):
        """2/3 truncation along all three axes (Methods, Dealiasing item 1)."""
        g = cheb_truncate(f, AX_R)
        g = cheb_truncate(g, AX_TH)
        return fourier_truncate(g, AX_PH)


# ---- Chebyshev (numpy.polynomial.chebyshev, as the paper does) -------------

def _to_coeffs(f, axis):
    n = f.shape[axis]
    V = npcheb.chebvander(cgl_nodes(n), n - 1)  # V[j, k] = T_k(x_j)
    fa = np.moveaxis(f, axis, 0)
    shp = fa.shape
    coef = np.linalg.solve(V, fa.reshape(n, -1))
    return coef, shp


def _from_coeffs(coef, n, shp, axis):
    # evaluate sum_k c_k T_k(x_j) at the n CGL nodes
    vals = npcheb.chebvander(cgl_nodes(n), coef.shape[0] - 1) @ coef
    return np.moveaxis(vals.reshape(shp), 0, axis)


def cheb_deriv(f, axis, m):
    """m-th derivative in the reference coordinate of the degree n-1
    Chebyshev interpolant at the CGL nodes: coefficients by solving the
    Vandermonde system, chebder, then evaluation (Methods, Radial Chebyshev
    Spectral Derivative)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    coef, shp = _to_coeffs(f, axis)
    dcoef = npcheb.chebder(coef, m=m, axis=0)
    return _from_coeffs(dcoef, n, shp, axis)


def cheb_filter(f, axis, alpha, order):
    """Multiply Chebyshev mode k by exp(-alpha (k/(n-1))^order)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    coef, shp = _to_coeffs(f, axis)
    k = np.arange(n, dtype=np.float64)
    coef = coef * np.exp(-alpha * (k / (n - 1)) ** order)[:, None]
    return _from_coeffs(coef, n, shp, axis)


def cheb_truncate(f, axis):
    """Zero Chebyshev modes k > 2(n-1)/3."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    coef, shp = _to_coeffs(f, axis)
    k = np.arange(n)
    coef = coef * (k <= 2.0 * (n - 1) / 3.0)[:, None]
    return _from_coeffs(coef, n, shp, axis)


# ---- Fourier ---------------------------------------------------------------

def fourier_wavenumbers(n):
    """k = 0, 1, .., n/2, -n/2+1, .., -1 (the paper's set; Nyquist is +n/2)."""
    k = np.fft.fftfreq(n, d=1.0 / n)
    k[n // 2] = n // 2
    return k


def _along(v, axis, ndim):
    shape = [1] * ndim
    shape[axis] = -1
    return v.reshape(shape)


def fourier_deriv(f, axis, d):
    """Re IFFT((ik)^d FFT f) along `axis`."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    mult = (1j * fourier_wavenumbers(n)) ** d
    F = np.fft.fft(f, axis=axis)
    return np.real(np.fft.ifft(F * _along(mult, axis, f.ndim), axis=axis))


def fourier_filter(f, axis, alpha, order):
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    k = np.abs(fourier_wavenumbers(n))
    sig = np.exp(-alpha * (k / (n // 2)) ** order)
    F = np.fft.fft(f, axis=axis)
    return np.real(np.fft.ifft(F * _along(sig, axis, f.ndim), axis=axis))


def fourier_truncate(f, axis):
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    keep = np.abs(fourier_wavenumbers(n)) <= n / 3.0
    F = np.fft.fft(f, axis=axis)
    return np.real(np.fft.ifft(F * _along(keep.astype(np.float64), axis, f.ndim), axis=axis))


# ---- quadrature (diagnostics) -----------------------------------------------

def clenshaw_curtis_weights(n):
    """Weights w_j with sum_j w_j f(x_j) = integral_{-1}^{1} f for every
    polynomial of degree <= n-1 at the CGL nodes (computed from the moments of
    T_k: integral T_k = 2/(1-k^2) for even k, 0 for odd k)."""
    V = npcheb.chebvander(cgl_nodes(n), n - 1)
    k = np.arange(n)
    mom = np.zeros(n)
    ev = k % 2 == 0
    mom[ev] = 2.0 / (1.0 - k[ev].astype(np.float64) ** 2)
    # integral of sum_k c_k T_k = mom . c, with c = V^{-1} f  =>  w = V^{-T} mom
    return np.linalg.solve(V.T, mom)
