"""Exact free-space potential of a separable polynomial density (oracle).

The screen potential of eq. screenintegral,
    Phi_sc(x) = int rho(xi) / |x - xi| d xi ,
is evaluated for tensor-product densities rho = f_x (x) f_y (x) f_z, each f a
polynomial on the element [-1/2, 1/2] (zero outside), through the Gaussian
identity 1/r = (2/sqrt(pi)) int_0^inf exp(-r^2 t^2) dt:

    Phi(x) = (2/sqrt(pi)) int_0^inf  F_x(t) F_y(t) F_z(t) dt ,
    F(t; x) = int_{-1/2}^{1/2} f(s) exp(-t^2 (x - s)^2) ds .

The t-integral is taken in tau = ln t with composite Gauss-Legendre panels;
F uses Gauss-Legendre in s while the Gaussian is wide (t <= 4) and the
closed form through erf/erfc and the recursion for int s^k exp(-s^2) ds
otherwise.  Element units (h = 1).
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import polynomial as P
from scipy.special import erf, erfc

from . import fe1d

_SQRT_PI = math.sqrt(math.pi)


def _tau_rule(tau_min=-36.0, tau_max=22.0, width=0.5, pts=16):
    t, w = np.polynomial.legendre.leggauss(pts)
    edges = np.arange(tau_min, tau_max + 1e-12, width)
    taus, ws = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        taus.append(0.5 * (b - a) * t + 0.5 * (b + a))
        ws.append(0.5 * (b - a) * w)
    return np.concatenate(taus), np.concatenate(ws)


_TAU, _TAU_W = _tau_rule()
_SQ, _SW = fe1d.gauss_legendre(48)


def _gauss_moments(A, B, kmax):
    """J_k = int_A^B s^k exp(-s^2) ds for k = 0..kmax (arrays A <= B)."""
    J = np.zeros((kmax + 1,) + A.shape)
    pos = A >= 0
    neg = B <= 0
    mid = ~(pos | neg)
    J0 = np.empty_like(A)
    J0[pos] = 0.5 * _SQRT_PI * (erfc(A[pos]) - erfc(B[pos]))
    J0[neg] = 0.5 * _SQRT_PI * (erfc(-B[neg]) - erfc(-A[neg]))
    J0[mid] = 0.5 * _SQRT_PI * (erf(B[mid]) - erf(A[mid]))
    J[0] = J0
    eA = np.exp(-A * A)
    eB = np.exp(-B * B)
    if kmax >= 1:
        J[1] = 0.5 * (eA - eB)
    for k in range(2, kmax + 1):
        J[k] = 0.5 * (k - 1) * J[k - 2] + 0.5 * (A ** (k - 1) * eA - B ** (k - 1) * eB)
    return J


def gaussian_factor(coef, t, x):
    """F(t; x) = int_{-1/2}^{1/2} f(s) exp(-t^2 (x-s)^2) ds for the polynomial f
    with monomial coefficients `coef` (ascending).  t: (T,), x: (X,) -> (T, X)."""
    t = np.asarray(t, dtype=np.float64)[:, None]
    x = np.asarray(x, dtype=np.float64)[None, :]
    out = np.zeros(np.broadcast(t, x).shape)
    # wide Gaussian: plain Gauss-Legendre in s
    wide = (t <= 4.0)[:, 0]
    if wide.any():
        fs = P.polyval(_SQ, coef)                             # (S,)
        tw = t[wide]                                          # (Tw,1)
        g = np.exp(-(tw[:, :, None] ** 2) * (x[:, :, None] - _SQ[None, None, :]) ** 2)
        out[wide] = np.einsum("tis,s->ti", g, fs * _SW)
    narrow = ~wide
    if narrow.any():
        tn = np.broadcast_to(t[narrow], (narrow.sum(), x.shape[1]))
        xn = np.broadcast_to(x, tn.shape)
        A = tn * (-0.5 - xn)
        B = tn * (0.5 - xn)
        dist = np.maximum(np.maximum(-0.5 - xn, xn - 0.5), 0.0)
        far = tn * dist > 10.0
        kmax = len(coef) - 1
        J = _gauss_moments(A, B, kmax)
        # f(x + s/t) = sum_j d_j(x) (s/t)^j with d_j = f^(j)(x)/j!
        val = np.zeros(tn.shape)
        dcoef = np.array(coef, dtype=np.float64)
        fact = 1.0
        for j in range(kmax + 1):
            dj = P.polyval(xn, dcoef) / fact
            val += dj * J[j] / tn ** (j + 1)
            dcoef = P.polyder(dcoef) if len(dcoef) > 1 else np.array([0.0])
            fact *= (j + 1)
        val[far] = 0.0
        out[narrow] = val
    return out


def _axis_factor(f, t, x):
    """1-D factor of one axis: f is either the monomial coefficients of a
    polynomial on the element [-1/2, 1/2], or a list of (offset, coefficients)
    pieces, each a polynomial on the element centred at `offset` (in the local
    coordinate of that element).  The factor of a sum of pieces is the sum of
    their factors."""
    if isinstance(f, list) and f and isinstance(f[0], tuple):
        return sum(gaussian_factor(c, t, np.asarray(x) - off) for off, c in f)
    return gaussian_factor(f, t, x)


def separable_potential(coefs, pts, chunk=2048):
    """Potential of rho = f_0(x) f_1(y) f_2(z) at points pts (M,3).
    coefs: one entry per axis, monomial coefficients of a polynomial on the
    element or a list of (offset, coefficients) pieces (see _axis_factor)."""
    pts = np.asarray(pts, dtype=np.float64)
    t = np.exp(_TAU)
    wt = _TAU_W * t * (2.0 / _SQRT_PI)
    out = np.empty(len(pts))
    for s in range(0, len(pts), chunk):
        q = pts[s:s + chunk]
        Fx = _axis_factor(coefs[0], t, q[:, 0])
        Fy = _axis_factor(coefs[1], t, q[:, 1])
        Fz = _axis_factor(coefs[2], t, q[:, 2])
        out[s:s + chunk] = wt @ (Fx * Fy * Fz)
    return out


def dual_polynomials(q, support="one"):
    """The dual functions r_l as polynomial pieces.  One-element support:
    per l the monomial coefficients on the element (degree q).  27-element
    support: per l a list of (offset, coefficients) for the elements at
    offsets -1, 0, 1 (coefficients in the local coordinate of each)."""
    from . import screens
    s = screens.span(support)
    xs = np.linspace(-0.5, 0.5, q + 3)
    d = screens.moment_degree(q, support)
    if s == 1:
        r = screens.dual_functions(q, xs, support)
        return [P.polyfit(xs, r[:, l], q) for l in range(d + 1)]
    out = [[] for _ in range(d + 1)]
    for off in (-1, 0, 1):
        # sample strictly inside the element so each piece is fitted alone
        xi = 0.499 * np.linspace(-1.0, 1.0, q + 3)
        r = screens.dual_functions(q, xi + off, support)
        for l in range(d + 1):
            out[l].append((float(off), P.polyfit(xi, r[:, l], q)))
    return out


def uniform_box_potential(lo, hi, x):
    """Closed-form potential of unit density on the box [lo, hi] (3-vectors)
    at point x: the classical prism formula, sum over corners with
    alternating signs of
      XY ln(Z+r) + YZ ln(X+r) + ZX ln(Y+r)
      - X^2/2 atan(YZ/(Xr)) - Y^2/2 atan(ZX/(Yr)) - Z^2/2 atan(XY/(Zr)),
    X, Y, Z the corner coordinates relative to x.  Points must avoid the
    box's edge lines (log/atan singular sets)."""
    x = np.asarray(x, dtype=np.float64)

    def at(a, b):
        return 0.0 if b == 0.0 else math.atan(a / b)

    tot = 0.0
    for i, X in enumerate((lo[0] - x[0], hi[0] - x[0])):
        for j, Y in enumerate((lo[1] - x[1], hi[1] - x[1])):
            for k, Z in enumerate((lo[2] - x[2], hi[2] - x[2])):
                r = math.sqrt(X * X + Y * Y + Z * Z)
                f = (X * Y * math.log(Z + r) + Y * Z * math.log(X + r)
                     + Z * X * math.log(Y + r)
                     - 0.5 * X * X * at(Y * Z, X * r)
                     - 0.5 * Y * Y * at(Z * X, Y * r)
                     - 0.5 * Z * Z * at(X * Y, Z * r))
                tot += (-1) ** (i + j + k + 1) * f
    return tot
