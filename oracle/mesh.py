"""Mesh side of the method (oracle): load vector and exact periodic solve.

Periodic order-p FE space on n^3 unit elements, (p n)^3 DOFs, arrays indexed
[z, y, x] with global node index p*e + k (mod p n) along each axis.

  load (eq. defineassign with eq. poisson, Gaussian units):
      b_m = 4 pi sum_E sum_a C[E][a] int u_m R_a(. - xbar_E)
  compatibility: b <- b - (1^T b / V) M 1  (uniform neutralising background;
      acts only at round-off level for neutral input)
  solve: K phi = b on the complement of the constants, by fast
      diagonalisation (K1 V = M1 V Lambda, V^T M1 V = I); the zero mode is
      dropped, which fixes the gauge int phi = 0.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from . import fe1d, screens

_EIG: dict = {}


def _eig(p, n):
    key = (p, n)
    if key not in _EIG:
        K1, M1 = fe1d.periodic_matrices(p, n)
        lam, V = scipy.linalg.eigh(K1, M1)
        _EIG[key] = (K1, M1, lam, V)
    return _EIG[key]


def element_node_index(p, n):
    """Global 1-D node index of local node k of element e: (p e + k) mod p n."""
    return (p * np.arange(n)[:, None] + np.arange(p + 1)[None, :]) % (p * n)


def support_node_index(p, n, s):
    """Global 1-D node index of the support-local node k = 0 .. s p of the
    screens of element e (s = 1 or 3 elements per axis, the support starting
    (s - 1) / 2 elements below e): (p (e - (s-1)/2) + k) mod p n."""
    e0 = np.arange(n) - (s - 1) // 2
    return (p * e0[:, None] + np.arange(s * p + 1)[None, :]) % (p * n)


def load_vector(C, n, p, q, support="one"):
    """b_m = 4 pi sum_E sum_a C[E][a] int u_m R_a(. - xbar_E): every element
    adds its screens' load to the nodes of its support."""
    d = screens.moment_degree(q, support)
    s = screens.span(support)
    g = screens.load_weights(p, q, support)
    A = screens.moment_exponents(d)
    P = p * n
    Cg = C.reshape(n, n, n, len(A))                       # [ez, ey, ex, a]
    Gs = np.stack([np.einsum("k,j,i->kji", g[az], g[ay], g[ax]) for (ax, ay, az) in A])
    loc = 4.0 * math.pi * np.einsum("zyxa,akji->zyxkji", Cg, Gs, optimize=True)
    b = np.zeros((P, P, P))
    idx = support_node_index(p, n, s)
    K = s * p + 1
    # for a fixed local node (mz, my, mx) the global nodes of different
    # elements are distinct, so the fancy-indexed += does not drop terms
    for mz in range(K):
        for my in range(K):
            for mx in range(K):
                b[np.ix_(idx[:, mz], idx[:, my], idx[:, mx])] += loc[:, :, :, mz, my, mx]
    return b


def mass_ones(p, n):
    """(M 1) as the 1-D factor w1 = M1 1 (the 3-D vector is w1 (x) w1 (x) w1)."""
    _, M1, _, _ = _eig(p, n)
    return M1.sum(axis=1)


def project_compatible(b, p, n):
    w1 = mass_ones(p, n)
    V = float(n) ** 3
    s = b.sum() / V
    return b - s * np.einsum("k,j,i->kji", w1, w1, w1)


def solve_periodic(b, p, n):
    _, _, lam, V = _eig(p, n)
    y = fe1d.kron_apply(V.T, V.T, V.T, b)
    D = lam[:, None, None] + lam[None, :, None] + lam[None, None, :]
    D[0, 0, 0] = np.inf                                   # constant mode (lam[0] = 0)
    return fe1d.kron_apply(V, V, V, y / D)


def stiffness_apply(phi, p, n):
    K1, M1, _, _ = _eig(p, n)
    return fe1d.stiffness_apply(K1, M1, phi)


def mean_value(phi, p, n):
    """(1/V) int phi = (M 1)^T phi / V."""
    w1 = mass_ones(p, n)
    return np.einsum("kji,k,j,i->", phi, w1, w1, w1) / float(n) ** 3
