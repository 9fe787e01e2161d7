"""Polynomial screens (oracle).

A charge at offset delta from the centre of its element gets a screen
density rho(x) built from order-q Lagrange basis functions whose moments
about the charge vanish up to a given order (Section 2.1, eq. moments,
Table moments).  On a uniform cubic mesh the 3-D moment system separates
into three 1-D systems (eq. oned, eq. moment1d): per axis, solve

    sum_i  mom_i^(l) w_i = delta^l ,  l = 0..d ,

with the moment matrix inverted once for all charges.  Writing the solution
as w(delta) = Minv [1, delta, ..., delta^d] shows the 1-D screen is
rho_1(x; delta) = sum_l delta^l r_l(x) with "dual" functions r_l that satisfy
int x^m r_l = [m == l].  The 3-D screen is the product over the axes, so the
combined screen of all charges in an element E is

    sum_{j in E} Q_j rho_j = sum_a C[E][a] R_a ,  R_a = r_ax (x) r_ay (x) r_az,
    C[E][a] = sum_{j in E} Q_j delta_j^a   (a in {0..d}^3).

Two supports are implemented:

  "27"   the paper's construction (Section 2.1): the order-q Lagrange
         functions of the nodes in the closed element of the charge; the
         functions of its face nodes reach into the neighbouring elements,
         so the support is the 3^3 block of elements and the (q+1) functions
         per axis cancel d = q moments (short-range decay R^-(q+2)).  The
         order-q mesh nodes are equispaced in every element (the paper does
         not name the node family; for q >= 2 the span depends on it).
  "one"  the one-element variant of the Discussion (Section 5): only the
         (q-1) functions interior to the element; d = q-2 moments are
         cancelled (q = 3: monopole and dipole, R^-3).  Its span,
         bubble * P_{q-2}, does not depend on the node family.

The mesh solve uses order p = q + 2 in both cases (Section 2.2).

Everything is in element units (h = 1, element = [-1/2, 1/2], delta = u).
"""
from __future__ import annotations

import numpy as np

from . import fe1d

SUPPORTS = ("one", "27")


def moment_degree(q, support="one"):
    """Moments cancelled per axis: d = q - 2 (one element) or q (27 elements)."""
    return q - 2 if support == "one" else q


def span(support="one"):
    """Elements per axis covered by one element's screens."""
    return 1 if support == "one" else 3


def _check(q, support):
    if support not in SUPPORTS:
        raise ValueError(f"unknown screen support {support!r}")
    if support == "one" and q < 2:
        raise ValueError("one-element screens need q >= 2")
    if support == "27" and q < 1:
        raise ValueError("27-element screens need q >= 1")


def interior_basis_nodes(q):
    """Nodes of the order-q element (equispaced); the one-element screen uses
    the interior ones.  The span of the interior functions, bubble * P_{q-2},
    does not depend on this choice."""
    return np.linspace(-0.5, 0.5, q + 1)


def screen_basis(q, support, x):
    """Values of the screen basis functions psi_i at points x (element units,
    the charge's element is [-1/2, 1/2]): shape (len(x), number of functions).

    one: the q-1 interior order-q Lagrange functions of the element.
    27:  the q+1 order-q Lagrange functions of the nodes of the closed
         element; the end functions continue into the element below (node
         at -1/2, the upper node there) or above (node at +1/2, the lower
         node there) and vanish beyond."""
    _check(q, support)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    nodes = interior_basis_nodes(q)
    if support == "one":
        out = fe1d.lagrange(nodes, x)[:, 1:q]
        out[np.abs(x) > 0.5] = 0.0
        return out
    out = np.zeros((len(x), q + 1))
    mid = np.abs(x) <= 0.5
    out[mid] = fe1d.lagrange(nodes, x[mid])
    lo = (x < -0.5) & (x >= -1.5)
    out[lo, 0] = fe1d.lagrange(nodes, x[lo] + 1.0)[:, q]
    hi = (x > 0.5) & (x <= 1.5)
    out[hi, q] = fe1d.lagrange(nodes, x[hi] - 1.0)[:, 0]
    return out


def _element_rule(q, support, m):
    """Gauss-Legendre points and weights covering the support element by
    element (m points per element)."""
    xq, wq = fe1d.gauss_legendre(m)
    s = span(support)
    offs = np.arange(s) - (s - 1) // 2
    return (offs[:, None] + xq[None, :]).ravel(), np.tile(wq, s)


def moment_matrix_1d(q, support="one"):
    """mom[l, i] = int x^l psi_i(x) dx over the support for the screen basis
    functions psi_i, l = 0..d (eq. moment1d)."""
    d = moment_degree(q, support)
    xs, ws = _element_rule(q, support, q + 3)
    psi = screen_basis(q, support, xs)
    return np.array([[np.sum(ws * xs**l * psi[:, i]) for i in range(psi.shape[1])]
                     for l in range(d + 1)])


def dual_coefficients(q, support="one"):
    """Coefficients c[i, l] of the dual functions r_l = sum_i c[i,l] psi_i,
    i.e. the inverse of the 1-D moment matrix."""
    return np.linalg.inv(moment_matrix_1d(q, support))


def dual_functions(q, x, support="one"):
    """r_l(x) for l = 0..d (zero outside the support): shape (len(x), d+1)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    return screen_basis(q, support, x) @ dual_coefficients(q, support)


def screen_1d(q, x, delta, support="one"):
    """1-D screen of a charge at offset delta: sum_l delta^l r_l(x)."""
    r = dual_functions(q, x, support)
    d = r.shape[1] - 1
    return r @ (np.asarray(delta) ** np.arange(d + 1))


def load_weights(p, q, support="one"):
    """g[l, k] = int l_k^(p)(x) r_l(x) dx for the order-p GLL basis functions
    l_k of the support's nodes: k = 0 .. s p along one axis (s = 1 or 3
    elements; node s p is the upper end), the first at the lower end of the
    support.  The load of element E on the node with support-local index
    (kx, ky, kz) is 4 pi sum_a C[E][a] g[ax,kx] g[ay,ky] g[az,kz] (eq.
    defineassign with the Galerkin right-hand side of eq. poisson)."""
    s = span(support)
    nodes_p = fe1d.gll_nodes(p)
    xq, wq = fe1d.gauss_legendre(p + 1)   # degree p + q <= 2p + 1 per element
    lp = fe1d.lagrange(nodes_p, xq)        # (Q, p+1)
    d = moment_degree(q, support)
    g = np.zeros((d + 1, s * p + 1))
    for e in range(s):
        off = e - (s - 1) // 2
        r = dual_functions(q, xq + off, support)
        g[:, e * p:e * p + p + 1] += (r * wq[:, None]).T @ lp
    return g


def axis_moment_coefficients(q, support="one"):
    """nu[l] = int x r_l(x) dx and mu[l] = int x^2 r_l(x) dx: the 1-D screen
    rho_1 = sum_l delta^l r_l has first and second moments (about the
    element centre) sum_l delta^l nu[l] and sum_l delta^l mu[l]."""
    d = moment_degree(q, support)
    xs, ws = _element_rule(q, support, q + 3)
    r = dual_functions(q, xs, support)
    nu = np.array([np.sum(ws * xs * r[:, l]) for l in range(d + 1)])
    mu = np.array([np.sum(ws * xs**2 * r[:, l]) for l in range(d + 1)])
    return nu, mu


def moment_exponents(d):
    """Multi-indices a = (ax, ay, az) in {0..d}^3, x fastest (as in eq. oned)."""
    out = []
    for az in range(d + 1):
        for ay in range(d + 1):
            for ax in range(d + 1):
                out.append((ax, ay, az))
    return np.array(out, dtype=np.int64)


def element_moments(e_lin, u, Q, n_elem, d):
    """C[E][a] = sum_{j in E} Q_j u_j^a (u = offset from the element centre in
    element units).  Returns shape (n_elem, (d+1)^3)."""
    A = moment_exponents(d)
    mono = np.prod(u[:, None, :] ** A[None, :, :], axis=2) * Q[:, None]
    C = np.zeros((n_elem, len(A)))
    np.add.at(C, e_lin, mono)
    return C


def screen_3d_dense(q, delta, support="one"):
    """Screen coefficients from the full 3-D moment system (eq. momentmatrix):
    unknowns are the products of the 1-D screen basis functions, rows the
    moments (l,m,n) <= (d,d,d) about the charge.  Used only to check that the
    separable route gives the same screen.  Returns c (ordered x fastest)."""
    d = moment_degree(q, support)
    xq, wq = _element_rule(q, support, q + 4)
    psi = screen_basis(q, support, xq)
    nb = psi.shape[1]
    A = moment_exponents(d)
    rows = []
    for (l, m, nn) in A:
        mx = [np.sum(wq * (xq - delta[0])**l * psi[:, i]) for i in range(nb)]
        my = [np.sum(wq * (xq - delta[1])**m * psi[:, i]) for i in range(nb)]
        mz = [np.sum(wq * (xq - delta[2])**nn * psi[:, i]) for i in range(nb)]
        rows.append(np.einsum("k,j,i->kji", mz, my, mx).ravel())
    Mat = np.array(rows)
    rhs = np.zeros(len(A))
    rhs[0] = 1.0
    return np.linalg.solve(Mat, rhs)
