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

Variant implemented: the one-element support of the Discussion (Section 5):
only DOFs interior to the charge's element, i.e. the (q-1) interior order-q
Lagrange functions per axis; d = q-2 moments per axis are cancelled.  With
q = 3 this is the lowest order that cancels monopole and dipole, so the
short-range potential decays like R^-3, while the mesh solve uses p = q+2.

Everything is in element units (h = 1, element = [-1/2, 1/2], delta = u).
"""
from __future__ import annotations

import numpy as np

from . import fe1d


def interior_basis_nodes(q):
    """Nodes of the order-q element (equispaced); the screen uses the
    interior ones.  The span of the interior functions, bubble * P_{q-2},
    does not depend on this choice."""
    return np.linspace(-0.5, 0.5, q + 1)


def moment_matrix_1d(q):
    """mom[l, i] = int_{-1/2}^{1/2} x^l psi_i(x) dx for the q-1 interior
    order-q basis functions psi_i, l = 0..q-2 (eq. moment1d, one-element
    support)."""
    nodes = interior_basis_nodes(q)
    xq, wq = fe1d.gauss_legendre(q + 2)
    psi = fe1d.lagrange(nodes, xq)[:, 1:q]      # interior functions only
    d = q - 2
    mom = np.array([[np.sum(wq * xq**l * psi[:, i]) for i in range(q - 1)]
                    for l in range(d + 1)])
    return mom


def dual_coefficients(q):
    """Coefficients c[i, l] of the dual functions r_l = sum_i c[i,l] psi_i,
    i.e. the inverse of the 1-D moment matrix."""
    return np.linalg.inv(moment_matrix_1d(q))


def dual_functions(q, x):
    """r_l(x) for l = 0..d on the element (zero outside): shape (len(x), d+1)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    nodes = interior_basis_nodes(q)
    psi = fe1d.lagrange(nodes, x)[:, 1:q]
    r = psi @ dual_coefficients(q)
    r[np.abs(x) > 0.5] = 0.0
    return r


def screen_1d(q, x, delta):
    """1-D screen of a charge at offset delta: sum_l delta^l r_l(x)."""
    r = dual_functions(q, x)
    d = r.shape[1] - 1
    return r @ (np.asarray(delta) ** np.arange(d + 1))


def load_weights(p, q):
    """g[l, k] = int l_k^(p)(x) r_l(x) dx over the element, for the order-p
    GLL basis l_k.  The load of element E on its node m = (mx, my, mz) is
    4 pi sum_a C[E][a] g[ax,mx] g[ay,my] g[az,mz] (eq. defineassign with the
    Galerkin right-hand side of eq. poisson)."""
    nodes_p = fe1d.gll_nodes(p)
    xq, wq = fe1d.gauss_legendre(p + 1)   # degree p + q <= 2p + 1
    lp = fe1d.lagrange(nodes_p, xq)
    r = dual_functions(q, xq)
    return (r * wq[:, None]).T @ lp


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


def screen_3d_dense(q, delta):
    """Screen coefficients from the full 3-D moment system (eq. momentmatrix)
    for the one-element support: unknowns are the (q-1)^3 products of
    interior basis functions, rows the moments (l,m,n) <= (d,d,d) about the
    charge.  Used only to check that the separable route gives the same
    screen.  Returns c (ordered x fastest)."""
    d = q - 2
    nodes = interior_basis_nodes(q)
    xq, wq = fe1d.gauss_legendre(q + 4)
    psi = fe1d.lagrange(nodes, xq)[:, 1:q]
    nb = q - 1
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
