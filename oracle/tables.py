"""Near-field screen-potential tables (oracle).

The short-range step subtracts the potential of every screen whose host
element lies in the near block of a target (eq. sc: the screen potential is
a combination, with the screen coefficients, of per-basis-function tables).
Following the Remark of Section 4, each table is the order-p finite element
solution of the Poisson problem for one basis screen, computed on a domain
larger than the part kept, and stored by its order-p nodal values so it can
be combined exactly like the mesh potential.

Here the basis screens are the dual functions R_a = r_ax (x) r_ay (x) r_az
(a in {0..d}^3), so the combined screen of an element with moments C[E][a]
has near-field potential  sum_a C[E][a] T_a .  For each a:

  * domain: B^3 unit elements centred on the source element (B odd); the
    screen covers the source element (one-element support) or the 3^3
    elements around it (27-element support),
  * weak form  K w = 4 pi G_a  (G_a = int u_m R_a),
  * Dirichlet data on the outer nodes: the exact free-space potential of R_a
    (all multipole terms, the Remark's boundary condition taken to all
    orders),
  * solved exactly by fast diagonalisation of the interior 1-D pencil.

T[a, D, m] is w at node m = (mx, my, mz) of the element at offset
D = (Dx, Dy, Dz) in [-n_sr, n_sr]^3 from the source (x fastest in both
indices).  Element units: physical tables are T / h.

The alternative reading (the order-p nodal interpolant of the exact
potential, bc="interp") is kept for comparison against Ewald.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from . import fe1d, potential, screens

_CACHE: dict = {}


def _potential_grid(coef3, coords):
    """Exact potential of the separable density with per-axis polynomial
    coefficients coef3 on the full tensor grid coords^3 -> [z, y, x]."""
    t = np.exp(potential._TAU)
    wt = potential._TAU_W * t * (2.0 / math.sqrt(math.pi))
    Fx = potential._axis_factor(coef3[0], t, coords)
    Fy = potential._axis_factor(coef3[1], t, coords)
    Fz = potential._axis_factor(coef3[2], t, coords)
    T, n = Fx.shape
    ZY = ((Fz * wt[:, None])[:, :, None] * Fy[:, None, :]).reshape(T, n * n)
    return (ZY.T @ Fx).reshape(n, n, n)


def node_coords(p, B):
    """Coordinates of the B*p+1 nodes along one axis of the table box."""
    c = (B - 1) // 2
    g = fe1d.gll_nodes(p)
    xs = [e - c + g[k] for e in range(B) for k in range(p)] + [B - c - 0.5]
    return np.array(xs)


def screen_tables(p=5, q=3, n_sr=3, B=None, bc="exact", support="one"):
    B = 2 * n_sr + 1 + 8 if B is None else B
    key = (p, q, n_sr, B, bc, support)
    if key in _CACHE:
        return _CACHE[key]
    if B % 2 == 0 or B < 2 * n_sr + 3:
        raise ValueError("table box must be odd and larger than the near block")
    d = screens.moment_degree(q, support)
    sp = screens.span(support)
    c = (B - 1) // 2
    S = 2 * n_sr + 1
    nn = B * p + 1
    coords = node_coords(p, B)
    polys = potential.dual_polynomials(q, support)
    g = screens.load_weights(p, q, support)           # (d+1, sp p + 1)
    A = screens.moment_exponents(d)
    Kd, Md = fe1d.dirichlet_matrices(p, B)
    inner = np.arange(1, nn - 1)
    Ki = Kd[np.ix_(inner, inner)]
    Mi = Md[np.ix_(inner, inner)]
    lam, V = scipy.linalg.eigh(Ki, Mi)
    Lsum = lam[:, None, None] + lam[None, :, None] + lam[None, None, :]

    T = np.zeros((len(A), S**3, (p + 1) ** 3))
    for ia, (ax, ay, az) in enumerate(A):
        exact = _potential_grid([polys[ax], polys[ay], polys[az]], coords)
        if bc == "interp":
            w = exact
        else:
            b = np.zeros((nn, nn, nn))
            k0 = p * (c - (sp - 1) // 2)
            sl = slice(k0, k0 + sp * p + 1)
            b[sl, sl, sl] = 4.0 * math.pi * np.einsum("k,j,i->kji", g[az], g[ay], g[ax])
            gext = exact.copy()
            gext[1:-1, 1:-1, 1:-1] = 0.0
            rhs = b - fe1d.stiffness_apply(Kd, Md, gext)
            r = rhs[1:-1, 1:-1, 1:-1]
            y = fe1d.kron_apply(V.T, V.T, V.T, r) / Lsum
            w = gext
            w[1:-1, 1:-1, 1:-1] = fe1d.kron_apply(V, V, V, y)
        for iD, (Dx, Dy, Dz) in enumerate(_offsets(n_sr)):
            z0, y0, x0 = p * (c + Dz), p * (c + Dy), p * (c + Dx)
            blk = w[z0:z0 + p + 1, y0:y0 + p + 1, x0:x0 + p + 1]
            T[ia, iD] = blk.reshape(-1)
    _CACHE[key] = T
    return T


def _offsets(n_sr):
    r = range(-n_sr, n_sr + 1)
    return [(dx, dy, dz) for dz in r for dy in r for dx in r]


def offsets(n_sr):
    return np.array(_offsets(n_sr), dtype=np.int64)
