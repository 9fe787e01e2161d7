"""The whole FE-P3M method, stage by stage (oracle).

Follows Algorithm 1 of the paper (charge assignment, mesh solve, evaluation
of the smooth potential, short-range potential) for a periodic cube
[0, L]^3 meshed by n^3 elements of size h = L/n, with polynomial screens
of degree q (one-element support, Section 5, or the 27-element support of
Section 2.1) and an order p = q + 2 mesh.

Element units (h = 1) are used throughout; physical potentials are the
element-unit values divided by h.

Stages (names used by the tests):
  bin     e = floor(n * frac(x/L)) clamped to n-1, u = n*frac(x/L) - e - 1/2
  C       per-element screen moments  C[E][a] = sum_{j in E} Q_j u_j^a
  b       load vector (projected compatible)
  phi     periodic FE potential with int phi = 0
  Psi     near screen field  Psi_E = sum_D sum_a T_a[D] C[E - D][a]
          (D over the (2 n_sr + 1)^3 block; D = 0 is the self term)
  Phi_m   sum_m (phi_E - Psi_E)[m] u_m(u_i)            (eq. evalsmooth)
  Phi_p   sum_D sum_{j in E_i + D, j != i} Q_j / |D + u_j - u_i|
  Phi     (Phi_p + Phi_m) / h ;  U = 1/2 sum Q_i Phi_i (eq. potentialenergy)
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import fe1d, mesh, screens, tables


@dataclass
class Params:
    L: float
    n: int
    q: int = 3
    n_sr: int = 3
    B: int | None = None
    table_bc: str = "exact"
    support: str = "one"

    @property
    def p(self):
        return self.q + 2

    @property
    def d(self):
        return screens.moment_degree(self.q, self.support)

    @property
    def h(self):
        return self.L / self.n


def bin_particles(x, L, n):
    """Periodic wrap and element binning.  A point on a face belongs to the
    element on its + side; the index is clamped to n-1 for points that
    round onto L."""
    s = x / L
    s = s - np.floor(s)
    t = s * n
    e = np.floor(t)
    e = np.minimum(e, n - 1)
    u = t - e - 0.5
    e = e.astype(np.int64)
    e_lin = e[:, 0] + n * (e[:, 1] + n * e[:, 2])
    return e, e_lin, u


def check_neutral(Q, rtol=1e-10):
    tot = float(np.sum(Q))
    scale = float(np.sum(np.abs(Q)))
    if abs(tot) > rtol * max(scale, 1e-300):
        raise ValueError(f"charges are not neutral: sum Q = {tot}")


def element_phi(phi, p, n, elems):
    """Local (p+1)^3 nodal values of the global field on the given elements
    (linear element ids), flattened x fastest."""
    idx = mesh.element_node_index(p, n)
    ex = elems % n
    ey = (elems // n) % n
    ez = elems // (n * n)
    out = phi[idx[ez][:, :, None, None], idx[ey][:, None, :, None], idx[ex][:, None, None, :]]
    return out.reshape(len(elems), -1)


def near_field(C, T, n, n_sr, elems):
    """Psi_E for the given target elements: sum over offsets D and moments a
    of T[a, D, :] * C[(E - D) mod n, a]."""
    offs = tables.offsets(n_sr)
    ex = elems % n
    ey = (elems // n) % n
    ez = elems // (n * n)
    out = np.zeros((len(elems), T.shape[2]))
    for iD, (Dx, Dy, Dz) in enumerate(offs):
        src = ((ex - Dx) % n) + n * (((ey - Dy) % n) + n * ((ez - Dz) % n))
        out += C[src] @ T[:, iD, :]
    return out


def basis_values(p, u):
    """u_m(u_i) for all particles: the order-p GLL Lagrange basis of the
    element evaluated at the local offset, flattened x fastest: (N, (p+1)^3)."""
    nodes = fe1d.gll_nodes(p)
    lx = fe1d.lagrange(nodes, u[:, 0])
    ly = fe1d.lagrange(nodes, u[:, 1])
    lz = fe1d.lagrange(nodes, u[:, 2])
    return np.einsum("nk,nj,ni->nkji", lz, ly, lx).reshape(len(u), -1)


def pair_potential(e, e_lin, u, Q, n, n_sr, targets):
    """Singular near sum in element units for the target particles."""
    order = np.argsort(e_lin, kind="stable")
    counts = np.bincount(e_lin, minlength=n ** 3)
    start = np.concatenate([[0], np.cumsum(counts)])
    offs = tables.offsets(n_sr)
    out = np.zeros(len(targets))
    tgt_e = e_lin[targets]
    for E in np.unique(tgt_e):
        sel = np.nonzero(tgt_e == E)[0]
        ti = targets[sel]
        ex, ey, ez = E % n, (E // n) % n, E // (n * n)
        srcs, shifts = [], []
        for (Dx, Dy, Dz) in offs:
            S = ((ex + Dx) % n) + n * (((ey + Dy) % n) + n * ((ez + Dz) % n))
            js = order[start[S]:start[S + 1]]
            srcs.append(js)
            shifts.append(np.tile([Dx, Dy, Dz], (len(js), 1)))
        js = np.concatenate(srcs)
        sh = np.concatenate(shifts).astype(np.float64)
        dvec = sh[None, :, :] + u[js][None, :, :] - u[ti][:, None, :]
        r = np.sqrt(np.sum(dvec * dvec, axis=2))
        self_mask = js[None, :] == ti[:, None]
        r[self_mask] = np.inf
        out[sel] = np.sum(Q[js][None, :] / r, axis=1)
    return out


def ewald_constant(u, Q, params: Params):
    """Constant c with  Phi + c  comparable to the tin-foil Ewald potential.

    For a neutral set of compact charge distributions the zero-mean
    periodic potential differs from the tin-foil Ewald (image-sum) potential
    by a constant set by the distributions' second moments.  Each point
    charge minus its screen is such a distribution, with second moment
    -s_j, s_j = int |xi - x_j|^2 rho_j(xi) dxi, so (with int phi = 0)

        c = -(2 pi / 3 V) sum_j Q_j s_j .

    Per axis the screen's second moment about its charge is
    m2 - 2 delta m1 + delta^2 with m_k = sum_l delta^l int x^k r_l: for
    d >= 2 it is zero (the x^2 moment is cancelled); for d = 1 it is
    mu_0 - delta^2 (mu_0 = int x^2 r_0), and mu_0 drops out by neutrality,
    leaving c = (2 pi / 3V) sum_j Q_j |delta_j|^2.  Physical units."""
    h = params.h
    V = params.L ** 3
    m1c, m2c = screens.axis_moment_coefficients(params.q, params.support)
    d = len(m1c) - 1
    pw = u[:, :, None] ** np.arange(d + 1)[None, None, :]
    s2 = np.sum(pw @ m2c - 2.0 * u * (pw @ m1c) + u**2, axis=1)   # per charge, element units
    return -2.0 * math.pi / (3.0 * V) * float(np.sum(Q * s2)) * h * h


def run(x, Q, params: Params, targets=None, stages=False):
    """Evaluate Phi at `targets` (default: all particles) and U (only when
    all particles are targets)."""
    x = np.asarray(x, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    check_neutral(Q)
    n, p, q, d = params.n, params.p, params.q, params.d
    if n < 2 * params.n_sr + 1:
        raise ValueError("mesh too coarse for the near block")
    e, e_lin, u = bin_particles(x, params.L, n)
    C = screens.element_moments(e_lin, u, Q, n ** 3, d)
    b = mesh.load_vector(C, n, p, q, params.support)
    b = mesh.project_compatible(b, p, n)
    phi = mesh.solve_periodic(b, p, n)
    phi = phi - mesh.mean_value(phi, p, n)
    T = tables.screen_tables(p, q, params.n_sr, params.B, params.table_bc, params.support)
    all_targets = targets is None
    targets = np.arange(len(Q)) if all_targets else np.asarray(targets)
    te = e_lin[targets]
    uel, inv = np.unique(te, return_inverse=True)
    phiE = element_phi(phi, p, n, uel)
    PsiE = near_field(C, T, n, params.n_sr, uel)
    basis = basis_values(p, u[targets])
    Phi_m = np.sum((phiE - PsiE)[inv] * basis, axis=1)
    Phi_p = pair_potential(e, e_lin, u, Q, n, params.n_sr, targets)
    h = params.h
    Phi = (Phi_p + Phi_m) / h
    out = {"Phi": Phi}
    if all_targets:
        out["U"] = 0.5 * float(np.sum(Q * Phi))
    if stages:
        out.update(e=e, e_lin=e_lin, u=u, C=C, b=b, phi=phi, Psi_elems=uel,
                   Psi=PsiE, phiE=phiE, Phi_m=Phi_m / h, Phi_p=Phi_p / h)
    return out
