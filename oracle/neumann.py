"""The method with a homogeneous Neumann boundary (oracle; test
infrastructure, not part of the product).

Section 2.6 ("Alternate boundary conditions") notes that the adjustment of
eq. bcadjust carries over to Neumann conditions, with the usual constraint
for the non-uniqueness of the pure Neumann problem.  With dPhi/dn = 0 on
the faces of V = [0, L]^3 (an insulating box) the mesh potential must have
the normal derivative -dPhi_sr/dn there, which enters the weak form as the
surface load

    t_m = - sum over the boundary faces F of int_F dPhi_sr/dn u_m dS,

Phi_sr on a face of element E being the near sum of E's (cut) near block
minus its screen potential Psi_E (the tables' order-p field, differentiated
exactly).  The load b + t is projected onto the compatible subspace
(b + t <- b + t - (1^T (b + t) / V) M 1, as for the periodic case) and the
singular system K phi = b + t is solved on every node of the box by fast
diagonalisation of the box pencil with the constant mode dropped (gauge
int phi = 0).  The potential is defined up to a constant; the charges must
be neutral (the flux of the field through the faces is -4 pi sum Q).

The face integrals use a tensor Gauss-Legendre rule of NQ points per
direction on each element face (exact for the table part, which is a
polynomial of degree 2 p on the face for NQ >= p + 1; the pair part
1/r^3-like is smooth for charges at least half an element from the face).

Ground truth: even reflections of every charge in the three coordinate
planes (8 charges of the same sign per charge in [0, 2L)^3), whose
2L-periodic potential is even about every face, so its normal derivative
vanishes there; the image set is neutral with zero dipole moment when the
charges are (`image_ewald`).  Potentials agree up to a constant; the
energy 1/2 sum Q Phi of a neutral set does not depend on it.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from . import dirichlet, ewald, fe1d, fep3m, screens, tables

NQ = 10   # Gauss-Legendre points per direction on an element face

_EIG: dict = {}


def boundary_faces(n):
    """Element faces on the boundary: (element index (ex, ey, ez), axis a,
    side s) with s = 0 for the face at x_a = 0 and 1 for x_a = n."""
    out = []
    for a in range(3):
        for s in (0, 1):
            for j in range(n):
                for i in range(n):
                    e = [0, 0, 0]
                    t = [c for c in range(3) if c != a]
                    e[a] = 0 if s == 0 else n - 1
                    e[t[0]], e[t[1]] = i, j
                    out.append((tuple(e), a, s))
    return out


def surface_load(e, e_lin, u, Q, C, T, n, p, n_sr):
    """t_m = - sum_F int_F dPhi_sr/dn u_m dS (element units) on the box
    nodes."""
    P = p * n + 1
    t = np.zeros((P, P, P))
    nodes = fe1d.gll_nodes(p)
    xq, wq = fe1d.gauss_legendre(NQ)
    Lq = fe1d.lagrange(nodes, xq)                     # (NQ, p+1)
    order, start = dirichlet._sorted(e_lin, n)
    y = e + 0.5 + u
    faces = boundary_faces(n)
    elems = np.array([f[0][0] + n * (f[0][1] + n * f[0][2]) for f in faces])
    uE, inv = np.unique(elems, return_inverse=True)
    Psi = dirichlet.near_field(C, T, n, n_sr, uE).reshape(len(uE), p + 1, p + 1, p + 1)   # [z, y, x]
    end = np.array([-0.5, 0.5])
    Lend = fe1d.lagrange(nodes, end)                  # values at the element ends
    Dend = fe1d.lagrange_deriv(nodes, end)            # derivatives at the element ends
    for fi, (ec, a, s) in enumerate(faces):
        tg = [c for c in range(3) if c != a]          # tangential axes (lower first)
        sign = -1.0 if s == 0 else 1.0                # outward normal along axis a
        # quadrature points on the face (element units, global)
        X = np.zeros((NQ, NQ, 3))
        X[:, :, a] = 0.0 if s == 0 else float(n)
        X[:, :, tg[0]] = (ec[tg[0]] + 0.5 + xq)[None, :]
        X[:, :, tg[1]] = (ec[tg[1]] + 0.5 + xq)[:, None]
        # pair part: n . grad_x sum_j Q_j / |x - y_j| = -sum_j Q_j n.(x - y_j) / r^3
        js = dirichlet.near_sources(elems[fi], n, n_sr, order, start)
        dv = X[:, :, None, :] - y[js][None, None, :, :]
        r = np.sqrt(np.sum(dv * dv, axis=3))
        dn_pair = -sign * np.sum(Q[js][None, None, :] * dv[:, :, :, a] / r**3, axis=2)
        # table part: n . grad Psi_E, exact from the nodal values
        ps = Psi[inv[fi]]                              # [kz, ky, kx]
        # move axis a to the front, tangential axes after: (k_a, k_t1, k_t0)
        perm = {0: (2, 0, 1), 1: (1, 0, 2), 2: (0, 1, 2)}[a]
        psa = np.transpose(ps, perm)                  # [k_a, k_t1, k_t0]
        dnorm = sign * np.einsum("a,abc->bc", Dend[s], psa)        # [k_t1, k_t0]
        dn_tab = np.einsum("ib,jc,bc->ij", Lq, Lq, dnorm)          # at (t1 point i, t0 point j)
        flux = (dn_pair - dn_tab) * wq[:, None] * wq[None, :]      # dPhi_sr/dn times weights, [t1, t0]
        loc = -np.einsum("ij,ib,jc->bc", flux, Lq, Lq)             # [k_t1, k_t0]
        g = [0, 0, 0]
        g[a] = 0 if s == 0 else P - 1
        for kb in range(p + 1):
            for kc in range(p + 1):
                g[tg[1]] = p * ec[tg[1]] + kb
                g[tg[0]] = p * ec[tg[0]] + kc
                t[g[2], g[1], g[0]] += loc[kb, kc]
    return t


def _box_eig(p, n):
    key = (p, n)
    if key not in _EIG:
        K1, M1 = fe1d.dirichlet_matrices(p, n)         # non-periodic assembly on all p n + 1 nodes
        lam, V = scipy.linalg.eigh(K1, M1)
        _EIG[key] = (K1, M1, lam, V)
    return _EIG[key]


def solve(f, p, n):
    """phi = K^+ f on all box nodes (f compatible), int phi = 0."""
    _, _, lam, V = _box_eig(p, n)
    y = fe1d.kron_apply(V.T, V.T, V.T, f)
    D = lam[:, None, None] + lam[None, :, None] + lam[None, None, :]
    D[0, 0, 0] = np.inf                                # the constant mode (lam[0] = 0)
    return fe1d.kron_apply(V, V, V, y / D)


def project_compatible(f, p, n):
    _, M1, _, _ = _box_eig(p, n)
    w1 = M1.sum(axis=1)
    return f - f.sum() / float(n) ** 3 * np.einsum("k,j,i->kji", w1, w1, w1)


def run(x, Q, params: fep3m.Params, targets=None, stages=False):
    """Phi (up to a constant) at `targets` and U for the insulating box."""
    if params.support != "one":
        raise ValueError("the box form takes the one-element screens")
    x = np.asarray(x, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    fep3m.check_neutral(Q)
    n, p, q, d, n_sr = params.n, params.p, params.q, params.d, params.n_sr
    if n < 2 * n_sr + 1:
        raise ValueError("mesh too coarse for the near block")
    e, e_lin, u = dirichlet.bin_box(x, params.L, n)
    C = screens.element_moments(e_lin, u, Q, n ** 3, d)
    T = tables.screen_tables(p, q, n_sr, params.B, params.table_bc, "one")
    b = dirichlet.load_vector(C, n, p, q)
    t = surface_load(e, e_lin, u, Q, C, T, n, p, n_sr)
    f = project_compatible(b + t, p, n)
    phi = solve(f, p, n)
    all_targets = targets is None
    targets = np.arange(len(Q)) if all_targets else np.asarray(targets)
    uel, inv = np.unique(e_lin[targets], return_inverse=True)
    phiE = dirichlet.element_phi(phi, p, n, uel)
    PsiE = dirichlet.near_field(C, T, n, n_sr, uel)
    Phi_m = np.sum((phiE - PsiE)[inv] * fep3m.basis_values(p, u[targets]), axis=1)
    Phi_p = dirichlet.pair_potential(e, e_lin, u, Q, n, n_sr, targets)
    h = params.h
    Phi = (Phi_p + Phi_m) / h
    out = {"Phi": Phi}
    if all_targets:
        out["U"] = 0.5 * float(np.sum(Q * Phi))
    if stages:
        out.update(e=e, e_lin=e_lin, u=u, C=C, b=b, t=t, f=f, phi=phi, Phi_m=Phi_m / h, Phi_p=Phi_p / h)
    return out


def image_charges(x, Q, L):
    """The 8 even images of every charge in [0, 2L)^3 (same sign)."""
    X, QQ = dirichlet.image_charges(x, Q, L)
    return X, np.repeat(Q, 8)


def image_ewald(x, Q, L=1.0, targets=None, points=None, alpha=None, nimg=2, mmax=8):
    """Potential of the insulating box (the gauge of the tin-foil Ewald sum
    of the image set) at the charges or at `points`."""
    X, QQ = image_charges(x, Q, L)
    L2 = 2.0 * L
    alpha = 5.0 / L2 if alpha is None else alpha
    if points is not None:
        Pp = np.asarray(points, dtype=np.float64)
        Xall = np.concatenate([X, Pp])
        Qall = np.concatenate([QQ, np.zeros(len(Pp))])
        t = np.arange(len(X), len(Xall))
        return ewald.ewald(Xall, Qall, L=L2, alpha=alpha, nimg=nimg, mmax=mmax, targets=t)["Phi"]
    N = len(Q)
    t = 8 * (np.arange(N) if targets is None else np.asarray(targets))
    return ewald.ewald(X, QQ, L=L2, alpha=alpha, nimg=nimg, mmax=mmax, targets=t)["Phi"]


def energy_forces(x, Q, params: fep3m.Params):
    """U, F and dU/dQ of the insulating-box method (every charge a target)
    by the adjoint.  In element units, with G the assembled deposit and
    lambda = K^+ G (the gauge-fixed pseudo-inverse; its mean vanishes, so
    the compatibility projection drops out of the adjoint):

      U_m = 1/2 <G, phi> - 1/2 sum_E <g_E, Psi_E>,  <G, phi> = <lambda, b + t>.

    The surface load t depends on the moments (the faces' screen fields) and
    on the positions (the faces' near sums).  With Lam_q = lambda at the
    face's Gauss point x_q and w_q its weight:
      A[E][a] += sum_F sum_m h_F[m] T_a[e(F) - E][m],
                 h_F[m] = sum_q w_q Lam_q dn u_m(x_q)
      dU_hat/dg_i += 1/2 Q_i sum_F sum_q w_q Lam_q (-n / r^3 + 3 (n.d) d / r^5)
      dU_hat/dQ_i += 1/2 sum_F sum_q w_q Lam_q (n.d) / r^3,   d = x_q - g_i,
    F over the boundary faces whose element's near block holds the charge
    (or E); the rest as in the periodic method (near block cut at the
    faces)."""
    from . import adjoint

    x = np.asarray(x, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    n, p, q, d, n_sr, h = params.n, params.p, params.q, params.d, params.n_sr, params.h
    fw = run(x, Q, params, stages=True)
    e, e_lin, u, C, phi = fw["e"], fw["e_lin"], fw["u"], fw["C"], fw["phi"]
    T = tables.screen_tables(p, q, n_sr, params.B, params.table_bc, "one")
    allE = np.arange(n**3)
    W = dirichlet.element_phi(phi, p, n, allE) - dirichlet.near_field(C, T, n, n_sr, allE)
    gE = adjoint.element_deposit(e_lin, u, Q, n, p)
    G = dirichlet.assemble(gE, n, p)
    lam = solve(project_compatible(G, p, n), p, n)
    g1 = screens.load_weights(p, q, "one")
    A_exp = screens.moment_exponents(d)
    Gs = np.stack([np.einsum("k,j,i->kji", g1[az], g1[ay], g1[ax]).ravel() for (ax, ay, az) in A_exp])
    A = 4.0 * math.pi * dirichlet.element_phi(lam, p, n, allE) @ Gs.T
    offs = tables.offsets(n_sr)
    ex, ey, ez = allE % n, (allE // n) % n, allE // (n * n)
    for iD, (Dx, Dy, Dz) in enumerate(offs):
        sx, sy, sz = ex + Dx, ey + Dy, ez + Dz
        ok = (sx >= 0) & (sx < n) & (sy >= 0) & (sy < n) & (sz >= 0) & (sz < n)
        src = sx[ok] + n * (sy[ok] + n * sz[ok])
        A[ok] -= gE[src] @ T[:, iD, :].T
    # face terms
    nodes = fe1d.gll_nodes(p)
    xq, wq = fe1d.gauss_legendre(NQ)
    Lq = fe1d.lagrange(nodes, xq)
    Dend = fe1d.lagrange_deriv(nodes, np.array([-0.5, 0.5]))
    y = e + 0.5 + u
    lamE = dirichlet.element_phi(lam, p, n, allE).reshape(n**3, p + 1, p + 1, p + 1)   # [z, y, x]
    dU_face = np.zeros((len(Q), 3))
    dQ_face = np.zeros(len(Q))
    for (ec, a, s) in boundary_faces(n):
        E = ec[0] + n * (ec[1] + n * ec[2])
        tg = [c for c in range(3) if c != a]
        sign = -1.0 if s == 0 else 1.0
        perm = {0: (2, 0, 1), 1: (1, 0, 2), 2: (0, 1, 2)}[a]
        la = np.transpose(lamE[E], perm)[0 if s == 0 else p]       # face nodes [k_t1, k_t0]
        Lam = np.einsum("ib,jc,bc->ij", Lq, Lq, la)                # lambda at the face points
        Lw = Lam * wq[:, None] * wq[None, :]
        # h_F[m] = sum_q w_q Lam_q dn u_m(x_q), m over the element's nodes [k_a, k_t1, k_t0]
        hF = sign * np.einsum("ij,ib,jc,k->kbc", Lw, Lq, Lq, Dend[s])
        hm = np.transpose(hF, np.argsort(perm)).reshape(-1)        # back to [z, y, x], x fastest
        for iD, (Dx, Dy, Dz) in enumerate(offs):
            sx, sy, sz = ec[0] - Dx, ec[1] - Dy, ec[2] - Dz
            if 0 <= sx < n and 0 <= sy < n and 0 <= sz < n:
                A[sx + n * (sy + n * sz)] += T[:, iD, :] @ hm
        # charges whose element lies in the face element's near block
        near = np.nonzero(np.all(np.abs(e - np.array(ec)[None, :]) <= n_sr, axis=1))[0]
        if len(near) == 0:
            continue
        X = np.zeros((NQ, NQ, 3))
        X[:, :, a] = 0.0 if s == 0 else float(n)
        X[:, :, tg[0]] = (ec[tg[0]] + 0.5 + xq)[None, :]
        X[:, :, tg[1]] = (ec[tg[1]] + 0.5 + xq)[:, None]
        dv = X[None, :, :, :] - y[near][:, None, None, :]        # (k, NQ, NQ, 3)
        r = np.sqrt(np.sum(dv * dv, axis=3))
        nd = sign * dv[..., a]
        nvec = np.zeros(3)
        nvec[a] = sign
        gterm = -nvec[None, None, None, :] / r[..., None] ** 3 + 3.0 * (nd / r**5)[..., None] * dv
        dU_face[near] += 0.5 * Q[near][:, None] * np.einsum("ij,kijc->kc", Lw, gterm)
        dQ_face[near] += 0.5 * np.einsum("ij,kij->k", Lw, nd / r**3)
    grad_v = adjoint.basis_gradients(p, u)
    grad_a = adjoint.monomial_gradients(u, d)
    mesh_grad = 0.5 * Q[:, None] * (np.einsum("nkm,nm->nk", grad_v, W[e_lin])
                                    + np.einsum("nka,na->nk", grad_a, A[e_lin]))
    dUp = dirichlet._pair_forces(e, e_lin, u, Q, n, n_sr)
    dU = dUp + mesh_grad + dU_face
    mono = np.prod(u[:, None, :] ** A_exp[None, :, :], axis=2)
    dUdQ = (fw["Phi_p"] * h + 0.5 * fw["Phi_m"] * h + 0.5 * np.sum(A[e_lin] * mono, axis=1) + dQ_face) / h
    return {"U": fw["U"], "Phi": fw["Phi"], "F": -dU / h**2, "dUdQ": dUdQ, "A": A, "lam": lam}
