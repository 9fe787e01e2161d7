"""Analytic gradients of the discrete FE-P3M energy (oracle).

The paper evaluates potentials only and notes that its operators are not
symmetric (no exact momentum conservation) and that the C^0 basis gives no
straightforward analytic derivative at element faces (Section 5).  Inside
elements, however, every stage of the discrete method is smooth, so the
energy U = 1/2 sum Q_i Phi_i of the method as implemented has exact
derivatives there.  In element units (g = position / h, U_hat = h U):

  pair part   U_p = 1/2 sum_i sum_{j near i, j != i} Q_i Q_j / r_ij
              dU_p/dg_i = sum_j Q_i Q_j (g_j - g_i) / r_ij^3
  mesh part   U_m = 1/2 sum_E <g_E, phi_E - Psi_E>,
              g_E[m] = sum_{i in E} Q_i u_m(u_i)          (charge deposit)
              dU_m/dg_i = 1/2 Q_i [ sum_m W_E[m] grad u_m(u_i)
                                    + sum_a A[E][a] grad u^a(u_i) ],
              A[E][a] = 4 pi <lambda_E, G_a> - sum_D <g_{E+D}, T_a[D]>,
              lambda = (gauge) K^+ (compatible part of) assemble(g)
  charges     dU/dQ_i = Phi_p_i + 1/2 Phi_m_i + 1/2 sum_a A[E_i][a] u_i^a

Physical: F = -(1/h^2) dU_hat/dg, dU/dQ = (1/h) dU_hat/dQ.
"""
from __future__ import annotations

import math

import numpy as np

from . import fe1d, fep3m, mesh, screens, tables


def basis_gradients(p, u):
    """grad u_m(u_i): (N, 3, (p+1)^3), flattened x fastest."""
    nodes = fe1d.gll_nodes(p)
    L = [fe1d.lagrange(nodes, u[:, k]) for k in range(3)]
    D = [fe1d.lagrange_deriv(nodes, u[:, k]) for k in range(3)]
    gx = np.einsum("nk,nj,ni->nkji", L[2], L[1], D[0]).reshape(len(u), -1)
    gy = np.einsum("nk,nj,ni->nkji", L[2], D[1], L[0]).reshape(len(u), -1)
    gz = np.einsum("nk,nj,ni->nkji", D[2], L[1], L[0]).reshape(len(u), -1)
    return np.stack([gx, gy, gz], axis=1)


def monomial_gradients(u, d):
    """grad (u^a) for a in {0..d}^3 (x fastest): (N, 3, (d+1)^3)."""
    A = screens.moment_exponents(d)
    out = np.zeros((len(u), 3, len(A)))
    for ia, a in enumerate(A):
        for k in range(3):
            if a[k] == 0:
                continue
            t = a[k] * u[:, k] ** (a[k] - 1)
            for j in range(3):
                if j != k:
                    t = t * u[:, j] ** a[j]
            out[:, k, ia] = t
    return out


def element_deposit(e_lin, u, Q, n, p):
    """g_E[m] = sum_{i in E} Q_i u_m(u_i): (n^3, (p+1)^3)."""
    vals = fep3m.basis_values(p, u) * Q[:, None]
    g = np.zeros((n**3, vals.shape[1]))
    np.add.at(g, e_lin, vals)
    return g


def assemble(gE, n, p):
    """Sum per-element nodal values into the periodic global vector."""
    P = p * n
    q1 = p + 1
    loc = gE.reshape(n, n, n, q1, q1, q1)
    out = np.zeros((P, P, P))
    idx = mesh.element_node_index(p, n)
    for mz in range(q1):
        for my in range(q1):
            for mx in range(q1):
                out[np.ix_(idx[:, mz], idx[:, my], idx[:, mx])] += loc[:, :, :, mz, my, mx]
    return out


def patch_values(v, p, n, elems, s):
    """Nodal values of the global field on the support patch of each given
    element (s elements per axis around it, (s p + 1)^3 nodes, x fastest)."""
    idx = mesh.support_node_index(p, n, s)
    ex, ey, ez = elems % n, (elems // n) % n, elems // (n * n)
    out = v[idx[ez][:, :, None, None], idx[ey][:, None, :, None], idx[ex][:, None, None, :]]
    return out.reshape(len(elems), -1)


def moment_adjoint(lam, gE, T, n, p, q, n_sr, elems=None, support="one"):
    """A[E][a] = 4 pi <lambda on the support of E, G_a> - sum_D <g_{E+D}, T_a[D]>
    for the given elements (default: all)."""
    d = screens.moment_degree(q, support)
    sp = screens.span(support)
    g = screens.load_weights(p, q, support)
    A_exp = screens.moment_exponents(d)
    E = np.arange(n**3) if elems is None else np.asarray(elems)
    lamE = patch_values(lam, p, n, E, sp)
    Gs = np.stack([np.einsum("k,j,i->kji", g[az], g[ay], g[ax]).ravel() for (ax, ay, az) in A_exp])
    A1 = 4.0 * math.pi * lamE @ Gs.T
    A2 = np.zeros_like(A1)
    ex, ey, ez = E % n, (E // n) % n, E // (n * n)
    for iD, (Dx, Dy, Dz) in enumerate(tables.offsets(n_sr)):
        src = ((ex + Dx) % n) + n * (((ey + Dy) % n) + n * ((ez + Dz) % n))
        A2 += gE[src] @ T[:, iD, :].T
    return A1 - A2


def pair_forces(e, e_lin, u, Q, n, n_sr, targets=None):
    """dU_p/dg_i (element units) for the target charges (default: all)."""
    order = np.argsort(e_lin, kind="stable")
    counts = np.bincount(e_lin, minlength=n**3)
    start = np.concatenate([[0], np.cumsum(counts)])
    targets = np.arange(len(Q)) if targets is None else np.asarray(targets)
    out = np.zeros((len(targets), 3))
    tgt_e = e_lin[targets]
    for E in np.unique(tgt_e):
        sel = np.nonzero(tgt_e == E)[0]
        ti = targets[sel]
        ex, ey, ez = E % n, (E // n) % n, E // (n * n)
        srcs, shifts = [], []
        for (Dx, Dy, Dz) in tables.offsets(n_sr):
            S = ((ex + Dx) % n) + n * (((ey + Dy) % n) + n * ((ez + Dz) % n))
            js = order[start[S]:start[S + 1]]
            srcs.append(js)
            shifts.append(np.tile([Dx, Dy, Dz], (len(js), 1)))
        js = np.concatenate(srcs)
        sh = np.concatenate(shifts).astype(np.float64)
        dvec = sh[None, :, :] + u[js][None, :, :] - u[ti][:, None, :]     # g_j - g_i
        r = np.sqrt(np.sum(dvec * dvec, axis=2))
        self_mask = js[None, :] == ti[:, None]
        r[self_mask] = np.inf
        w = Q[ti][:, None] * Q[js][None, :] / r**3
        out[sel] = np.einsum("ij,ijk->ik", w, dvec)
    return out


def energy_forces(x, Q, params: fep3m.Params, targets=None):
    """U, F (N,3) and dU/dQ (N) of the discrete method, plus Phi.  With
    `targets`, Phi, F and dU/dQ are evaluated for those charges only (the
    mesh solves and deposits still cover every charge) and U is omitted."""
    x = np.asarray(x, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    n, p, q, d, h = params.n, params.p, params.q, params.d, params.h
    all_targets = targets is None
    tgt = np.arange(len(Q)) if all_targets else np.asarray(targets)
    fw = fep3m.run(x, Q, params, targets=None if all_targets else tgt, stages=True)
    e, e_lin, u, C, phi = fw["e"], fw["e_lin"], fw["u"], fw["C"], fw["phi"]
    T = tables.screen_tables(p, q, params.n_sr, params.B, params.table_bc, params.support)
    uel, inv = np.unique(e_lin[tgt], return_inverse=True)
    W = fep3m.element_phi(phi, p, n, uel) - fep3m.near_field(C, T, n, params.n_sr, uel)
    gE = element_deposit(e_lin, u, Q, n, p)
    G = mesh.project_compatible(assemble(gE, n, p), p, n)
    lam = mesh.solve_periodic(G, p, n)
    lam = lam - mesh.mean_value(lam, p, n)
    A = moment_adjoint(lam, gE, T, n, p, q, params.n_sr, uel, params.support)
    ut = u[tgt]
    Qt = Q[tgt]
    grad_v = basis_gradients(p, ut)                      # (T,3,M)
    grad_a = monomial_gradients(ut, d)                   # (T,3,(d+1)^3)
    mesh_grad = 0.5 * Qt[:, None] * (np.einsum("nkm,nm->nk", grad_v, W[inv])
                                     + np.einsum("nka,na->nk", grad_a, A[inv]))
    dUp = pair_forces(e, e_lin, u, Q, n, params.n_sr, tgt)
    F = -(dUp + mesh_grad) / h**2
    mono = np.prod(ut[:, None, :] ** screens.moment_exponents(d)[None, :, :], axis=2)
    dUdQ = (fw["Phi_p"] * h + 0.5 * fw["Phi_m"] * h + 0.5 * np.sum(A[inv] * mono, axis=1)) / h
    out = {"Phi": fw["Phi"], "F": F, "dUdQ": dUdQ, "A": A, "lam": lam, "gE": gE, "phi": phi}
    if all_targets:
        out["U"] = fw["U"]
    return out
