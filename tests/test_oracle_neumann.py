"""Pins of the oracle's insulating-box form (Section 2.6 with a homogeneous
Neumann condition): the even-image ground truth has zero normal field on
the faces; the pure-Neumann solve reproduces a polynomial with zero normal
derivatives; the surface load's pair part carries Gauss's law and its table
part the screen's flux; the whole method against the ground truth, with and
without the surface load."""
import math

import numpy as np
import pytest

from oracle import dirichlet as odir
from oracle import fe1d, fep3m, neumann as oneu, screens, tables


def test_image_field_is_tangential_on_faces():
    rng = np.random.default_rng(3)
    N = 10
    x = rng.uniform(0.1, 0.9, (N, 3))
    Q = rng.uniform(-1, 1, N)
    Q -= Q.mean()
    dlt = 1e-5
    for a in range(3):
        for side in (0.0, 1.0):
            pts = rng.uniform(0.05, 0.95, (6, 3))
            pts[:, a] = side
            plus, minus = pts.copy(), pts.copy()
            plus[:, a] += dlt
            minus[:, a] -= dlt
            d = (oneu.image_ewald(x, Q, points=plus) - oneu.image_ewald(x, Q, points=minus)) / (2 * dlt)
            b = (a + 1) % 3                    # a tangential direction: its derivative does not vanish
            plus[:, a] -= dlt
            minus[:, a] += dlt
            plus[:, b] += dlt
            minus[:, b] -= dlt
            dt = (oneu.image_ewald(x, Q, points=plus) - oneu.image_ewald(x, Q, points=minus)) / (2 * dlt)
            assert np.max(np.abs(d)) < 1e-5 * np.max(np.abs(dt)), (a, side, d, dt)


@pytest.mark.parametrize("p,n", [(3, 2), (5, 3)])
def test_neumann_solve_reproduces_polynomial(p, n):
    """u = w(x) w(y) w(z), w(s) = s^2 (3 n - 2 s) (w'(0) = w'(n) = 0, cubic):
    with the load M f of f = -lap u the gauge-fixed solve returns u minus its
    mean at every node."""
    pos = odir.node_positions(p, n)
    w = pos**2 * (3 * n - 2 * pos)
    w2 = 6.0 * n - 12.0 * pos
    u = np.einsum("k,j,i->kji", w, w, w)
    f = -(np.einsum("k,j,i->kji", w, w, w2) + np.einsum("k,j,i->kji", w, w2, w)
          + np.einsum("k,j,i->kji", w2, w, w))
    _, M1 = fe1d.dirichlet_matrices(p, n)
    b = fe1d.kron_apply(M1, M1, M1, f)
    assert abs(b.sum()) < 1e-9 * np.abs(b).sum()          # compatible: the flux of grad u is zero
    phi = oneu.solve(oneu.project_compatible(b, p, n), p, n)
    w1 = M1.sum(axis=1)
    mean_u = np.einsum("kji,k,j,i->", u, w1, w1, w1) / n**3
    np.testing.assert_allclose(phi, u - mean_u, rtol=0, atol=1e-10 * np.max(np.abs(u)))


def _center_charge(n):
    """One charge in the central element of an odd mesh: every boundary
    face's near block holds it when n <= 2 n_sr + 1."""
    x = np.array([[0.5 + 0.13 / n, 0.5 - 0.21 / n, 0.5 + 0.05 / n]])
    return x, np.array([0.7])


def test_surface_load_pair_part_is_gauss_law():
    """With the tables switched off the surface load is the quadrature of
    -dQ/r/dn over the faces: its total is 4 pi Q (Gauss's law)."""
    n, p, nsr = 7, 5, 3
    x, Q = _center_charge(n)
    e, e_lin, u = odir.bin_box(x, 1.0, n)
    d = screens.moment_degree(3)
    C = screens.element_moments(e_lin, u, Q, n**3, d)
    T0 = np.zeros_like(tables.screen_tables(p, 3, nsr, None, "exact", "one"))
    t = oneu.surface_load(e, e_lin, u, Q, C, T0, n, p, nsr)
    assert abs(t.sum() - 4 * math.pi * Q[0]) < 1e-9


def test_surface_load_table_part_is_the_screen_flux():
    """With the pair part switched off (no charges in the near sums, the
    moments kept) the surface load is the flux of the screen's table field
    through the faces: -4 pi Q for a screen inside the box, to the tables'
    accuracy."""
    n, p, nsr = 7, 5, 3
    x, Q = _center_charge(n)
    e, e_lin, u = odir.bin_box(x, 1.0, n)
    C = screens.element_moments(e_lin, u, Q, n**3, screens.moment_degree(3))
    T = tables.screen_tables(p, 3, nsr, None, "exact", "one")
    t = oneu.surface_load(e, e_lin, u, np.zeros_like(Q), C, T, n, p, nsr)
    assert abs(t.sum() + 4 * math.pi * Q[0]) < 1e-4 * 4 * math.pi * abs(Q[0])


def _layer(N, seed, n, L=1.0):
    rng = np.random.default_rng(seed)
    h = L / n
    x = rng.uniform(0.5 * h, L - 0.5 * h, (N, 3))
    k = N // 2
    ax = rng.integers(0, 3, k)
    side = rng.integers(0, 2, k)
    d = rng.uniform(0.5, 1.0, k) * h
    x[np.arange(k), ax] = np.where(side == 1, L - d, d)
    Q = rng.permutation(np.repeat([1.0, -1.0], N // 2))   # neutral
    return x, Q


def _rel_up_to_constant(a, b):
    c = np.mean(b - a)
    return float(np.linalg.norm(a + c - b) / np.linalg.norm(b - b.mean()))


def test_method_matches_images_and_needs_the_surface_load():
    """The insulating-box method against the even-image sum: the potential
    up to a constant and the energy within the screen's truncation error;
    without the surface load (dPhi_sm/dn = 0 instead of -dPhi_sr/dn) the
    potential is several times worse."""
    N, n = 300, 8
    x, Q = _layer(N, 21, n)
    P = fep3m.Params(L=1.0, n=n)
    ref = oneu.image_ewald(x, Q)
    out = oneu.run(x, Q, P, stages=True)
    e_phi = _rel_up_to_constant(out["Phi"], ref)
    U_ref = 0.5 * float(np.sum(Q * ref))
    e_U = abs(out["U"] - U_ref) / abs(U_ref)
    phi0 = oneu.solve(oneu.project_compatible(out["b"], P.p, n), P.p, n)
    allE = np.unique(out["e_lin"])
    _, inv = np.unique(out["e_lin"], return_inverse=True)
    T = tables.screen_tables(P.p, 3, 3, None, "exact", "one")
    W0 = odir.element_phi(phi0, P.p, n, allE) - odir.near_field(out["C"], T, n, 3, allE)
    Phi0 = out["Phi_p"] + np.sum(W0[inv] * fep3m.basis_values(P.p, out["u"]), axis=1) / P.h
    e0 = _rel_up_to_constant(Phi0, ref)
    print(f"insulating box N={N} n={n}: Phi {e_phi:.3e} (up to a constant), U {e_U:.3e}; "
          f"without the surface load {e0:.3e}")
    assert e_phi < 5e-3 and e_U < 5e-3
    assert e0 > 3 * e_phi


def test_non_neutral_charges_are_refused():
    x, Q = _layer(20, 22, 8)
    Q[0] += 1.0
    with pytest.raises(ValueError):
        oneu.run(x, Q, fep3m.Params(L=1.0, n=8))


def test_insulated_gradients_match_central_differences():
    """Forces and dU/dQ of the insulating box by the adjoint (with the terms
    of the surface load: its dependence on the moments and on the
    positions) equal central differences of the oracle's energy.  dU/dQ is
    checked along neutral directions (dQ_i = -dQ_j), the only ones the
    neutrality constraint allows."""
    N, n = 60, 7
    x, Q = _layer(N, 23, n)
    P = fep3m.Params(L=1.0, n=n)
    out = oneu.energy_forces(x, Q, P)
    h = P.h
    frac = (x / h) % 1.0
    ok = np.nonzero(np.all((frac > 0.1) & (frac < 0.9), axis=1))[0][:6]
    assert len(ok) >= 4
    dx = 1e-6
    scale = np.max(np.abs(out["F"][ok]))
    for i in ok:
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += dx
            xm[i, k] -= dx
            fd = -(oneu.run(xp, Q, P)["U"] - oneu.run(xm, Q, P)["U"]) / (2 * dx)
            assert abs(out["F"][i, k] - fd) < 1e-5 * scale, (i, k, out["F"][i, k], fd)
    j = ok[-1]
    for i in ok[:-1]:
        Qp, Qm = Q.copy(), Q.copy()
        Qp[i] += 1e-6
        Qp[j] -= 1e-6
        Qm[i] -= 1e-6
        Qm[j] += 1e-6
        fdq = (oneu.run(x, Qp, P)["U"] - oneu.run(x, Qm, P)["U"]) / 2e-6
        assert abs((out["dUdQ"][i] - out["dUdQ"][j]) - fdq) < 1e-6 * np.max(np.abs(out["dUdQ"])), (i, fdq)


def test_insulated_forces_against_images():
    N, n = 200, 8
    x, Q = _layer(N, 24, n)
    out = oneu.energy_forces(x, Q, fep3m.Params(L=1.0, n=n))
    X, QQ = oneu.image_charges(x, Q, 1.0)
    from oracle import ewald
    ref = ewald.ewald(X, QQ, L=2.0, alpha=2.5, nimg=2, mmax=8, forces=True, targets=8 * np.arange(N))["F"]
    err = np.linalg.norm(out["F"] - ref) / np.linalg.norm(ref)
    print(f"insulating box forces vs images: {err:.3e}")
    assert err < 1e-2
