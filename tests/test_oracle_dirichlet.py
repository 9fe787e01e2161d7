"""Pins of the oracle's grounded-box form (Section 2.6, eq. bcadjust with
g = 0).  The ground truth (odd images of every charge, Ewald-summed in the
2L-periodic box) is checked against an independent textbook construction:
the eigenfunction expansion of the cube's Green's function in x and y with
the exact one-dimensional Green's function in z.  The finite element solve
with boundary data is checked on polynomials it must reproduce exactly, the
load on the moments it must carry, and the whole method against the ground
truth, with and without the boundary adjustment."""
import math

import numpy as np
import pytest

from oracle import dirichlet as odir
from oracle import fe1d, fep3m, screens


def green_series(x, y, L=1.0, kmax=60):
    """Potential at x of a unit charge at y in the grounded cube [0, L]^3:
    sum over l, m >= 1 of (4 / L^2) sin(l pi x1/L) sin(l pi y1/L)
    sin(m pi x2/L) sin(m pi y2/L) g_lm(x3, y3), with g_lm the Green's function
    of -d^2/dz^2 + kappa^2 on [0, L] with zero ends (times 4 pi):
    4 pi sinh(kappa z<) sinh(kappa (L - z>)) / (kappa sinh(kappa L)).  It
    converges exponentially when x3 != y3."""
    l = np.arange(1, kmax + 1)
    sx = np.sin(l * math.pi * x[0] / L) * np.sin(l * math.pi * y[0] / L)
    sy = np.sin(l * math.pi * x[1] / L) * np.sin(l * math.pi * y[1] / L)
    kap = math.pi * np.sqrt(l[:, None] ** 2 + l[None, :] ** 2) / L
    zl, zg = min(x[2], y[2]), max(x[2], y[2])
    # sinh(a) sinh(b) / sinh(c) with c = a + b + (L - ...) written with exponentials (no overflow)
    a, b = kap * zl, kap * (L - zg)
    g = 4.0 * math.pi * 0.5 * (np.exp(a + b - kap * L) - np.exp(-a + b - kap * L)
                               - np.exp(a - b - kap * L) + np.exp(-a - b - kap * L)) \
        / (kap * (1.0 - np.exp(-2.0 * kap * L)))
    return float(4.0 / L**2 * np.sum(sx[:, None] * sy[None, :] * g))


def test_image_ewald_matches_eigenfunction_series():
    rng = np.random.default_rng(5)
    for _ in range(4):
        y = rng.uniform(0.1, 0.9, 3)
        x = rng.uniform(0.1, 0.9, 3)
        x[2] = y[2] + (0.25 if y[2] < 0.5 else -0.25)      # separated in z: fast convergence
        ref = green_series(x, y)
        got = odir.image_ewald(y[None, :], np.array([1.0]), points=x[None, :])[0]
        assert abs(got - ref) < 1e-9 * abs(ref), (got, ref)


def test_image_ewald_vanishes_on_faces_and_is_reciprocal():
    rng = np.random.default_rng(6)
    N = 12
    x = rng.uniform(0.05, 0.95, (N, 3))
    Q = rng.uniform(-1, 1, N)               # not neutral: the box takes any net charge
    pts = rng.uniform(0, 1, (30, 3))
    for k in range(30):
        pts[k, k % 3] = float(k % 2)       # on the faces x_a = 0 or 1
    phi_face = odir.image_ewald(x, Q, points=pts)
    scale = np.max(np.abs(odir.image_ewald(x, Q)))
    assert np.max(np.abs(phi_face)) < 1e-10 * scale
    a, b = x[0], x[1]
    gab = odir.image_ewald(b[None, :], np.array([1.0]), points=a[None, :])[0]
    gba = odir.image_ewald(a[None, :], np.array([1.0]), points=b[None, :])[0]
    assert abs(gab - gba) < 1e-12 * abs(gab)


@pytest.mark.parametrize("p,n", [(3, 2), (5, 3)])
def test_solve_reproduces_polynomials_with_boundary_data(p, n):
    """u = x^2 y^2 + z (degree 2 per axis, in the order-p space, nonzero on
    the faces): with its boundary values and the exact load M f of
    f = -lap u, the Dirichlet solve returns u at every node."""
    pos = odir.node_positions(p, n)
    Z, Y, X = np.meshgrid(pos, pos, pos, indexing="ij")
    u = X**2 * Y**2 + Z
    f = -(2.0 * Y**2 + 2.0 * X**2)
    _, M1 = fe1d.dirichlet_matrices(p, n)
    b = fe1d.kron_apply(M1, M1, M1, f)
    phiB = np.where(odir.boundary_mask(p, n), u, 0.0)
    phi = odir.solve(b, phiB, p, n)
    np.testing.assert_allclose(phi, u, rtol=0, atol=1e-10 * np.max(np.abs(u)))


def test_load_carries_charge_and_dipole():
    """The screens integrate to their charges and reproduce first moments
    (d >= 1), and the order-p basis sums to one and reproduces x: so
    sum_m b_m = 4 pi sum Q and sum_m b_m x_m = 4 pi sum Q_j x_j."""
    n, p, q = 4, 5, 3
    rng = np.random.default_rng(7)
    x = rng.uniform(0, 1, (40, 3))
    Q = rng.uniform(-1, 1, 40)
    e, e_lin, u = odir.bin_box(x, 1.0, n)
    C = screens.element_moments(e_lin, u, Q, n**3, screens.moment_degree(q))
    b = odir.load_vector(C, n, p, q)
    assert abs(b.sum() - 4 * math.pi * Q.sum()) < 1e-11
    pos = odir.node_positions(p, n)
    y = x * n
    for axis, sl in ((2, (None, None, slice(None))), (1, (None, slice(None), None)), (0, (slice(None), None, None))):
        coord = pos[sl]
        assert abs(np.sum(b * coord) - 4 * math.pi * np.sum(Q * y[:, 2 - axis])) < 1e-10


def test_boundary_values_vanish_away_from_the_faces():
    """Charges more than n_sr elements from every face leave no short-range
    trace on the boundary."""
    n, p = 9, 5
    P = fep3m.Params(L=1.0, n=n)
    rng = np.random.default_rng(8)
    x = rng.uniform(4.0 / n, 5.0 / n, (10, 3))         # the central element
    Q = rng.uniform(-1, 1, 10)
    out = odir.run(x, Q, P, stages=True)
    assert np.max(np.abs(out["phiB"])) == 0.0


def _boundary_layer(N, seed, n, L=1.0):
    """Charges of random sign at least half an element from every face, half
    of them within one element of a face.  (Closer charges have images
    within h of the face, which the order-p mesh potential cannot resolve:
    their error is of order one, a property of the boundary adjustment.)"""
    rng = np.random.default_rng(seed)
    h = L / n
    x = rng.uniform(0.5 * h, L - 0.5 * h, (N, 3))
    k = N // 2
    ax = rng.integers(0, 3, k)
    side = rng.integers(0, 2, k)
    d = rng.uniform(0.5, 1.0, k) * h
    x[np.arange(k), ax] = np.where(side == 1, L - d, d)
    Q = rng.choice([-1.0, 1.0], N)
    return x, Q


def test_method_matches_ground_truth_and_needs_the_boundary_term():
    """The grounded-box method against the image sum: within the one-element
    q = 3 screen's truncation error (a few 1e-3, as for periodic input); the
    same run with zero mesh boundary values (no eq. bcadjust) is an order of
    magnitude worse, since half the charges sit within an element of a
    face."""
    N, n = 300, 8
    x, Q = _boundary_layer(N, 9, n)
    P = fep3m.Params(L=1.0, n=n)
    ref = odir.image_ewald(x, Q)
    out = odir.run(x, Q, P, stages=True)
    err = np.linalg.norm(out["Phi"] - ref) / np.linalg.norm(ref)
    # the same method with phiB = 0
    st = out
    phi0 = odir.solve(st["b"], np.zeros_like(st["phiB"]), P.p, n)
    uel = st["Psi_elems"]
    _, inv = np.unique(st["e_lin"], return_inverse=True)
    phiE0 = odir.element_phi(phi0, P.p, n, uel)
    Phi_m0 = np.sum((phiE0 - st["Psi"])[inv] * fep3m.basis_values(P.p, st["u"]), axis=1) / P.h
    err0 = np.linalg.norm(st["Phi_p"] + Phi_m0 - ref) / np.linalg.norm(ref)
    print(f"grounded box N={N} n={n}: Phi rel RMS {err:.3e}; without the boundary term {err0:.3e}")
    assert err < 5e-3
    assert err0 > 5 * err
    assert abs(out["U"] - 0.5 * np.sum(Q * ref)) < 1e-2 * abs(0.5 * np.sum(Q * ref))


def test_method_error_falls_with_the_near_block():
    """Larger near blocks (n_sr = 1, 2, 3 at fixed h) move the truncation
    further out: the error against the image sum falls."""
    N, n = 200, 8
    x, Q = _boundary_layer(N, 10, n)
    ref = odir.image_ewald(x, Q)
    errs = []
    for nsr in (1, 2, 3):
        out = odir.run(x, Q, fep3m.Params(L=1.0, n=n, n_sr=nsr))
        errs.append(np.linalg.norm(out["Phi"] - ref) / np.linalg.norm(ref))
    print("grounded box, n_sr = 1, 2, 3:", ", ".join(f"{e:.3e}" for e in errs))
    assert errs[0] > errs[1] > errs[2]


def test_charges_outside_the_box_are_rejected():
    with pytest.raises(ValueError):
        odir.bin_box(np.array([[0.5, 1.0, 0.5]]), 1.0, 8)


def test_box_gradients_match_central_differences():
    """The adjoint forces and charge derivatives of the grounded-box energy
    (with the two terms that eq. bcadjust adds: the boundary values depend
    on the moments and on the positions) equal central differences of the
    oracle's own energy, for charges next to the faces."""
    N, n = 60, 7
    x, Q = _boundary_layer(N, 12, n)
    P = fep3m.Params(L=1.0, n=n)
    out = odir.energy_forces(x, Q, P)
    h = P.h
    # probe charges away from element faces (the energy is smooth inside elements)
    frac = (x / h) % 1.0
    ok = np.nonzero(np.all((frac > 0.1) & (frac < 0.9), axis=1))[0][:6]
    assert len(ok) >= 4
    dx = 1e-6
    for i in ok:
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += dx
            xm[i, k] -= dx
            fd = -(odir.run(xp, Q, P)["U"] - odir.run(xm, Q, P)["U"]) / (2 * dx)
            assert abs(out["F"][i, k] - fd) < 1e-5 * np.max(np.abs(out["F"][ok])), (i, k, out["F"][i, k], fd)
        Qp, Qm = Q.copy(), Q.copy()
        Qp[i] += 1e-6
        Qm[i] -= 1e-6
        fdq = (odir.run(x, Qp, P)["U"] - odir.run(x, Qm, P)["U"]) / 2e-6
        assert abs(out["dUdQ"][i] - fdq) < 1e-6 * np.max(np.abs(out["dUdQ"])), (i, out["dUdQ"][i], fdq)


def test_box_forces_against_images():
    """Forces of the grounded-box method against the image-charge forces
    (Ewald of the image set): within the screen's truncation error."""
    N, n = 200, 8
    x, Q = _boundary_layer(N, 13, n)
    out = odir.energy_forces(x, Q, fep3m.Params(L=1.0, n=n))
    X, QQ = odir.image_charges(x, Q, 1.0)
    from oracle import ewald
    ref = ewald.ewald(X, QQ, L=2.0, alpha=2.5, nimg=2, mmax=8, forces=True, targets=8 * np.arange(N))["F"]
    err = np.linalg.norm(out["F"] - ref) / np.linalg.norm(ref)
    print(f"grounded box forces vs images: {err:.3e}")
    assert err < 1e-2
