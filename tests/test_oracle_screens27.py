"""Pins for the oracle's screen families beyond the one-element q = 3 screen:
the 27-element screens of Section 2.1 (q = 1..4) and one-element screens of
higher degree (Section 5).  Each check is against something fixed
independently of the oracle's formulas: exact rational arithmetic, closed
forms, the paper's decay rates, Ewald, or central differences."""
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads
from oracle import adjoint, ewald, fe1d, fep3m, mesh, potential, screens, tables


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------- exact duals

def _poly_mul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _lagrange_exact(nodes, k):
    """Monomial coefficients of the Lagrange polynomial of nodes[k]."""
    c = [Fraction(1)]
    for j, xj in enumerate(nodes):
        if j != k:
            c = _poly_mul(c, [-xj / (nodes[k] - xj), 1 / (nodes[k] - xj)])
    return c


def _integ(c, lo, hi):
    return sum(ck * (hi ** (k + 1) - lo ** (k + 1)) / (k + 1) for k, ck in enumerate(c))


def _shift(c, s):
    """Coefficients of c(x - s)."""
    out = [Fraction(0)] * len(c)
    for k, ck in enumerate(c):
        for j in range(k + 1):
            out[j] += ck * math.comb(k, j) * (-s) ** (k - j)
    return out


def _exact_duals_27(q):
    """Dual functions of the 27-element screen in exact rationals, as pieces
    {offset: coefficients in the global coordinate} per l."""
    half = Fraction(1, 2)
    nodes = [Fraction(k, q) - half for k in range(q + 1)]          # central element
    pieces = []                                                      # per basis function: {offset: coef}
    for i in range(q + 1):
        pc = {0: _lagrange_exact(nodes, i)}
        if i == 0:                                                   # continues below as the upper node
            pc[-1] = _shift(_lagrange_exact(nodes, q), Fraction(-1))
        if i == q:
            pc[1] = _shift(_lagrange_exact(nodes, 0), Fraction(1))
        pieces.append(pc)
    Mx = [[sum(_integ(_poly_mul([Fraction(0)] * m + [Fraction(1)], c), o - half, o + half)
               for o, c in pc.items()) for pc in pieces] for m in range(q + 1)]
    nb = q + 1
    A = [row[:] + [Fraction(int(i == j)) for j in range(nb)] for i, row in enumerate(Mx)]
    for col in range(nb):
        piv = next(r for r in range(col, nb) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        pv = A[col][col]
        A[col] = [v / pv for v in A[col]]
        for r in range(nb):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [a - f * b for a, b in zip(A[r], A[col])]
    X = [row[nb:] for row in A]
    duals = []
    for l in range(nb):
        d = {}
        for i, pc in enumerate(pieces):
            for o, c in pc.items():
                acc = d.setdefault(o, [Fraction(0)] * (q + 1))
                for k, v in enumerate(c):
                    acc[k] += X[i][l] * v
        duals.append(d)
    return duals


@pytest.mark.parametrize("q", [1, 2, 3, 4])
def test_27_dual_functions_exact(q):
    xs = np.linspace(-1.49, 1.49, 41)
    r = screens.dual_functions(q, xs, "27")
    ex = _exact_duals_27(q)
    for l, d in enumerate(ex):
        vals = []
        for x in xs:
            o = int(np.floor(x + 0.5))
            c = d.get(o)
            vals.append(0.0 if c is None else float(sum(ck * Fraction(float(x)) ** k for k, ck in enumerate(c))))
        np.testing.assert_allclose(r[:, l], vals, atol=1e-11 * max(1.0, np.abs(vals).max()))


def test_27_q1_closed_forms():
    """q = 1: r0 = (h(x + 1/2) + h(x - 1/2)) / 2 and r1 = h(x - 1/2) - h(x + 1/2)
    with the unit hat h(x) = max(0, 1 - |x|) (support two elements)."""
    xs = np.linspace(-1.5, 1.5, 61)
    r = screens.dual_functions(1, xs, "27")
    hat = lambda x: np.maximum(0.0, 1.0 - np.abs(x))
    np.testing.assert_allclose(r[:, 0], 0.5 * (hat(xs + 0.5) + hat(xs - 0.5)), atol=1e-14)
    np.testing.assert_allclose(r[:, 1], hat(xs - 0.5) - hat(xs + 0.5), atol=1e-14)


@pytest.mark.parametrize("q,support", [(1, "27"), (2, "27"), (3, "27"), (4, "27"), (4, "one"), (5, "one")])
def test_screen_moments_about_charge(q, support):
    """int (x - delta)^m rho_1(x; delta) dx = [m == 0] for m <= d (Table moments)."""
    d = screens.moment_degree(q, support)
    xq, wq = screens._element_rule(q, support, 12)
    for delta in (-0.47, -0.2, 0.0, 0.31, 0.5):
        rho = screens.screen_1d(q, xq, delta, support)
        for m in range(d + 1):
            mom = np.sum(wq * (xq - delta) ** m * rho)
            assert abs(mom - (1.0 if m == 0 else 0.0)) < 1e-12


@pytest.mark.parametrize("q", [1, 2])
def test_27_dense_moment_system_matches_separable(q):
    """eq. momentmatrix over the (q+1)^3 basis functions equals the product
    of the three 1-D solutions of eq. moment1d."""
    delta = np.array([0.21, -0.33, 0.08])
    c = screens.screen_3d_dense(q, delta, "27")
    w = [screens.dual_coefficients(q, "27") @ (delta[k] ** np.arange(q + 1)) for k in range(3)]
    np.testing.assert_allclose(c, np.einsum("k,j,i->kji", w[2], w[1], w[0]).ravel(), atol=1e-12)


@pytest.mark.parametrize("q,support", [(1, "27"), (2, "27"), (4, "27"), (4, "one")])
def test_load_weights_reproduce_moments(q, support):
    """sum_k g_l[k] x_k^m = int r_l x^m = [l == m] for m <= d: the order-p
    space over the support interpolates x^m exactly."""
    p = q + 2
    s = screens.span(support)
    g = screens.load_weights(p, q, support)
    gl = fe1d.gll_nodes(p)
    xs = np.array([e - (s - 1) // 2 + gl[k] for e in range(s) for k in range(p)] + [(s - 1) // 2 + 0.5])
    d = screens.moment_degree(q, support)
    for l in range(d + 1):
        for m in range(d + 1):
            assert abs(g[l] @ xs**m - (1.0 if l == m else 0.0)) < 1e-12


# ---------------------------------------------------------------- decay (Fig. decayavg)

def _short_range(q, support, delta, pts):
    polys = potential.dual_polynomials(q, support)
    phi = np.zeros(len(pts))
    for a in screens.moment_exponents(screens.moment_degree(q, support)):
        phi += np.prod(delta ** a) * potential.separable_potential([polys[a[0]], polys[a[1]], polys[a[2]]], pts)
    R = np.linalg.norm(pts - delta, axis=1)
    return 1.0 / R - phi


@pytest.mark.parametrize("q,support,rate", [(1, "27", 3), (2, "27", 4), (3, "27", 5), (4, "one", 4)])
def test_point_minus_screen_decay_rate(q, support, rate):
    """|1/R - Phi_sc| falls like R^-(q+2) for the 27-element screens and like
    R^-q for the one-element ones (Section 2.1, Fig. decayavg; Section 5)."""
    delta = np.array([0.23, -0.11, 0.37])
    dirs = np.array([[1, 0, 0], [0, 1, 0], [1, 1, 1], [1, -2, 0.5], [0.3, 0.2, -1]], float)
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    Rs = np.array([6.0, 12.0, 24.0])
    res = [np.abs(_short_range(q, support, delta, delta + R * dirs)).max() for R in Rs]
    slopes = np.diff(np.log(res)) / np.diff(np.log(Rs))
    assert np.all(np.abs(slopes + rate) < 0.2), slopes


# ---------------------------------------------------------------- tables and load

def test_27_tables_converged_and_symmetric():
    """The Dirichlet box converges: at p = 3 the FE error of the far field
    inside the box moves the tables by 2.5e-9 from B = 11 to 15 and by ten
    times less from 15 to 19 (the one-element q = 3 tables at p = 5 move by
    1e-14); the tables are odd in x for odd ax."""
    p, q = 3, 1
    T11 = tables.screen_tables(p, q, 1, B=11, support="27")
    T15 = tables.screen_tables(p, q, 1, B=15, support="27")
    T19 = tables.screen_tables(p, q, 1, B=19, support="27")
    scale = np.abs(T15).max()
    assert np.abs(T11 - T15).max() < 1e-8 * scale
    assert np.abs(T15 - T19).max() < 0.2 * np.abs(T11 - T15).max()
    S = 3
    A = screens.moment_exponents(1)
    T6 = T15.reshape(len(A), S, S, S, p + 1, p + 1, p + 1)
    for i, (ax, ay, az) in enumerate(A):
        np.testing.assert_allclose(T6[i], T6[i][:, :, ::-1, :, :, ::-1] * (-1) ** ax, atol=1e-11)


def test_27_load_vector_moments():
    """A single element's load spreads over its 3^3 support and reproduces
    4 pi times its charge moments up to degree d (here q = 2, d = 2)."""
    q, n = 2, 7
    p = q + 2
    rng = np.random.default_rng(9)
    u = rng.uniform(-0.5, 0.5, (5, 3))
    Q = rng.standard_normal(5)
    e_lin = np.full(5, 3 + n * (2 + n * 4))
    C = screens.element_moments(e_lin, u, Q, n**3, q)
    b = mesh.load_vector(C, n, p, q, "27")
    g = fe1d.gll_nodes(p)
    xs = np.array([e + 0.5 + g[k] for e in range(n) for k in range(p)])
    cx, cy, cz = xs - 3.5, xs - 2.5, xs - 4.5
    assert abs(b.sum() - 4 * math.pi * Q.sum()) < 1e-12
    for (mx, my, mz) in [(1, 0, 0), (0, 2, 0), (1, 1, 0), (0, 1, 2), (2, 2, 2)]:
        got = np.einsum("kji,k,j,i->", b, cz**mz, cy**my, cx**mx)
        ref = 4 * math.pi * np.sum(Q * u[:, 0]**mx * u[:, 1]**my * u[:, 2]**mz)
        assert abs(got - ref) < 1e-11


# ---------------------------------------------------------------- whole method

@pytest.fixture(scope="module")
def small():
    return workloads.uniform(200, seed=11)


@pytest.mark.parametrize("q,support,bound", [(1, "27", 1e-2), (2, "27", 2e-3), (4, "one", 1e-3)])
def test_matches_ewald_within_truncation_error(small, q, support, bound):
    """Phi + c (c from the screens' second moments: zero once d >= 2) against
    tin-foil Ewald; the U error is of the same order."""
    x, Q = small
    E = ewald.ewald(x, Q)
    P = fep3m.Params(L=1.0, n=8, q=q, support=support)
    o = fep3m.run(x, Q, P, stages=True)
    c = fep3m.ewald_constant(o["u"], Q, P)
    if P.d >= 2:
        assert abs(c) < 1e-12
    assert _rel(o["Phi"] + c, E["Phi"]) < bound
    assert abs(o["U"] - E["U"]) < bound * abs(E["U"])


def test_27_gauge_constant_vanishes_for_q2():
    """With the x^2 moments cancelled (d = 2) no constant separates the mesh
    gauge from Ewald: on charges placed to make a d = 1 constant large
    (positive ones near element corners, negative near centres) Phi alone
    matches Ewald and the best-fit constant is at the error level."""
    n, N = 8, 200
    rng = np.random.default_rng(77)
    e = rng.integers(0, n, size=(N, 3))
    half = N // 2
    u = np.empty((N, 3))
    u[:half] = rng.choice([-1.0, 1.0], size=(half, 3)) * rng.uniform(0.40, 0.46, size=(half, 3))
    u[half:] = rng.uniform(-0.05, 0.05, size=(half, 3))
    x = (e + 0.5 + u) / n
    Q = np.concatenate([np.ones(half), -np.ones(half)])
    E = ewald.ewald(x, Q)
    o = fep3m.run(x, Q, fep3m.Params(L=1.0, n=n, q=2, support="27"))
    err = _rel(o["Phi"], E["Phi"])
    assert err < 2e-3
    d1 = (2 * math.pi / 3) * np.sum(Q * np.sum((u / n) ** 2, axis=1))   # the d = 1 constant here
    assert d1 > 1.0
    assert abs(float(np.mean(E["Phi"] - o["Phi"]))) < 0.02 * d1


@pytest.mark.parametrize("q,support,n", [(1, "27", 7), (4, "one", 7)])
def test_forces_match_central_differences(q, support, n):
    """Analytic F and dU/dQ of the discrete energy against central differences
    (charges away from element faces; Section 5 on derivatives)."""
    rng = np.random.default_rng(5)
    N = 24
    e = rng.integers(0, n, size=(N, 3))
    x = (e + 0.5 + rng.uniform(-0.35, 0.35, (N, 3))) / n
    Q = rng.uniform(-1, 1, N)
    Q -= Q.mean()
    P = fep3m.Params(L=1.0, n=n, q=q, support=support, n_sr=2)
    out = adjoint.energy_forces(x, Q, P)
    hstep = 1e-6
    for i in (0, 7, 13):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += hstep
            xm[i, k] -= hstep
            fd = -(fep3m.run(xp, Q, P)["U"] - fep3m.run(xm, Q, P)["U"]) / (2 * hstep)
            assert abs(out["F"][i, k] - fd) < 2e-6 * max(1.0, abs(fd))
    # dU/dQ along a neutral direction (charge moved from j to i)
    for (i, j) in ((2, 9), (11, 20)):
        dq = np.zeros(N)
        dq[i], dq[j] = 1e-6, -1e-6
        fd = (fep3m.run(x, Q + dq, P)["U"] - fep3m.run(x, Q - dq, P)["U"]) / 2e-6
        assert abs((out["dUdQ"][i] - out["dUdQ"][j]) - fd) < 2e-6 * max(1.0, abs(fd))
