"""Pins for the oracle's 1-D FE ingredients, screens, exact screen
potentials, tables and mesh solve (CPU).  Each check is against something
fixed independently of the oracle's own formulas: textbook values, exact
rational arithmetic, closed forms, or a different algorithm."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.linalg
from numpy.polynomial import polynomial as P
from scipy import integrate

from oracle import fe1d, mesh, potential, screens, tables


# ---------------------------------------------------------------- 1-D FE

def test_gll_nodes_textbook():
    # GLL nodes on [-1,1]: p=2 {0}, p=3 {+-1/sqrt5}, p=4 {0, +-sqrt(3/7)}
    np.testing.assert_allclose(fe1d.gll_nodes(2) * 2, [-1, 0, 1], atol=1e-15)
    np.testing.assert_allclose(fe1d.gll_nodes(3) * 2, [-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1], atol=1e-15)
    np.testing.assert_allclose(fe1d.gll_nodes(4) * 2, [-1, -math.sqrt(3 / 7), 0, math.sqrt(3 / 7), 1], atol=1e-15)
    # p = 5: interior roots of P5' are +-sqrt(1/3 +- 2 sqrt(7)/21)
    a = math.sqrt(1 / 3 - 2 * math.sqrt(7) / 21)
    b = math.sqrt(1 / 3 + 2 * math.sqrt(7) / 21)
    np.testing.assert_allclose(fe1d.gll_nodes(5) * 2, [-1, -b, -a, a, b, 1], atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 6])
def test_periodic_matrices_basic(p):
    n = 5
    K1, M1 = fe1d.periodic_matrices(p, n)
    assert np.abs(K1 @ np.ones(p * n)).max() < 1e-12          # constants in the kernel
    assert abs(np.ones(p * n) @ M1 @ np.ones(p * n) - n) < 1e-12  # int 1 = domain length
    assert np.allclose(K1, K1.T) and np.allclose(M1, M1.T)
    assert np.linalg.eigvalsh(M1).min() > 0


@pytest.mark.parametrize("p", [2, 5])
def test_stiffness_is_exact_for_polynomials(p):
    """v^T K w = int v' w' and v^T M w = int v w for polynomials of degree <= p,
    which the order-p space contains exactly (Dirichlet assembly on [-n/2, n/2])."""
    n = 3
    K, M = fe1d.dirichlet_matrices(p, n)
    g = fe1d.gll_nodes(p)
    xs = np.array([e - n / 2 + 0.5 + g[k] for e in range(n) for k in range(p)] + [n / 2])
    rng = np.random.default_rng(p)
    cv, cw = rng.standard_normal(p + 1), rng.standard_normal(p + 1)
    v, w = P.polyval(xs, cv), P.polyval(xs, cw)
    dv, dw = P.polyder(cv), P.polyder(cw)
    lo, hi = -n / 2, n / 2
    ex_k = P.polyval(hi, P.polyint(P.polymul(dv, dw))) - P.polyval(lo, P.polyint(P.polymul(dv, dw)))
    ex_m = P.polyval(hi, P.polyint(P.polymul(cv, cw))) - P.polyval(lo, P.polyint(P.polymul(cv, cw)))
    assert abs(v @ K @ w - ex_k) < 1e-11 * max(1, abs(ex_k))
    assert abs(v @ M @ w - ex_m) < 1e-11 * max(1, abs(ex_m))


def test_1d_poisson_nodally_exact():
    """Textbook special case: for -u'' = f with f of degree p-2 the exact
    solution is a degree-p polynomial, so the FE solution equals it at every
    node (Dirichlet data from the exact solution)."""
    p, n = 5, 4
    K, M = fe1d.dirichlet_matrices(p, n)
    g = fe1d.gll_nodes(p)
    xs = np.array([e - n / 2 + 0.5 + g[k] for e in range(n) for k in range(p)] + [n / 2])
    cu = np.array([0.3, -1.0, 0.5, 0.2, -0.1, 0.05])          # exact u, degree 5
    f = -P.polyder(cu, 2)
    u = P.polyval(xs, cu)
    b = M @ P.polyval(xs, f)                                  # f in the space: int f v exactly
    inner = np.arange(1, len(xs) - 1)
    bnd = np.array([0, len(xs) - 1])
    ui = np.linalg.solve(K[np.ix_(inner, inner)], b[inner] - K[np.ix_(inner, bnd)] @ u[bnd])
    np.testing.assert_allclose(ui, u[inner], atol=1e-12)


# ---------------------------------------------------------------- screens

def _exact_duals(q):
    """Dual functions of the one-element screen in exact rationals: the
    interior order-q functions span bubble * P_{q-2}, bubble = 1/4 - x^2;
    solve int x^m r_l = [m == l] exactly."""
    d = q - 2

    def integ(c):                     # int_{-1/2}^{1/2} of polynomial coeffs c
        return sum(Fraction(ck) * (Fraction(1, 2) ** (k + 1) - Fraction(-1, 2) ** (k + 1)) / (k + 1)
                   for k, ck in enumerate(c))

    bubble = [Fraction(1, 4), Fraction(0), Fraction(-1)]
    basis = []
    for j in range(d + 1):
        c = [Fraction(0)] * (j + 3)
        for k, bk in enumerate(bubble):
            c[k + j] += bk
        basis.append(c)
    Mx = [[integ([Fraction(0)] * m + b) for b in basis] for m in range(d + 1)]
    # solve Mx X = I in rationals (Gauss-Jordan)
    nb = d + 1
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
        c = [Fraction(0)] * (d + 3)
        for j in range(nb):
            for k, v in enumerate(basis[j]):
                c[k] += X[j][l] * v
        duals.append(c)
    return duals


@pytest.mark.parametrize("q", [3, 4, 5])
def test_dual_functions_exact(q):
    xs = np.linspace(-0.5, 0.5, 23)
    r = screens.dual_functions(q, xs)
    ex = _exact_duals(q)
    for l, c in enumerate(ex):
        vals = np.array([float(sum(ck * Fraction(float(x)) ** k for k, ck in enumerate(c))) for x in xs])
        np.testing.assert_allclose(r[:, l], vals, atol=1e-12)


def test_q3_closed_forms():
    # one-element q = 3: r0 = 3/2 (1 - 4x^2), r1 = 30 x (1 - 4x^2)
    xs = np.linspace(-0.5, 0.5, 17)
    r = screens.dual_functions(3, xs)
    np.testing.assert_allclose(r[:, 0], 1.5 * (1 - 4 * xs**2), atol=1e-13)
    np.testing.assert_allclose(r[:, 1], 30 * xs * (1 - 4 * xs**2), atol=1e-12)


def test_screen_moments_about_charge():
    """int (x - delta)^m rho_1(x; delta) dx = [m == 0] for m <= d (Table moments)."""
    xq, wq = fe1d.gauss_legendre(12)
    for q in (3, 4):
        for delta in (-0.41, 0.0, 0.17, 0.49):
            rho = screens.screen_1d(q, xq, delta)
            for m in range(q - 1):
                mom = np.sum(wq * (xq - delta) ** m * rho)
                assert abs(mom - (1.0 if m == 0 else 0.0)) < 1e-13


def test_dense_3d_moment_system_matches_separable():
    """The full moment system (eq. momentmatrix) and the three 1-D systems
    (eq. moment1d) give the same screen."""
    q = 3
    delta = np.array([0.21, -0.33, 0.08])
    c = screens.screen_3d_dense(q, delta)
    nb = q - 1
    w = [screens.dual_coefficients(q) @ (delta[k] ** np.arange(q - 1)) for k in range(3)]
    sep = np.einsum("k,j,i->kji", w[2], w[1], w[0]).ravel()
    np.testing.assert_allclose(c, sep, atol=1e-12)
    assert len(c) == nb ** 3


@pytest.mark.parametrize("p,q", [(5, 3), (6, 4)])
def test_load_weights_reproduce_moments(p, q):
    """sum_k g_l[k] x_k^m = int r_l x^m = [l == m] for m <= p (interpolation of
    x^m in the order-p space is exact)."""
    g = screens.load_weights(p, q)
    nodes = fe1d.gll_nodes(p)
    for l in range(q - 1):
        for m in range(q - 1):
            assert abs(g[l] @ nodes**m - (1.0 if l == m else 0.0)) < 1e-13


# ---------------------------------------------------------------- exact screen potential

def test_uniform_cube_closed_form():
    const = [np.array([1.0])] * 3
    pts = np.array([[3.0, 0.2, 0.1], [0.1, 0.2, -0.3], [0.7, 0.6, 0.2], [0.03, 0.01, 0.02], [7.5, 0.3, -2.0]])
    v = potential.separable_potential(const, pts)
    for pt, vv in zip(pts, v):
        ref = potential.uniform_box_potential(np.full(3, -0.5), np.full(3, 0.5), pt)
        assert abs(vv - ref) < 1e-12 * abs(ref)


def test_screen_potential_brute_force_far():
    """Tensor Gauss quadrature of int R_a(y)/|x-y| dy (smooth integrand for
    far points) agrees with the Gaussian-identity evaluation."""
    polys = potential.dual_polynomials(3)
    xq, wq = fe1d.gauss_legendre(20)
    pts = np.array([[2.5, 0.3, -0.1], [1.9, -1.7, 0.6]])
    for a in [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1)]:
        v = potential.separable_potential([polys[a[0]], polys[a[1]], polys[a[2]]], pts)
        f = [P.polyval(xq, polys[a[k]]) for k in range(3)]
        Y = np.stack(np.meshgrid(xq, xq, xq, indexing="ij"), -1)
        W = np.einsum("i,j,k->ijk", wq * f[0], wq * f[1], wq * f[2])
        for pt, vv in zip(pts, v):
            ref = np.sum(W / np.linalg.norm(Y - pt, axis=-1))
            assert abs(vv - ref) < 1e-11 * max(1e-3, abs(ref))


def test_point_minus_screen_decays_like_R3():
    """|1/R - Phi_sc| of the one-element q = 3 screen falls like R^-3
    (monopole and dipole cancelled; Discussion, Section 5)."""
    q = 3
    polys = potential.dual_polynomials(q)
    delta = np.array([0.23, -0.11, 0.37])
    dirs = np.array([[1, 0, 0], [0, 1, 0], [1, 1, 1], [1, -2, 0.5], [0.3, 0.2, -1]], float)
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    Rs = np.array([4.0, 8.0, 16.0, 32.0])
    resid = []
    for R in Rs:
        pts = delta + R * dirs
        phi = np.zeros(len(pts))
        for ax in range(2):
            for ay in range(2):
                for az in range(2):
                    c = delta[0] ** ax * delta[1] ** ay * delta[2] ** az
                    phi += c * potential.separable_potential([polys[ax], polys[ay], polys[az]], pts)
        resid.append(np.abs(1.0 / R - phi).max())
    slopes = np.diff(np.log(resid)) / np.diff(np.log(Rs))
    assert np.all(np.abs(slopes + 3.0) < 0.15), slopes


# ---------------------------------------------------------------- tables

def test_tables_converged_in_box_size():
    T15 = tables.screen_tables(5, 3, 3, B=15)
    T19 = tables.screen_tables(5, 3, 3, B=19)
    assert np.abs(T15 - T19).max() < 1e-11 * np.abs(T15).max()


def test_tables_match_exact_potential_away_from_source():
    """FE tables equal the exact screen potential up to an FE error that is
    large only near the source element."""
    T = tables.screen_tables(5, 3, 3)
    Ti = tables.screen_tables(5, 3, 3, bc="interp")
    offs = tables.offsets(3)
    dist = np.abs(offs).max(axis=1)
    far = dist == 3
    near = dist == 0
    rel_far = np.abs(T[:, far] - Ti[:, far]).max() / np.abs(Ti[:, far]).max()
    rel_near = np.abs(T[:, near] - Ti[:, near]).max() / np.abs(Ti[:, near]).max()
    assert rel_far < 1e-3
    assert rel_far < 0.05 * rel_near
    assert 1e-3 < rel_near < 0.1


def test_tables_cubic_symmetry():
    """Swapping x and y maps the table of moment (ax, ay, az) at offset
    (Dx, Dy, Dz), node (mx, my, mz) onto (ay, ax, az), (Dy, Dx, Dz), (my, mx, mz);
    reflecting x flips the sign for odd ax."""
    p = 5
    T = tables.screen_tables(p, 3, 3)
    S = 7
    A = screens.moment_exponents(1)
    aidx = {tuple(a): i for i, a in enumerate(A)}
    T6 = T.reshape(len(A), S, S, S, p + 1, p + 1, p + 1)    # [a, Dz, Dy, Dx, mz, my, mx]
    for i, (ax, ay, az) in enumerate(A):
        j = aidx[(ay, ax, az)]
        np.testing.assert_allclose(T6[i], T6[j].transpose(0, 2, 1, 3, 5, 4), atol=1e-11)
        refl = T6[i][:, :, ::-1, :, :, ::-1] * (-1) ** ax
        np.testing.assert_allclose(T6[i], refl, atol=1e-11)


# ---------------------------------------------------------------- mesh solve

def test_periodic_solve_manufactured():
    p, n = 5, 4
    rng = np.random.default_rng(7)
    phi_star = rng.standard_normal((p * n,) * 3)
    b = mesh.stiffness_apply(phi_star, p, n)
    phi = mesh.solve_periodic(b, p, n)
    ref = phi_star - mesh.mean_value(phi_star, p, n)
    assert np.abs(phi - ref).max() < 1e-10 * np.abs(ref).max()
    assert abs(mesh.mean_value(phi, p, n)) < 1e-13


def test_periodic_solve_matches_sparse_cg():
    p, n = 3, 4
    K1, M1 = fe1d.periodic_matrices(p, n)
    K = (scipy.sparse.kron(scipy.sparse.kron(K1, M1), M1) + scipy.sparse.kron(scipy.sparse.kron(M1, K1), M1)
         + scipy.sparse.kron(scipy.sparse.kron(M1, M1), K1)).tocsr()
    rng = np.random.default_rng(8)
    b = rng.standard_normal((p * n,) * 3)
    b = mesh.project_compatible(b, p, n)
    assert abs(b.sum()) < 1e-12
    x, info = scipy.sparse.linalg.cg(K, b.ravel(), rtol=1e-14, maxiter=5000)
    assert info == 0
    x = x.reshape(b.shape)
    x -= mesh.mean_value(x, p, n)
    ref = mesh.solve_periodic(b, p, n)
    assert np.abs(x - ref).max() < 1e-9 * np.abs(ref).max()


def test_load_vector_moments():
    """The load of one element reproduces 4 pi times its charge moments:
    sum_m b_m = 4 pi sum Q and sum_m b_m x_m = 4 pi sum Q u (the order-p
    basis interpolates 1 and x exactly)."""
    p, q, n = 5, 3, 7
    rng = np.random.default_rng(9)
    u = rng.uniform(-0.5, 0.5, (5, 3))
    Q = rng.standard_normal(5)
    e_lin = np.full(5, 3 + n * (2 + n * 4))
    C = screens.element_moments(e_lin, u, Q, n**3, 1)
    b = mesh.load_vector(C, n, p, q)
    assert abs(b.sum() - 4 * math.pi * Q.sum()) < 1e-12
    g = fe1d.gll_nodes(p)
    xs = np.array([e + g[k] for e in range(n) for k in range(p)])   # node offset from element centre - 1/2..
    # coordinate of each node relative to the centre of element (3, 2, 4)
    cx = xs - 3.0
    cy = xs - 2.0
    bx = np.einsum("kji,i->", b, cx)
    by = np.einsum("kji,j->", b, cy)
    assert abs(bx - 4 * math.pi * np.sum(Q * u[:, 0])) < 1e-11
    assert abs(by - 4 * math.pi * np.sum(Q * u[:, 1])) < 1e-11
