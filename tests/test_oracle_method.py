"""Whole-method pins for the FE-P3M oracle (CPU).

The method is an approximation (truncated near field), so its result is
pinned against the independently verified Ewald sum within the method's
truncation error, and by exact invariances of the discretisation: a shift
of every charge by whole elements, permutations and reflections of the
axes, and linearity in the charges."""
import math

import numpy as np
import pytest

import workloads
from oracle import ewald, fep3m


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def small():
    x, Q = workloads.uniform(200, seed=11)
    return x, Q


def test_matches_ewald_within_truncation_error(small):
    """Config-1-like mesh: Phi + c vs tin-foil Ewald.  The one-element q = 3
    screen leaves an R^-3 tail beyond the 7^3 block, measured at a few 1e-3;
    a dropped 4 pi, a wrong sign or a missing self term gives O(1)."""
    x, Q = small
    E = ewald.ewald(x, Q)
    P = fep3m.Params(L=1.0, n=8)
    o = fep3m.run(x, Q, P, stages=True)
    c = fep3m.ewald_constant(o["u"], Q, P)
    assert _rel(o["Phi"] + c, E["Phi"]) < 1e-2
    assert abs(o["U"] - E["U"]) < 1e-2 * abs(E["U"])


def test_gauge_constant_pinned_against_ewald():
    """The constant c that relates the zero-mean mesh gauge to tin-foil Ewald
    (c = (2 pi / 3V) sum_j Q_j |delta_j|^2 for this screen) is pinned on
    charges chosen so that it dominates the truncation error: positive
    charges near element corners (|delta|^2 ~ 0.6 h^2), negative charges
    near element centres.  Phi + c must match Ewald, while Phi alone and
    Phi + 2c must miss by far more; the constant that best fits Ewald in the
    least-squares sense (the mean difference) must equal c (Section 4
    compares potentials up to an additive constant)."""
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
    P = fep3m.Params(L=1.0, n=n)
    o = fep3m.run(x, Q, P, stages=True)
    c = fep3m.ewald_constant(o["u"], Q, P)
    assert c > 1.0
    good = _rel(o["Phi"] + c, E["Phi"])
    assert good < 2e-3
    assert _rel(o["Phi"], E["Phi"]) > 10 * good
    assert _rel(o["Phi"] + 2 * c, E["Phi"]) > 10 * good
    c_fit = float(np.mean(E["Phi"] - o["Phi"]))
    assert abs(c_fit - c) < 0.01 * c


def test_larger_near_block_is_more_accurate(small):
    """Truncation error falls with the near-block radius (R^-3 tail)."""
    x, Q = small
    E = ewald.ewald(x, Q)
    errs = []
    for nsr in (3, 5):
        P = fep3m.Params(L=1.0, n=16, n_sr=nsr)
        o = fep3m.run(x, Q, P, stages=True)
        errs.append(_rel(o["Phi"] + fep3m.ewald_constant(o["u"], Q, P), E["Phi"]))
    assert errs[1] < 0.7 * errs[0]


def test_scale_invariance(small):
    """Potentials scale as 1/L for the same charges in a scaled box."""
    x, Q = small
    a = fep3m.run(x, Q, fep3m.Params(L=1.0, n=8))
    b = fep3m.run(2.5 * x, Q, fep3m.Params(L=2.5, n=8))
    np.testing.assert_allclose(b["Phi"] * 2.5, a["Phi"], rtol=1e-11, atol=1e-11)


def test_mesh_aligned_translation(small):
    x, Q = small
    P = fep3m.Params(L=1.0, n=8)
    a = fep3m.run(x, Q, P)
    b = fep3m.run(x + np.array([3, -2, 9]) * P.h, Q, P)
    assert np.abs(a["Phi"] - b["Phi"]).max() < 1e-11 * np.abs(a["Phi"]).max()


def test_axis_permutation_and_reflection(small):
    x, Q = small
    P = fep3m.Params(L=1.0, n=8)
    a = fep3m.run(x, Q, P)
    b = fep3m.run(x[:, [2, 0, 1]], Q, P)
    assert np.abs(a["Phi"] - b["Phi"]).max() < 1e-11 * np.abs(a["Phi"]).max()
    c = fep3m.run(np.column_stack([1.0 - x[:, 0], x[:, 1], x[:, 2]]), Q, P)
    assert np.abs(a["Phi"] - c["Phi"]).max() < 1e-10 * np.abs(a["Phi"]).max()


def test_linear_in_charges(small):
    x, Q = small
    rng = np.random.default_rng(2)
    Q2 = rng.permutation(Q)
    P = fep3m.Params(L=1.0, n=8)
    a = fep3m.run(x, Q, P)["Phi"]
    b = fep3m.run(x, Q2, P)["Phi"]
    c = fep3m.run(x, 0.5 * Q - 2.0 * Q2, P)["Phi"]
    assert np.abs(c - (0.5 * a - 2.0 * b)).max() < 1e-11 * np.abs(c).max()


def test_pair_sum_brute_force(small):
    """The element-offset pair sum equals a brute-force minimum-image sum
    restricted to the element block (n > 2 n_sr + 1 keeps images apart)."""
    x, Q = small
    n, nsr = 9, 3
    P = fep3m.Params(L=1.0, n=n, n_sr=nsr)
    o = fep3m.run(x, Q, P, stages=True)
    e = o["e"]
    h = P.h
    ref = np.zeros(len(Q))
    for i in range(len(Q)):
        de = e - e[i]
        de = (de + n // 2) % n - n // 2
        near = np.all(np.abs(de) <= nsr, axis=1)
        near[i] = False
        d = x[near] - x[i]
        d -= np.round(d)
        ref[i] = np.sum(Q[near] / np.linalg.norm(d, axis=1))
    np.testing.assert_allclose(o["Phi_p"], ref, rtol=1e-12, atol=1e-9)


def test_targets_subset_matches_full(small):
    x, Q = small
    P = fep3m.Params(L=1.0, n=8)
    full = fep3m.run(x, Q, P)
    t = np.array([3, 17, 150, 199])
    sub = fep3m.run(x, Q, P, targets=t)
    np.testing.assert_allclose(sub["Phi"], full["Phi"][t], rtol=1e-13, atol=1e-12)


def test_rejects_non_neutral(small):
    x, Q = small
    with pytest.raises(ValueError):
        fep3m.run(x, Q + 0.01, fep3m.Params(L=1.0, n=8))
