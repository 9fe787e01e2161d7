"""Pins for the Ewald ground truth (CPU)."""
import json
import math
import os

import numpy as np

import workloads
from oracle import ewald

HERE = os.path.dirname(__file__)


def _nacl(shift=(0.1, 0.1, 0.1)):
    g = json.load(open(os.path.join(HERE, "golden", "nacl.json")))
    x = np.array(g["Na"] + g["Cl"], dtype=np.float64) + np.array(shift)
    Q = np.array([1.0] * 4 + [-1.0] * 4)
    return g, x, Q


def test_nacl_madelung():
    g, x, Q = _nacl()
    out = ewald.ewald(x, Q, forces=True)
    M = g["madelung"]
    assert abs(out["U"] - (-8.0 * M)) < 1e-10
    np.testing.assert_allclose(out["Phi"], -2.0 * M * Q, rtol=0, atol=1e-10)
    assert np.abs(out["F"]).max() < 1e-12           # every ion is a centre of symmetry


def test_alpha_independence():
    rng = np.random.default_rng(3)
    x = rng.random((40, 3))
    Q = rng.permutation(np.repeat([1.0, -1.0], 20))
    ref = ewald.ewald(x, Q, alpha=2.5, nimg=2, mmax=5, forces=True)
    for a, nimg, m in ((2.0, 3, 5), (3.0, 2, 6)):          # alpha -20% / +20%
        o = ewald.ewald(x, Q, alpha=a, nimg=nimg, mmax=m, forces=True)
        assert np.abs(o["Phi"] - ref["Phi"]).max() < 1e-10
        assert np.abs(o["F"] - ref["F"]).max() < 1e-9


def test_forces_are_gradient_and_sum_to_zero():
    rng = np.random.default_rng(4)
    x = rng.random((12, 3))
    Q = rng.uniform(-1, 1, 12)
    Q -= Q.mean()
    o = ewald.ewald(x, Q, forces=True)
    assert np.abs(o["F"].sum(axis=0)).max() < 1e-11
    eps = 1e-6
    for i in (0, 5):
        for k in range(3):
            xp = x.copy(); xp[i, k] += eps
            xm = x.copy(); xm[i, k] -= eps
            fd = -(ewald.ewald(xp, Q)["U"] - ewald.ewald(xm, Q)["U"]) / (2 * eps)
            assert abs(fd - o["F"][i, k]) < 1e-6 * max(1.0, abs(fd))


def test_translation_invariance():
    rng = np.random.default_rng(5)
    x = rng.random((30, 3))
    Q = rng.permutation(np.repeat([1.0, -1.0], 15))
    a = ewald.ewald(x, Q)
    b = ewald.ewald(x + np.array([0.37, -0.21, 1.9]), Q)
    assert abs(a["U"] - b["U"]) < 1e-11
    assert np.abs(a["Phi"] - b["Phi"]).max() < 1e-11


def test_direct_image_sum_equals_ewald_plus_surface_term():
    """Direct summation over spherically ordered whole cells converges to the
    tin-foil Ewald energy plus (2 pi / 3 V)|D|^2 (de Leeuw, Perram & Smith).
    The cell-sum error falls like 1/R; two radii are extrapolated."""
    rng = np.random.default_rng(6)
    x = rng.random((4, 3))
    Q = np.array([1.0, -1.0, 0.5, -0.5])
    target = ewald.ewald(x, Q)["U"] + ewald.surface_term(x, Q)
    R1, R2 = 24, 48
    U1 = ewald.direct_image_energy(x, Q, R=R1)
    U2 = ewald.direct_image_energy(x, Q, R=R2)
    Uext = (R2 * U2 - R1 * U1) / (R2 - R1)
    assert abs(U2 - target) < 0.05 * abs(ewald.surface_term(x, Q)) + 1e-3
    assert abs(Uext - target) < 2e-4 * abs(target)


def test_sampled_ewald_matches_full_sum():
    """The large-N form (real space to rcut = L with alpha = 6/L, reciprocal
    cube |m| <= 12 from separable structure factors) equals the paper's
    setting (alpha = 2.5, two image shells, four modes) on a small system,
    and does not depend on its own splitting (alpha 6 vs 7.5, mmax raised
    with it): both sums converge to the same periodic potential."""
    x, Q = workloads.uniform(300, seed=5, charges="uniform")
    t = np.array([0, 7, 150, 299])
    a = ewald.ewald(x, Q, forces=True, targets=t)
    b = ewald.ewald_sampled(x, Q, t, forces=True)
    c = ewald.ewald_sampled(x, Q, t, alpha=7.5, mmax=15, forces=True)
    for r in (b, c):
        assert np.abs(r["Phi"] - a["Phi"]).max() < 1e-12 * np.abs(a["Phi"]).max()
        assert np.abs(r["F"] - a["F"]).max() < 1e-12 * np.abs(a["F"]).max()
