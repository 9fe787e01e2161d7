"""Pins for the oracle's analytic gradients: central finite differences of
the oracle's own discrete energy (a different computation: two forward
evaluations, no adjoint), and the Ewald forces the method approximates."""
import numpy as np
import pytest

import workloads
from oracle import adjoint, ewald, fep3m


@pytest.fixture(scope="module")
def case():
    x, Q = workloads.uniform(60, seed=21)
    P = fep3m.Params(L=1.0, n=8)
    out = adjoint.energy_forces(x, Q, P)
    return x, Q, P, out


def _interior(x, P, margin=1e-3):
    g = (x / P.L) * P.n
    frac = g - np.floor(g)
    return np.all((frac > margin) & (frac < 1 - margin), axis=1)


def test_forces_match_central_differences(case):
    x, Q, P, out = case
    ok = np.nonzero(_interior(x, P))[0][:6]
    h = 1e-6
    for i in ok:
        for k in range(3):
            xp = x.copy(); xp[i, k] += h
            xm = x.copy(); xm[i, k] -= h
            fd = -(fep3m.run(xp, Q, P)["U"] - fep3m.run(xm, Q, P)["U"]) / (2 * h)
            assert abs(fd - out["F"][i, k]) < 2e-6 * max(1.0, np.abs(out["F"]).max()), (i, k, fd, out["F"][i, k])


def test_charge_derivative_along_neutral_directions(case):
    x, Q, P, out = case
    eps = 1e-6
    for (i, j) in ((0, 1), (5, 17), (30, 59)):
        Qp = Q.copy(); Qp[i] += eps; Qp[j] -= eps
        Qm = Q.copy(); Qm[i] -= eps; Qm[j] += eps
        fd = (fep3m.run(x, Qp, P)["U"] - fep3m.run(x, Qm, P)["U"]) / (2 * eps)
        an = out["dUdQ"][i] - out["dUdQ"][j]
        assert abs(fd - an) < 1e-6 * max(1.0, abs(an))


def test_dUdQ_differs_from_potential(case):
    """The discrete operator is not symmetric (Section 5), so dU/dQ != Phi;
    the difference is of truncation-error size."""
    x, Q, P, out = case
    diff = np.abs(out["dUdQ"] - out["Phi"]).max()
    assert 0 < diff < 1e-2 * np.abs(out["Phi"]).max()


def test_forces_close_to_ewald():
    x, Q = workloads.uniform(200, seed=22)
    P = fep3m.Params(L=1.0, n=8)
    out = adjoint.energy_forces(x, Q, P)
    E = ewald.ewald(x, Q, forces=True)
    rel = np.linalg.norm(out["F"] - E["F"]) / np.linalg.norm(E["F"])
    assert rel < 2e-2
    # momentum is not conserved exactly (non-symmetric operators), but the
    # net force is small compared with the forces themselves
    assert np.abs(out["F"].sum(axis=0)).max() < 1e-2 * np.abs(out["F"]).sum(axis=0).max()
