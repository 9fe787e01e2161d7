"""Mixed-precision path (float32 multigrid preconditioner, float32 near
field and interpolation with compensated sums; float64 PCG, norms,
projections, coarse solve and energy) against the FP64 oracle, to the
mixed-path tolerance 1e-5 relative RMS."""
import numpy as np
import pytest

import paper_1503_08509_amd as fp
import workloads
from oracle import adjoint, fep3m

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("near", [fp.NEAR_AUTO, fp.NEAR_DIRECT])
def test_mixed_config1_matches_oracle(torch, near):
    x, Q = workloads.make("uniform-1k-n8")
    ref = adjoint.energy_forces(x, Q, fep3m.Params(L=1.0, n=8))
    ctx = fp.Context(1.0, len(Q), 8, precision=fp.PRECISION_MIXED, near_field=near)
    out = ctx.energy_forces(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda(), dUdQ=True, Phi=True)
    assert _rel(out["Phi"].cpu().numpy(), ref["Phi"]) < MIXED_TOL
    assert _rel(out["F"].cpu().numpy(), ref["F"]) < MIXED_TOL
    assert _rel(out["dUdQ"].cpu().numpy(), ref["dUdQ"]) < MIXED_TOL
    assert abs(float(out["U"].item()) - ref["U"]) < MIXED_TOL * abs(ref["U"])
    st = ctx.stats()
    assert st["mg_rel_residual"] <= 1e-7 and st["mg_iterations"] <= 12


def test_mixed_config2_sampled(torch):
    """100k charges, 32^3: FP64 and mixed side by side; Phi of the mixed
    path on 300 sampled charges against the oracle, and in full against the
    FP64 GPU path."""
    x, Q = workloads.make("uniform-100k-n32")
    tx, tQ = torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda()
    P64, U64 = fp.Context(1.0, len(Q), 32).energy(tx, tQ)
    ctx = fp.Context(1.0, len(Q), 32, precision=fp.PRECISION_MIXED)
    Pm, Um = ctx.energy(tx, tQ)
    Pm, P64 = Pm.cpu().numpy(), P64.cpu().numpy()
    rng = np.random.default_rng(8)
    tgt = np.sort(rng.choice(len(Q), 300, replace=False))
    ref = fep3m.run(x, Q, fep3m.Params(L=1.0, n=32), targets=tgt)
    assert _rel(Pm[tgt], ref["Phi"]) < MIXED_TOL
    assert _rel(Pm, P64) < MIXED_TOL
    assert abs(float(Um.item()) - float(U64.item())) < MIXED_TOL * abs(float(U64.item()))


@pytest.mark.parametrize("case", ["two", "ragged17_n7", "faces"])
def test_mixed_small_and_ragged(torch, case):
    rng = np.random.default_rng(43)
    if case == "two":
        n, x, Q = 8, np.array([[0.1, 0.2, 0.3], [0.55, 0.6, 0.05]]), np.array([1.0, -1.0])
    elif case == "ragged17_n7":
        n = 7
        x = rng.random((17, 3)) * 3.0 - 1.0
        Q = rng.uniform(-1, 1, 17)
        Q -= Q.mean()
    else:
        n = 8
        x = np.array([[0.0, 0.125, 0.5], [1.0, 0.25, 0.375], [0.875, 1.0, 0.0],
                      [-0.125, 0.5, 0.625], [0.3, 0.7, 0.9], [0.5, 0.5, 0.5]])
        Q = np.array([1.0, -1.0, 0.5, -0.5, 2.0, -2.0])
    ref = fep3m.run(x, Q, fep3m.Params(L=1.0, n=n))
    ctx = fp.Context(1.0, len(Q), n, precision=fp.PRECISION_MIXED)
    Phi, U = ctx.energy(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda())
    assert _rel(Phi.cpu().numpy(), ref["Phi"]) < MIXED_TOL
    assert abs(float(U.item()) - ref["U"]) < MIXED_TOL * max(1.0, abs(ref["U"]))


def test_mixed_forces_1M_against_fp64(torch):
    """N = 1e6, 64^3: the mixed path's analytic forces against the FP64
    path's (finite differences cannot resolve float32 energies here)."""
    x, Q = workloads.make("uniform-1M-n64")
    tx, tQ = torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda()
    o64 = fp.Context(1.0, len(Q), 64).energy_forces(tx, tQ, dUdQ=True, Phi=True)
    om = fp.Context(1.0, len(Q), 64, precision=fp.PRECISION_MIXED).energy_forces(tx, tQ, dUdQ=True, Phi=True)
    for k in ("F", "dUdQ", "Phi"):
        assert _rel(om[k].cpu().numpy(), o64[k].cpu().numpy()) < MIXED_TOL, k
    assert abs(float(om["U"].item()) - float(o64["U"].item())) < MIXED_TOL * abs(float(o64["U"].item()))
