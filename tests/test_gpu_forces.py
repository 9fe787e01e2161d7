"""GPU forces and dU/dQ (the hand-written adjoint) against the oracle's
analytic gradients, and against central finite differences of the GPU
energy itself on the N = 1e6 configuration."""
import numpy as np
import pytest

import paper_1503_08509_amd as fp
import workloads
from oracle import adjoint, fep3m

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("wl,N,n,near", [("uniform-1k-n8", 1000, 8, fp.NEAR_AUTO),
                                         ("uniform-1k-n8", 1000, 8, fp.NEAR_DIRECT),
                                         ("adhoc-300-n9", 300, 9, fp.NEAR_AUTO)])
def test_forces_match_oracle(torch, wl, N, n, near):
    if wl in workloads.WORKLOADS:
        x, Q = workloads.make(wl)
    else:
        x, Q = workloads.uniform(N, seed=31, charges="uniform")
    ref = adjoint.energy_forces(x, Q, fep3m.Params(L=1.0, n=n))
    ctx = fp.Context(1.0, len(Q), n, mg_rtol=1e-13, near_field=near)
    assert ctx.stats()["near_fft"] == (near == fp.NEAR_AUTO and n == 8)
    out = ctx.energy_forces(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda(), dUdQ=True, Phi=True)
    F = out["F"].cpu().numpy()
    g = out["dUdQ"].cpu().numpy()
    assert _rel(F, ref["F"]) < 1e-9
    assert _rel(g, ref["dUdQ"]) < 1e-9
    assert _rel(out["Phi"].cpu().numpy(), ref["Phi"]) < 1e-10
    assert abs(float(out["U"].item()) - ref["U"]) < 1e-10 * abs(ref["U"])
    assert ctx.stats()["adj_iterations"] > 0


@pytest.mark.parametrize("near", [fp.NEAR_AUTO, fp.NEAR_DIRECT])
def test_forces_dense_elements_match_oracle(torch, near):
    """Elements holding more than 64 charges (several 64-charge chunks in the
    deposit, 8-target chunks in the pair sum): 150 charges inside one element
    and 90 inside another, plus 160 spread uniformly, on 8^3 elements."""
    rng = np.random.default_rng(41)
    h = 1.0 / 8
    a = (np.array([2, 5, 3]) + rng.uniform(0.05, 0.95, (150, 3))) * h
    b = (np.array([7, 0, 6]) + rng.uniform(0.05, 0.95, (90, 3))) * h
    x = np.concatenate([a, b, rng.random((160, 3))])
    Q = np.where(rng.random(400) < 0.5, 1.0, -1.0)
    Q -= Q.mean()
    ref = adjoint.energy_forces(x, Q, fep3m.Params(L=1.0, n=8))
    ctx = fp.Context(1.0, len(Q), 8, mg_rtol=1e-13, near_field=near)
    out = ctx.energy_forces(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda(), dUdQ=True, Phi=True)
    assert ctx.stats()["max_per_element"] >= 150
    assert _rel(out["F"].cpu().numpy(), ref["F"]) < 1e-9
    assert _rel(out["dUdQ"].cpu().numpy(), ref["dUdQ"]) < 1e-9
    assert _rel(out["Phi"].cpu().numpy(), ref["Phi"]) < 1e-10
    assert abs(float(out["U"].item()) - ref["U"]) < 1e-10 * abs(ref["U"])


def test_energy_forces_consistent_with_energy(torch):
    x, Q = workloads.make("uniform-1k-n8")
    ctx = fp.Context(1.0, len(Q), 8)
    tx, tQ = torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda()
    Phi, U = ctx.energy(tx, tQ)
    out = ctx.energy_forces(tx, tQ, Phi=True)
    assert float(out["U"].item()) == float(U.item())
    np.testing.assert_array_equal(out["Phi"].cpu().numpy(), Phi.cpu().numpy())


def test_forces_central_differences_1M(torch):
    """N = 1e6, 64^3 mesh: 32 particles at least 1e-4 h from every face,
    central differences of the GPU energy with step 1e-6 (FP64 path)."""
    x, Q = workloads.make("uniform-1M-n64")
    n, hstep = 64, 1e-6
    ctx = fp.Context(1.0, len(Q), n, mg_rtol=1e-12)
    tx, tQ = torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda()
    F = ctx.energy_forces(tx, tQ)["F"].cpu().numpy()
    g = x * n
    frac = g - np.floor(g)
    ok = np.nonzero(np.all((frac > 1e-4 + hstep * n) & (frac < 1 - 1e-4 - hstep * n), axis=1))[0]
    rng = np.random.default_rng(3)
    pick = rng.choice(ok, 32, replace=False)
    fd = np.zeros((32, 3))
    for r, i in enumerate(pick):
        for k in range(3):
            xp = tx.clone(); xp[i, k] += hstep
            xm = tx.clone(); xm[i, k] -= hstep
            Up = float(ctx.energy(xp, tQ)[1].item())
            Um = float(ctx.energy(xm, tQ)[1].item())
            fd[r, k] = -(Up - Um) / (2 * hstep)
    err = np.abs(fd - F[pick])
    scale = np.abs(F[pick]).max()
    assert err.max() < 1e-5 * scale, (err.max(), scale)


def test_dUdQ_neutral_directions(torch):
    x, Q = workloads.make("uniform-1k-n8")
    ctx = fp.Context(1.0, len(Q), 8, mg_rtol=1e-13)
    tx = torch.from_numpy(x).cuda()
    g = ctx.energy_forces(tx, torch.from_numpy(Q).cuda(), dUdQ=True)["dUdQ"].cpu().numpy()
    eps = 1e-6
    for (i, j) in ((0, 1), (10, 999), (400, 401)):
        Qp = Q.copy(); Qp[i] += eps; Qp[j] -= eps
        Qm = Q.copy(); Qm[i] -= eps; Qm[j] += eps
        Up = float(ctx.energy(tx, torch.from_numpy(Qp).cuda())[1].item())
        Um = float(ctx.energy(tx, torch.from_numpy(Qm).cuda())[1].item())
        assert abs((Up - Um) / (2 * eps) - (g[i] - g[j])) < 1e-5 * max(1.0, abs(g[i] - g[j]))


def test_autograd_function_matches_energy_forces(torch):
    """FEP3MEnergy's backward (reused forward state, recomputed pair terms)
    returns exactly the fused energy+force call's -F and dU/dQ."""
    x, Q = workloads.make("uniform-1k-n8")
    ctx = fp.Context(1.0, len(Q), 8)
    tx = torch.from_numpy(x).cuda().requires_grad_(True)
    tQ = torch.from_numpy(Q).cuda().requires_grad_(True)
    U = fp.FEP3MEnergy.apply(tx, tQ, ctx)
    (2.0 * U).backward()
    ref = ctx.energy_forces(tx.detach(), tQ.detach(), dUdQ=True)
    assert float(U.item()) == float(ref["U"].item())
    np.testing.assert_array_equal(tx.grad.cpu().numpy(), -2.0 * ref["F"].cpu().numpy())
    np.testing.assert_array_equal(tQ.grad.cpu().numpy(), 2.0 * ref["dUdQ"].cpu().numpy())


def test_autograd_single_input_and_stale_state(torch):
    x, Q = workloads.make("uniform-1k-n8")
    ctx = fp.Context(1.0, len(Q), 8)
    tQ = torch.from_numpy(Q).cuda()
    tx = torch.from_numpy(x).cuda().requires_grad_(True)
    U = fp.FEP3MEnergy.apply(tx, tQ, ctx)
    (gx,) = torch_autograd_grad(torch, U, [tx])
    F = ctx.energy_forces(tx.detach(), tQ)["F"]
    np.testing.assert_array_equal(gx.cpu().numpy(), -F.cpu().numpy())
    # a later evaluation on the same context invalidates the earlier forward state
    U1 = fp.FEP3MEnergy.apply(tx, tQ, ctx)
    ctx.energy(tx.detach(), tQ)
    with pytest.raises(fp.FEP3MError) as ei:
        U1.backward()
    assert ei.value.status == fp.ERR_ARG


def torch_autograd_grad(torch, out, inputs):
    return torch.autograd.grad(out, inputs)
