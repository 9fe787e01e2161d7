"""Exact fast-diagonalisation mesh solver (solver = FDM): mesh potential and
results against the oracle (whose periodic solve is the same exact
construction, in NumPy) and against the multigrid solver at a tight
tolerance; batches, mixed precision and graph mode with this solver."""
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


@pytest.mark.parametrize("N,n,seed", [(1000, 8, None), (300, 9, 5), (17, 7, 6)])
def test_fdm_matches_oracle(torch, N, n, seed):
    if seed is None:
        x, Q = workloads.make("uniform-1k-n8")
    else:
        x, Q = workloads.uniform(N, seed=seed, charges="uniform")
    ctx = fp.Context(1.0, len(Q), n, solver=fp.SOLVER_FDM)
    out = ctx.energy_forces(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda(), dUdQ=True, Phi=True)
    ref = adjoint.energy_forces(x, Q, fep3m.Params(L=1.0, n=n))
    st = fep3m.run(x, Q, fep3m.Params(L=1.0, n=n), stages=True)
    phi = ctx.stage("phi").cpu().numpy()
    assert np.abs(phi - st["phi"].ravel()).max() < 1e-11 * np.abs(st["phi"]).max()
    for k in ("Phi", "F", "dUdQ"):
        assert _rel(out[k].cpu().numpy(), ref[k]) < 1e-10, k
    assert ctx.stats()["mg_rel_residual"] < 1e-11


def test_fdm_matches_tight_multigrid_100k(torch):
    x, Q = workloads.make("uniform-100k-n32")
    tx, tQ = torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda()
    a = fp.Context(1.0, len(Q), 32, solver=fp.SOLVER_FDM).energy_forces(tx, tQ, Phi=True)
    b = fp.Context(1.0, len(Q), 32, mg_rtol=1e-13).energy_forces(tx, tQ, Phi=True)
    for k in ("Phi", "F"):
        assert _rel(a[k].cpu().numpy(), b[k].cpu().numpy()) < 1e-10, k


def test_fdm_batch_mixed_graph(torch):
    counts = [400, 90, 1500]
    rng = np.random.default_rng(13)
    xs = [rng.random((c, 3)) for c in counts]
    Qs = [rng.uniform(-1, 1, c) for c in counts]
    Qs = [q - q.mean() for q in Qs]
    tx = torch.from_numpy(np.concatenate(xs)).cuda()
    tQ = torch.from_numpy(np.concatenate(Qs)).cuda()
    bf = fp.Context(1.0, counts, 8, solver=fp.SOLVER_FDM).energy_forces(tx, tQ, Phi=True)
    off = np.concatenate([[0], np.cumsum(counts)])
    for b, N in enumerate(counts):
        s = fp.Context(1.0, N, 8, solver=fp.SOLVER_FDM).energy_forces(
            torch.from_numpy(xs[b]).cuda(), torch.from_numpy(Qs[b]).cuda(), Phi=True)
        assert _rel(bf["Phi"][off[b]:off[b + 1]].cpu().numpy(), s["Phi"].cpu().numpy()) < 1e-11
        assert _rel(bf["F"][off[b]:off[b + 1]].cpu().numpy(), s["F"].cpu().numpy()) < 1e-11
    m = fp.Context(1.0, counts, 8, solver=fp.SOLVER_FDM, precision=fp.PRECISION_MIXED).energy_forces(tx, tQ, Phi=True)
    for k in ("Phi", "F"):
        assert _rel(m[k].cpu().numpy(), bf[k].cpu().numpy()) < 1e-5, k
    g = fp.Context(1.0, counts, 8, solver=fp.SOLVER_FDM, use_graph=1)
    for _ in range(2):
        og = g.energy_forces(tx, tQ, Phi=True)
        np.testing.assert_array_equal(og["F"].cpu().numpy(), bf["F"].cpu().numpy())
    assert g.stats()["graph_replays"] == 0     # this solver always runs eagerly


@pytest.mark.parametrize("n,q,support", [(16, 3, 0), (8, 1, 1), (8, 4, 0)])
def test_fourier_solver_energy_only_and_screen_families(torch, n, q, support):
    """The Fourier-analysis path of the exact solver (meshes whose edge is a
    power of two): a single real system (energy only: the complex work
    system's imaginary part is empty) and the orders 3 and 6 of the other
    screen families, against the oracle's exact solve."""
    x, Q = workloads.uniform(500, seed=40 + n + q, charges="uniform")
    sup = "27" if support else "one"
    ctx = fp.Context(1.0, len(Q), n, q=q, support=support, solver=fp.SOLVER_FDM)
    Phi, U = ctx.energy(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda())
    st = fep3m.run(x, Q, fep3m.Params(L=1.0, n=n, q=q, support=sup), stages=True)
    phi = ctx.stage("phi").cpu().numpy()
    assert np.abs(phi - st["phi"].ravel()).max() < 1e-11 * np.abs(st["phi"]).max()
    assert _rel(Phi.cpu().numpy(), st["Phi"]) < 1e-10
    assert ctx.stats()["mg_rel_residual"] < 1e-11
