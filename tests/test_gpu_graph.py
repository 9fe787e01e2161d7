"""Graph mode: each evaluation replayed as one captured hipGraph.  Every
replay must equal an eager evaluation of the same inputs bit for bit; the
inputs change in place between replays (same buffers, new positions), with
eager torch work and synchronisations in between, and a failing input check
after a replay must raise and leave the context usable."""
import numpy as np
import pytest

import paper_1503_08509_amd as fp
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


@pytest.mark.parametrize("counts,n,precision", [(1000, 8, fp.PRECISION_FP64),
                                                 (100_000, 32, fp.PRECISION_MIXED),
                                                 ([300, 1200, 40, 700], 8, fp.PRECISION_FP64),
                                                 # 64^3 elements: the captured graph forks the pair sum
                                                 # onto the second stream and joins it before interpolation
                                                 (100_000, 64, fp.PRECISION_FP64)])
def test_graph_replays_equal_eager(torch, counts, n, precision):
    N = counts if np.isscalar(counts) else sum(counts)
    rng = np.random.default_rng(11)
    x0 = rng.random((N, 3))
    Q = rng.uniform(-1, 1, N)
    if np.isscalar(counts):
        Q -= Q.mean()
    else:
        off = np.concatenate([[0], np.cumsum(counts)])
        for b in range(len(counts)):
            Q[off[b]:off[b + 1]] -= Q[off[b]:off[b + 1]].mean()
    g = fp.Context(1.0, counts, n, precision=precision, use_graph=1)
    e = fp.Context(1.0, counts, n, precision=precision)
    tx = torch.from_numpy(x0).cuda()
    tQ = torch.from_numpy(Q).cuda()
    for k in range(4):
        if k:
            tx += 1e-3 * torch.from_numpy(rng.standard_normal((N, 3))).cuda()   # in place: same buffer
        scratch = (tx * 2.0).sum()      # eager work on the caller's stream between replays
        og = g.energy_forces(tx, tQ, dUdQ=True, Phi=True)
        torch.cuda.synchronize()
        oe = e.energy_forces(tx, tQ, dUdQ=True, Phi=True)
        for key in ("U", "F", "Phi", "dUdQ"):
            np.testing.assert_array_equal(og[key].cpu().numpy(), oe[key].cpu().numpy(), err_msg=f"{key} call {k}")
        assert float(scratch) == float((tx * 2.0).sum())
    assert g.stats()["graph_replays"] >= 2
    assert g.stats()["near_pairs"] == e.stats()["near_pairs"]


def test_graph_replay_input_errors(torch):
    x, Q = workloads.uniform(500, seed=12)
    g = fp.Context(1.0, 500, 8, use_graph=1)
    tx = torch.from_numpy(x).cuda()
    tQ = torch.from_numpy(Q).cuda()
    ref = g.energy(tx, tQ)[1].item()
    g.energy(tx, tQ)                      # replay
    tQ[3] += 0.5                          # no longer neutral
    with pytest.raises(fp.FEP3MError) as ei:
        g.energy(tx, tQ)
    assert ei.value.status == fp.ERR_NOT_NEUTRAL
    tQ[3] -= 0.5
    assert g.energy(tx, tQ)[1].item() == ref


def test_graph_replayed_energy_then_backward(torch):
    """Energy-only graph replays followed by the reverse pass (autograd): each
    backward call must solve the adjoint system of the replayed forward, not
    reuse the previous call's, and equal an eager energy_forces call."""
    N, n = 800, 8
    rng = np.random.default_rng(21)
    Q = rng.uniform(-1, 1, N)
    Q -= Q.mean()
    g = fp.Context(1.0, N, n, use_graph=1)
    e = fp.Context(1.0, N, n)
    tQ = torch.from_numpy(Q).cuda()
    tx = torch.from_numpy(rng.random((N, 3))).cuda()
    for k in range(4):
        if k:
            tx = (tx + 1e-2 * torch.from_numpy(rng.standard_normal((N, 3))).cuda()) % 1.0
        xg = tx.clone().requires_grad_(True)
        U = fp.FEP3MEnergy.apply(xg, tQ, g)
        U.sum().backward()
        oe = e.energy_forces(tx, tQ)
        np.testing.assert_allclose(-xg.grad.cpu().numpy(), oe["F"].cpu().numpy(), rtol=0, atol=1e-9 * float(
            oe["F"].abs().max()), err_msg=f"call {k}")
    assert g.stats()["graph_replays"] >= 2
