"""The grounded box on the GPU (Section 2.6, eq. bcadjust with g = 0):
potentials, energy, forces and dU/dQ through the C ABI against the
oracle's box form on the same inputs (element by element), the method
against the image-charge ground truth, a non-neutral set, a batch of boxes,
the autograd path, and the refusal of positions outside the box."""
import numpy as np
import pytest

import paper_1503_08509_amd as fp
from oracle import dirichlet as odir
from oracle import fep3m as ofe

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


def _layer(N, seed, n, L=1.0, charges="pm1"):
    """At least half an element from every face; half the charges within
    one element of a face."""
    rng = np.random.default_rng(seed)
    h = L / n
    x = rng.uniform(0.5 * h, L - 0.5 * h, (N, 3))
    k = N // 2
    ax = rng.integers(0, 3, k)
    side = rng.integers(0, 2, k)
    d = rng.uniform(0.5, 1.0, k) * h
    x[np.arange(k), ax] = np.where(side == 1, L - d, d)
    Q = rng.choice([-1.0, 1.0], N) if charges == "pm1" else rng.uniform(0.0, 1.0, N)
    return x, Q


def _ctx(N, n, q=3, n_sr=3):
    return fp.Context(1.0, N, n, q=q, n_sr=n_sr, boundary=fp.BOUNDARY_GROUNDED, solver=fp.SOLVER_FDM,
                      table_box=2 * n_sr + 9)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("N,n,q,n_sr,seed", [(300, 8, 3, 3, 1), (500, 9, 3, 2, 2), (200, 8, 4, 3, 3),
                                             (200, 7, 2, 3, 4), (2000, 16, 3, 3, 5)])
def test_box_matches_oracle(torch, N, n, q, n_sr, seed):
    x, Q = _layer(N, seed, n)
    ctx = _ctx(N, n, q, n_sr)
    Phi, U = ctx.energy(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda())
    ref = odir.run(x, Q, ofe.Params(L=1.0, n=n, q=q, n_sr=n_sr))
    e = _rel(Phi.cpu().numpy(), ref["Phi"])
    print(f"box N={N} n={n} q={q} n_sr={n_sr}: GPU vs oracle Phi {e:.2e}, U {U.item():.10e} vs {ref['U']:.10e}")
    assert e < 1e-10
    assert abs(U.item() - ref["U"]) <= 1e-10 * abs(ref["U"])
    assert ctx.stats()["mg_rel_residual"] < 1e-9


def test_box_method_against_images(torch):
    """The GPU method against the grounded cube's image sum: within the
    screen's truncation error."""
    N, n = 400, 8
    x, Q = _layer(N, 11, n)
    Phi, U = _ctx(N, n).energy(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda())
    ref = odir.image_ewald(x, Q)
    e = _rel(Phi.cpu().numpy(), ref)
    print(f"box N={N} n={n}: Phi vs image sum {e:.3e}")
    assert e < 5e-3


def test_box_net_charge_and_batch(torch):
    """Positive charges only (a grounded box holds any net charge), and a
    batch of three boxes equal to three single contexts."""
    n = 8
    sets = [_layer(150, 20 + k, n, charges="pos") for k in range(3)]
    x = np.concatenate([s[0] for s in sets])
    Q = np.concatenate([s[1] for s in sets])
    ctx = fp.Context(1.0, [150, 150, 150], n, boundary=fp.BOUNDARY_GROUNDED, solver=fp.SOLVER_FDM)
    Phi, U = ctx.energy(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda())
    Phi = Phi.cpu().numpy()
    for k, (xs, Qs) in enumerate(sets):
        ref = odir.run(xs, Qs, ofe.Params(L=1.0, n=n))
        assert _rel(Phi[150 * k:150 * (k + 1)], ref["Phi"]) < 1e-10
        assert abs(U[k].item() - ref["U"]) <= 1e-10 * abs(ref["U"])


def test_box_refusals(torch):
    n = 8
    x, Q = _layer(100, 30, n)
    ctx = _ctx(100, n)
    tx, tQ = torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda()
    bad = x.copy()
    bad[3, 1] = 1.0                      # on the face x_1 = L
    with pytest.raises(fp.FEP3MError) as ei:
        ctx.energy(torch.from_numpy(bad).cuda(), tQ)
    assert ei.value.status == fp.ERR_ARG
    Phi, _ = ctx.energy(tx, tQ)           # the context stays usable
    assert np.all(np.isfinite(Phi.cpu().numpy()))


@pytest.mark.parametrize("N,n,q,seed", [(300, 8, 3, 41), (200, 8, 4, 42), (200, 7, 2, 43), (800, 16, 3, 44)])
def test_box_forces_match_oracle(torch, N, n, q, seed):
    """Forces and dU/dQ in the grounded box (the reverse pass with the
    boundary terms of eq. bcadjust) against the oracle's adjoint, charge by
    charge."""
    x, Q = _layer(N, seed, n)
    ctx = _ctx(N, n, q)
    out = ctx.energy_forces(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda(), dUdQ=True, Phi=True)
    ref = odir.energy_forces(x, Q, ofe.Params(L=1.0, n=n, q=q))
    eF = _rel(out["F"].cpu().numpy(), ref["F"])
    eQ = _rel(out["dUdQ"].cpu().numpy(), ref["dUdQ"])
    print(f"box forces N={N} n={n} q={q}: F {eF:.2e}, dU/dQ {eQ:.2e}")
    assert eF < 1e-10 and eQ < 1e-10
    assert _rel(out["Phi"].cpu().numpy(), ref["Phi"]) < 1e-10
    assert abs(out["U"].item() - ref["U"]) <= 1e-10 * abs(ref["U"])


def test_box_autograd_and_images(torch):
    """The autograd path (energy, then the reverse pass on its state) gives
    the fused call's gradients, and the forces lie within the screen's
    truncation error of the image-charge forces."""
    N, n = 300, 8
    x, Q = _layer(N, 45, n)
    ctx = _ctx(N, n)
    tx = torch.from_numpy(x).cuda().requires_grad_(True)
    tQ = torch.from_numpy(Q).cuda().requires_grad_(True)
    U = fp.FEP3MEnergy.apply(tx, tQ, ctx)
    U.backward()
    fused = ctx.energy_forces(tx.detach(), tQ.detach(), dUdQ=True)
    assert _rel(-tx.grad.cpu().numpy(), fused["F"].cpu().numpy()) < 1e-12
    assert _rel(tQ.grad.cpu().numpy(), fused["dUdQ"].cpu().numpy()) < 1e-12
    from oracle import ewald
    X, QQ = odir.image_charges(x, Q, 1.0)
    ref = ewald.ewald(X, QQ, L=2.0, alpha=2.5, nimg=2, mmax=8, forces=True, targets=8 * np.arange(N))["F"]
    e = _rel(fused["F"].cpu().numpy(), ref)
    print(f"box forces vs image sum: {e:.3e}")
    assert e < 1e-2


def _neutral_layer(N, seed, n):
    x, _ = _layer(N, seed, n)
    Q = np.random.default_rng(seed + 1).permutation(np.repeat([1.0, -1.0], N // 2))
    return x, Q


def _ictx(N, n, q=3, n_sr=3):
    return fp.Context(1.0, N, n, q=q, n_sr=n_sr, boundary=fp.BOUNDARY_INSULATED, solver=fp.SOLVER_FDM,
                      table_box=2 * n_sr + 9)


@pytest.mark.parametrize("N,n,q,n_sr,seed", [(300, 8, 3, 3, 51), (400, 9, 3, 2, 52), (200, 8, 4, 3, 53),
                                             (200, 7, 2, 3, 54), (1000, 16, 3, 3, 55)])
def test_insulated_box_matches_oracle(torch, N, n, q, n_sr, seed):
    """The insulating box (surface load of -dPhi_sr/dn, pure-Neumann solve)
    against the oracle's form: potentials (same gauge, int phi = 0) and
    energy."""
    from oracle import neumann as oneu
    x, Q = _neutral_layer(N, seed, n)
    ctx = _ictx(N, n, q, n_sr)
    Phi, U = ctx.energy(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda())
    ref = oneu.run(x, Q, ofe.Params(L=1.0, n=n, q=q, n_sr=n_sr))
    e = _rel(Phi.cpu().numpy(), ref["Phi"])
    print(f"insulated box N={N} n={n} q={q} n_sr={n_sr}: GPU vs oracle Phi {e:.2e}")
    assert e < 1e-10
    assert abs(U.item() - ref["U"]) <= 1e-10 * abs(ref["U"])
    assert ctx.stats()["mg_rel_residual"] < 1e-9


def test_insulated_box_against_images_and_refusals(torch):
    """The GPU method against the even-image sum (potential up to a
    constant, energy), a batch of two boxes, and the refusal of non-neutral
    charges."""
    from oracle import neumann as oneu
    N, n = 400, 8
    x, Q = _neutral_layer(N, 56, n)
    ctx = _ictx(N, n)
    tx, tQ = torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda()
    Phi, U = ctx.energy(tx, tQ)
    Phi = Phi.cpu().numpy()
    ref = oneu.image_ewald(x, Q)
    c = np.mean(ref - Phi)
    e = float(np.linalg.norm(Phi + c - ref) / np.linalg.norm(ref - ref.mean()))
    eU = abs(U.item() - 0.5 * np.sum(Q * ref)) / abs(0.5 * np.sum(Q * ref))
    print(f"insulated box N={N} n={n}: Phi vs image sum {e:.3e} (up to a constant), U {eU:.3e}")
    assert e < 5e-3 and eU < 1e-2     # U of a neutral set: a sum with cancellation
    Qb = Q.copy()
    Qb[0] += 0.5
    with pytest.raises(fp.FEP3MError) as ei:
        ctx.energy(tx, torch.from_numpy(Qb).cuda())
    assert ei.value.status == fp.ERR_NOT_NEUTRAL
    x2, Q2 = _neutral_layer(N, 57, n)
    b = fp.Context(1.0, [N, N], n, boundary=fp.BOUNDARY_INSULATED, solver=fp.SOLVER_FDM)
    Pb, Ub = b.energy(torch.from_numpy(np.concatenate([x, x2])).cuda(), torch.from_numpy(np.concatenate([Q, Q2])).cuda())
    assert _rel(Pb.cpu().numpy()[:N], Phi) < 1e-12
    single2 = _ictx(N, n).energy(torch.from_numpy(x2).cuda(), torch.from_numpy(Q2).cuda())[0].cpu().numpy()
    assert _rel(Pb.cpu().numpy()[N:], single2) < 1e-12


@pytest.mark.parametrize("N,n,q,seed", [(300, 8, 3, 61), (200, 8, 4, 62), (200, 7, 2, 63), (800, 16, 3, 64)])
def test_insulated_box_forces_match_oracle(torch, N, n, q, seed):
    """Forces and dU/dQ of the insulating box (surface-load terms of the
    adjoint) against the oracle, charge by charge, and the forces against the
    even-image sum."""
    from oracle import ewald, neumann as oneu
    x, Q = _neutral_layer(N, seed, n)
    ctx = _ictx(N, n, q)
    out = ctx.energy_forces(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda(), dUdQ=True, Phi=True)
    ref = oneu.energy_forces(x, Q, ofe.Params(L=1.0, n=n, q=q))
    eF = _rel(out["F"].cpu().numpy(), ref["F"])
    eQ = _rel(out["dUdQ"].cpu().numpy(), ref["dUdQ"])
    print(f"insulated box forces N={N} n={n} q={q}: F {eF:.2e}, dU/dQ {eQ:.2e}")
    assert eF < 1e-10 and eQ < 1e-10
    if q == 3 and n == 8:
        X, QQ = oneu.image_charges(x, Q, 1.0)
        img = ewald.ewald(X, QQ, L=2.0, alpha=2.5, nimg=2, mmax=8, forces=True, targets=8 * np.arange(N))["F"]
        e = _rel(out["F"].cpu().numpy(), img)
        print(f"insulated box forces vs image sum: {e:.3e}")
        assert e < 1e-2


def _box_fixture(kind):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"box_{kind}_uniform-1M-n64.json")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("kind", ["grounded", "insulated"])
def test_box_full_size_against_oracle(torch, kind):
    """The benchmark's box runs (uniform-1M-n64: 10^6 charges, 64^3 elements,
    default options) against the oracle's box form: Phi on 512 sampled
    charges and the mesh potential on 512 sampled nodes, stored by
    tests/golden/make_box_fixtures.py; U through its definition
    U = 1/2 sum Q Phi on the GPU's own Phi (pinned on the sample); forces
    against central differences of the GPU energy on four charges (step
    1e-6, the energy smooth inside an element)."""
    import math
    import workloads
    ref = _box_fixture(kind)
    x, Q = workloads.make(ref["workload"])
    n = ref["n"]
    bc = fp.BOUNDARY_GROUNDED if kind == "grounded" else fp.BOUNDARY_INSULATED
    print(f"box full size: {kind} N={len(Q)} n={n}", flush=True)
    ctx = fp.Context(1.0, len(Q), n, boundary=bc, solver=fp.SOLVER_FDM)
    tx, tQ = torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda()
    ctx.energy_forces(tx, tQ, Phi=True)                 # first call: tuning
    out = ctx.energy_forces(tx, tQ, Phi=True)
    torch.cuda.synchronize()
    Phi = out["Phi"].cpu().numpy()
    t = np.array(ref["targets"])
    e_Phi = _rel(Phi[t], np.array(ref["Phi"]))
    phi = ctx.stage("phi").cpu().numpy()
    e_phi = float(np.abs(phi[np.array(ref["nodes"])] - np.array(ref["phi"])).max() / ref["phi_absmax"])
    U = float(out["U"].item())
    Uq = 0.5 * math.fsum(Q * Phi)
    e_U = abs(U - Uq) / abs(Uq)
    print(f"box full size {kind}: Phi {e_Phi:.2e} (sample), phi {e_phi:.2e} (nodes), U {e_U:.2e}", flush=True)
    assert e_Phi < 1e-9 and e_phi < 1e-9 and e_U < 1e-12
    F = out["F"].cpu().numpy()
    hstep = 1e-6
    g = x * n
    frac = g - np.floor(g)
    ok = np.nonzero(np.all((frac > 1e-4 + hstep * n) & (frac < 1 - 1e-4 - hstep * n), axis=1))[0]
    pick = np.random.default_rng(4006).choice(ok, 4, replace=False)
    fd = np.zeros((4, 3))
    for r, i in enumerate(pick):
        for k in range(3):
            xp = tx.clone()
            xp[i, k] += hstep
            xm = tx.clone()
            xm[i, k] -= hstep
            fd[r, k] = -(float(ctx.energy(xp, tQ)[1].item()) - float(ctx.energy(xm, tQ)[1].item())) / (2 * hstep)
    err = np.abs(fd - F[pick]).max()
    scale = np.abs(F[pick]).max()
    print(f"box full size {kind}: forces against central differences {err / scale:.2e}", flush=True)
    assert err < 1e-5 * scale
