"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on
the same seeded inputs.  Integer stages (sort, element starts) must match
bit for bit; floating stages within the stated tolerances; the end result
Phi within 1e-6 relative RMS (the FP64 target) and U within 1e-6."""
import numpy as np
import pytest

import paper_1503_08509_amd as fp
import workloads
from oracle import fep3m

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


def _rel_rms(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _gpu(torch, x, Q, L, n, **opts):
    ctx = fp.Context(L, len(Q), n, **opts)
    tx = torch.from_numpy(x).cuda()
    tQ = torch.from_numpy(Q).cuda()
    Phi, U = ctx.energy(tx, tQ)
    torch.cuda.synchronize()
    return ctx, Phi.cpu().numpy(), float(U.item())


def _stable_order(e_lin, n):
    return np.argsort(e_lin, kind="stable"), np.concatenate([[0], np.cumsum(np.bincount(e_lin, minlength=n**3))])


@pytest.mark.parametrize("near", [fp.NEAR_FFT, fp.NEAR_DIRECT])
def test_config1_stage_parity(torch, near):
    x, Q = workloads.make("uniform-1k-n8")
    L, n = 1.0, 8
    ref = fep3m.run(x, Q, fep3m.Params(L=L, n=n), stages=True)
    ctx, Phi, U = _gpu(torch, x, Q, L, n, mg_rtol=1e-13, near_field=near)     # tight solve: stages exact
    assert ctx.stats()["near_fft"] == (near == fp.NEAR_FFT)
    order, start = _stable_order(ref["e_lin"], n)
    np.testing.assert_array_equal(ctx.stage("perm").cpu().numpy(), order)
    np.testing.assert_array_equal(ctx.stage("start").cpu().numpy(), start)
    C = ctx.stage("C").cpu().numpy().reshape(-1, 8)
    assert np.abs(C - ref["C"]).max() < 1e-13
    b = ctx.stage("b").cpu().numpy()
    assert np.abs(b - ref["b"].ravel()).max() < 1e-12 * np.abs(ref["b"]).max()
    phi = ctx.stage("phi").cpu().numpy()
    assert np.abs(phi - ref["phi"].ravel()).max() < 1e-9 * np.abs(ref["phi"]).max()
    Pp = ctx.stage("Phi_p").cpu().numpy()
    np.testing.assert_allclose(Pp, ref["Phi_p"], rtol=1e-12, atol=1e-12 * np.abs(ref["Phi_p"]).max())
    Pm = ctx.stage("Phi_m").cpu().numpy()
    assert np.abs(Pm - ref["Phi_m"]).max() < 1e-8 * np.abs(ref["Phi"]).max()
    assert _rel_rms(Phi, ref["Phi"]) < 1e-6
    assert abs(U - ref["U"]) < 1e-6 * abs(ref["U"])
    st = ctx.stats()
    assert st["mg_rel_residual"] <= 1e-13
    counts = np.diff(start)
    assert st["max_per_element"] == counts.max()


def test_tables_stage_matches_host_precompute(torch):
    x, Q = workloads.uniform(20, seed=3)
    ctx, _, _ = _gpu(torch, x, Q, 1.0, 8)
    T = ctx.stage("T").cpu().numpy().reshape(8, 343, 216)
    np.testing.assert_array_equal(T, fp.host_tables(3, 3, 15))


def test_pair_count(torch):
    x, Q = workloads.make("uniform-1k-n8")
    n = 8
    ctx, _, _ = _gpu(torch, x, Q, 1.0, n)
    e, e_lin, _ = fep3m.bin_particles(x, 1.0, n)
    counts = np.bincount(e_lin, minlength=n**3).reshape(n, n, n)   # [ez, ey, ex]
    block = np.zeros_like(counts)
    for dz in range(-3, 4):
        for dy in range(-3, 4):
            for dx in range(-3, 4):
                block += np.roll(counts, (dz, dy, dx), axis=(0, 1, 2))
    expect = int(np.sum(counts * block) - len(Q))
    assert ctx.stats()["near_pairs"] == expect


@pytest.mark.parametrize("case", ["two", "three", "ragged17_n7", "ragged17_n9", "faces"])
def test_small_and_ragged(torch, case):
    rng = np.random.default_rng(42)
    L = 1.0
    if case == "two":
        n, x, Q = 8, np.array([[0.1, 0.2, 0.3], [0.55, 0.6, 0.05]]), np.array([1.0, -1.0])
    elif case == "three":
        n, x, Q = 8, rng.random((3, 3)), np.array([1.0, -0.5, -0.5])
    elif case.startswith("ragged17"):
        n = int(case.split("_n")[1])
        x = rng.random((17, 3)) * 3.0 - 1.0          # outside [0, L): wrapped
        Q = rng.uniform(-1, 1, 17)
        Q -= Q.mean()
    else:  # positions exactly on element faces, on L and at 0
        n = 8
        x = np.array([[0.0, 0.125, 0.5], [1.0, 0.25, 0.375], [0.875, 1.0, 0.0],
                      [-0.125, 0.5, 0.625], [0.3, 0.7, 0.9], [0.5, 0.5, 0.5]])
        Q = np.array([1.0, -1.0, 0.5, -0.5, 2.0, -2.0])
    ref = fep3m.run(x, Q, fep3m.Params(L=L, n=n), stages=True)
    ctx, Phi, U = _gpu(torch, x, Q, L, n, mg_rtol=1e-12)
    order, start = _stable_order(ref["e_lin"], n)
    np.testing.assert_array_equal(ctx.stage("perm").cpu().numpy(), order)
    assert _rel_rms(Phi, ref["Phi"]) < 1e-8
    assert abs(U - ref["U"]) < 1e-8 * max(1.0, abs(ref["U"]))


def test_config2_sampled_parity(torch):
    """100k charges, 32^3 mesh: mesh stages compared in full, Phi on a
    seeded sample of 400 charges the oracle evaluates one by one."""
    x, Q = workloads.make("uniform-100k-n32")
    L, n = 1.0, 32
    ctx, Phi, U = _gpu(torch, x, Q, L, n)
    rng = np.random.default_rng(7)
    tgt = np.sort(rng.choice(len(Q), 400, replace=False))
    ref = fep3m.run(x, Q, fep3m.Params(L=L, n=n), targets=tgt, stages=True)
    phi = ctx.stage("phi").cpu().numpy()         # default solve tolerance (relative residual 1e-7)
    assert np.abs(phi - ref["phi"].ravel()).max() < 5e-7 * np.abs(ref["phi"]).max()
    assert _rel_rms(Phi[tgt], ref["Phi"]) < 1e-6
    # every charge: the energy is consistent with the returned potentials
    assert abs(U - 0.5 * float(np.sum(Q * Phi))) < 1e-10 * abs(U)


def test_mesh_aligned_translation_invariance(torch):
    x, Q = workloads.make("uniform-1k-n8")
    # the multigrid hierarchy is not shift-equivariant: compare tight solves
    _, P1, U1 = _gpu(torch, x, Q, 1.0, 8, mg_rtol=1e-13)
    _, P2, U2 = _gpu(torch, x + np.array([2, -3, 5]) / 8.0, Q, 1.0, 8, mg_rtol=1e-13)
    assert np.abs(P1 - P2).max() < 1e-10 * np.abs(P1).max()


def test_repeatable_bitwise(torch):
    x, Q = workloads.make("uniform-1k-n8")
    ctx = fp.Context(1.0, len(Q), 8)
    tx, tQ = torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda()
    a = ctx.potential(tx, tQ).cpu().numpy()
    b = ctx.potential(tx, tQ).cpu().numpy()
    np.testing.assert_array_equal(a, b)


def test_error_paths(torch):
    x, Q = workloads.uniform(64, seed=1)
    ctx = fp.Context(1.0, 64, 8, mg_rtol=1e-12)
    tx = torch.from_numpy(x).cuda()
    with pytest.raises(fp.FEP3MError) as ei:
        ctx.potential(tx, torch.from_numpy(Q + 0.1).cuda())
    assert ei.value.status == fp.ERR_NOT_NEUTRAL
    xb = x.copy()
    xb[5, 1] = np.nan
    with pytest.raises(fp.FEP3MError) as ei:
        ctx.potential(torch.from_numpy(xb).cuda(), torch.from_numpy(Q).cuda())
    assert ei.value.status == fp.ERR_NONFINITE
    # the context still works after an error
    Phi = ctx.potential(tx, torch.from_numpy(Q).cuda())
    ref = fep3m.run(x, Q, fep3m.Params(L=1.0, n=8))
    assert _rel_rms(Phi.cpu().numpy(), ref["Phi"]) < 1e-8
