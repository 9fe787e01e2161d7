"""The screen families beyond the one-element q = 3 screen on the GPU: the
27-element screens of Section 2.1 (q = 1..4) and one-element screens of
degree 2 and 4 (Section 5), through the C ABI against the FP64 oracle on
the same seeded inputs: stage by stage (sort, moments, load, mesh
potential, pair sum, mesh term), Phi, U, and the adjoint (F, dU/dQ)."""
import numpy as np
import pytest

import paper_1503_08509_amd as fp
import workloads
from oracle import adjoint, fep3m

pytestmark = pytest.mark.gpu

SUP = {"one": fp.SUPPORT_ONE, "27": fp.SUPPORT_27}


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    assert _t.cuda.is_available()
    return _t


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# (q, support, n_sr): the degree-4 families on a 3^3 near block keep the
# oracle's table computation short; the rest use the paper's 7^3 block
FAMILIES = [(1, "27", 3), (2, "27", 3), (3, "27", 2), (4, "27", 1), (2, "one", 3), (4, "one", 2)]


@pytest.mark.parametrize("q,support,nsr", FAMILIES)
def test_family_stage_and_force_parity(torch, q, support, nsr):
    x, Q = workloads.uniform(600, seed=100 + q, charges="uniform")
    n = 8
    print(f"screens: q={q} support={support} n_sr={nsr} N={len(Q)} n={n}", flush=True)
    P = fep3m.Params(L=1.0, n=n, q=q, support=support, n_sr=nsr)
    ref = adjoint.energy_forces(x, Q, P)
    fw = fep3m.run(x, Q, P, stages=True)
    ctx = fp.Context(1.0, len(Q), n, q=q, support=SUP[support], n_sr=nsr, table_box=2 * nsr + 9, mg_rtol=1e-13)
    st = ctx.stats()
    assert st["near_fft"] == 0
    out = ctx.energy_forces(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda(), dUdQ=True, Phi=True)
    torch.cuda.synchronize()
    order = np.argsort(fw["e_lin"], kind="stable")
    np.testing.assert_array_equal(ctx.stage("perm").cpu().numpy(), order)
    na = (P.d + 1) ** 3
    C = ctx.stage("C").cpu().numpy().reshape(-1, na)
    assert np.abs(C - fw["C"]).max() < 1e-13
    b = ctx.stage("b").cpu().numpy()
    assert np.abs(b - fw["b"].ravel()).max() < 1e-12 * np.abs(fw["b"]).max()
    phi = ctx.stage("phi").cpu().numpy()
    assert np.abs(phi - fw["phi"].ravel()).max() < 1e-9 * np.abs(fw["phi"]).max()
    np.testing.assert_allclose(ctx.stage("Phi_p").cpu().numpy(), fw["Phi_p"], rtol=1e-12,
                               atol=1e-12 * np.abs(fw["Phi_p"]).max())
    assert np.abs(ctx.stage("Phi_m").cpu().numpy() - fw["Phi_m"]).max() < 1e-8 * np.abs(fw["Phi"]).max()
    T = ctx.stage("T").cpu().numpy()
    np.testing.assert_array_equal(T, fp.host_tables(q, nsr, 2 * nsr + 9, support).ravel())
    errs = {"Phi": _rel(out["Phi"].cpu().numpy(), ref["Phi"]), "F": _rel(out["F"].cpu().numpy(), ref["F"]),
            "dUdQ": _rel(out["dUdQ"].cpu().numpy(), ref["dUdQ"]),
            "U": abs(float(out["U"].item()) - ref["U"]) / abs(ref["U"])}
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < 1e-9, (k, v)


@pytest.mark.parametrize("q,support", [(2, "27"), (4, "one")])
def test_family_ragged_and_batch(torch, q, support):
    """Ragged sizes on an odd mesh (n = 7: separate residual and restriction,
    tiles cut by the mesh edge) and a batch of uneven configurations, each
    equal to its single-configuration run and to the oracle."""
    rng = np.random.default_rng(7 * q)
    counts = [17, 2, 300]
    xs = [rng.random((N, 3)) for N in counts]
    Qs = []
    for N in counts:
        Qv = rng.uniform(-1, 1, N)
        Qs.append(Qv - Qv.mean())
    n = 7
    P = fep3m.Params(L=1.0, n=n, q=q, support=support, n_sr=2)
    bctx = fp.Context(1.0, counts, n, q=q, support=SUP[support], n_sr=2, table_box=13, mg_rtol=1e-13)
    out = bctx.energy_forces(torch.from_numpy(np.concatenate(xs)).cuda(), torch.from_numpy(np.concatenate(Qs)).cuda(),
                             dUdQ=True, Phi=True)
    off = bctx.offsets
    for b_, N in enumerate(counts):
        print(f"screens batch: q={q} support={support} config {b_} N={N}", flush=True)
        ref = adjoint.energy_forces(xs[b_], Qs[b_], P)
        sl = slice(off[b_], off[b_ + 1])
        for k in ("Phi", "F", "dUdQ"):
            assert _rel(out[k][sl].cpu().numpy(), ref[k]) < 1e-9, (b_, k)
        assert abs(float(out["U"][b_]) - ref["U"]) < 1e-9 * abs(ref["U"])
        ctx = fp.Context(1.0, N, n, q=q, support=SUP[support], n_sr=2, table_box=13, mg_rtol=1e-13)
        one = ctx.energy_forces(torch.from_numpy(xs[b_]).cuda(), torch.from_numpy(Qs[b_]).cuda(), dUdQ=True, Phi=True)
        for k in ("Phi", "F", "dUdQ"):
            assert _rel(out[k][sl].cpu().numpy(), one[k].cpu().numpy()) < 1e-12, (b_, k)


@pytest.mark.parametrize("q,support", [(1, "27"), (2, "27"), (3, "27"), (4, "27"), (2, "one"), (4, "one")])
def test_family_full_size_against_oracle(torch, q, support):
    """Screen families at the benchmark's full size (uniform-1M-n64, 7^3
    near block, default options: multigrid at 1e-7, the matrix-core near
    field and moment adjoint, the separable load and lambda passes of the
    27-element screens): 27-element q = 1 (order-3 mesh, the direct
    8-moment adjoint), q = 2, 3, 4 (q = 4: 125 moments, order-6 mesh),
    one-element q = 2 (one moment: the table sums on the vector units) and
    q = 4 (order-6 mesh); Phi, F and dU/dQ on 256
    sampled charges and the mesh potential on 512 sampled nodes against the
    oracle's values stored by tests/golden/make_family_fixtures.py; U
    through its definition on the GPU's own Phi.  Gate 1e-6 (the solver
    tolerance moves the results by about 1e-8).  The 27-element q = 4
    screens' mesh potential is about 100 times larger than the others'
    (max |phi| 9e3 against 70-90) and cancels against the near-screen
    field, so the default tolerance moves their Phi by about 3e-7; that
    family is solved to 1e-11 here and gated at 1e-9 (measured 2e-11),
    which shows the difference is the solver's and not the kernels'."""
    import json
    import math
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        f"family_q{q}_{support}_uniform-1M-n64.json")
    with open(path) as f:
        ref = json.load(f)
    x, Q = workloads.make(ref["workload"])
    n = ref["n"]
    print(f"family full size: support {support} q={q} N={len(Q)} n={n}", flush=True)
    tight = (q, support) == (4, "27")
    ctx = fp.Context(1.0, len(Q), n, q=q, support=SUP[support], **({"mg_rtol": 1e-11} if tight else {}))
    tx, tQ = torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda()
    ctx.energy_forces(tx, tQ, dUdQ=True, Phi=True)          # first call: tuning
    out = ctx.energy_forces(tx, tQ, dUdQ=True, Phi=True)
    torch.cuda.synchronize()
    t = np.array(ref["targets"])
    Phi = out["Phi"].cpu().numpy()
    errs = {"Phi": _rel(Phi[t], np.array(ref["Phi"])),
            "F": _rel(out["F"].cpu().numpy()[t], np.array(ref["F"])),
            "dUdQ": _rel(out["dUdQ"].cpu().numpy()[t], np.array(ref["dUdQ"]))}
    phi = ctx.stage("phi").cpu().numpy()
    errs["phi"] = float(np.abs(phi[np.array(ref["nodes"])] - np.array(ref["phi"])).max() / ref["phi_absmax"])
    Uq = 0.5 * math.fsum(Q * Phi)
    errs["U"] = abs(float(out["U"].item()) - Uq) / abs(Uq)
    print(f"family full size {support} q={q}:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    for k, v in errs.items():
        assert v < (1e-9 if tight else 1e-6), (k, v)
