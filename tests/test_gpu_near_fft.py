"""Near-screen field and its transpose through FFTs (near_field = FFT)
against the direct table sums (near_field = DIRECT) on the same inputs.

Both evaluate the same linear maps (the periodic convolution of the element
moments with the tables, and its transpose), so in float64 the results
agree to rounding: Phi, F, dU/dQ and U to 1e-12 relative.  The
oracle parity of the FFT path itself is covered where the parity tests run
with the default options on power-of-two meshes."""
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _both(torch, x, Q, n, **opts):
    tx, tQ = torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda()
    out = {}
    for near in (fp.NEAR_FFT, fp.NEAR_DIRECT):
        ctx = fp.Context(1.0, Q.shape[0] if "counts" not in opts else opts["counts"], n,
                         near_field=near, **{k: v for k, v in opts.items() if k != "counts"})
        assert ctx.stats()["near_fft"] == (near == fp.NEAR_FFT)
        r = ctx.energy_forces(tx, tQ, dUdQ=True, Phi=True)
        out[near] = {k: v.cpu().numpy() for k, v in r.items()}
    return out[fp.NEAR_FFT], out[fp.NEAR_DIRECT]


@pytest.mark.parametrize("wl,n_sr", [("uniform-1k-n8", 3), ("uniform-1k-n8", 2), ("uniform-1k-n8", 1),
                                     ("uniform-100k-n32", 3)])
def test_fft_matches_direct_fp64(torch, wl, n_sr):
    x, Q = workloads.make(wl)
    n = 8 if wl.endswith("n8") else 32
    a, b = _both(torch, x, Q, n, n_sr=n_sr, mg_rtol=1e-13)
    for k in ("Phi", "F", "dUdQ"):
        assert _rel(a[k], b[k]) < 1e-12, k
    assert np.abs(a["U"] - b["U"]).max() < 1e-12 * np.abs(b["U"]).max()


def test_fft_matches_direct_1M_n64(torch):
    """The full-size workload (64^3 elements, 1e6 charges), in the launch
    configuration the benchmark times."""
    x, Q = workloads.make("uniform-1M-n64")
    a, b = _both(torch, x, Q, 64)
    for k in ("Phi", "F", "dUdQ"):
        assert _rel(a[k], b[k]) < 1e-12, k
    assert abs(float(a["U"]) - float(b["U"])) < 1e-12 * abs(float(b["U"]))


def test_fft_matches_direct_batch(torch):
    """A batch of ragged configurations on 16^3 meshes: one transform per
    configuration, one shared spectrum."""
    counts = [2000, 37, 5000, 2]
    rng = np.random.default_rng(21)
    xs = [rng.random((c, 3)) for c in counts]
    Qs = [rng.uniform(-1, 1, c) for c in counts]
    Qs = [q - q.mean() for q in Qs]
    x, Q = np.concatenate(xs), np.concatenate(Qs)
    a, b = _both(torch, x, Q, 16, counts=counts, mg_rtol=1e-13)
    for k in ("Phi", "F", "dUdQ"):
        assert _rel(a[k], b[k]) < 1e-12, k
    assert np.abs(a["U"] - b["U"]).max() < 1e-12 * np.abs(b["U"]).max()


def test_fft_mixed_precision(torch):
    """Mixed precision with the FFT near field (float64 transforms, float32
    element field) against float64."""
    x, Q = workloads.make("uniform-100k-n32")
    tx, tQ = torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda()
    r64 = fp.Context(1.0, len(Q), 32).energy_forces(tx, tQ, dUdQ=True, Phi=True)
    ctx = fp.Context(1.0, len(Q), 32, precision=fp.PRECISION_MIXED)
    assert ctx.stats()["near_fft"] == 1
    rm = ctx.energy_forces(tx, tQ, dUdQ=True, Phi=True)
    for k in ("Phi", "F", "dUdQ"):
        assert _rel(rm[k].cpu().numpy(), r64[k].cpu().numpy()) < 1e-5, k


def test_fft_repeatable_and_graph(torch):
    """Bitwise repeatable calls; a captured graph replays the transforms with
    the same results."""
    x, Q = workloads.make("uniform-1k-n8")
    tx, tQ = torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda()
    ctx = fp.Context(1.0, len(Q), 8, near_field=fp.NEAR_FFT)
    r1 = {k: v.cpu().numpy() for k, v in ctx.energy_forces(tx, tQ, dUdQ=True, Phi=True).items()}
    r2 = {k: v.cpu().numpy() for k, v in ctx.energy_forces(tx, tQ, dUdQ=True, Phi=True).items()}
    for k in r1:
        np.testing.assert_array_equal(r1[k], r2[k])
    g = fp.Context(1.0, len(Q), 8, near_field=fp.NEAR_FFT, use_graph=1)
    for _ in range(3):
        rg = {k: v.cpu().numpy() for k, v in g.energy_forces(tx, tQ, dUdQ=True, Phi=True).items()}
        torch.cuda.synchronize()
        for k in r1:
            np.testing.assert_array_equal(rg[k], r1[k])
    assert g.stats()["graph_replays"] >= 2
