"""Write the oracle's potentials, forces and charge derivatives of sampled
charges, and its mesh potential at sampled nodes, for the uniform-1M-n64
workload (10^6 charges, 64^3 elements, 7^3 near block) with the
27-element screens of Section 2.1 of degree q = 1 to 4 and the
one-element screens of degree 2 and 4 (Section 5), to
tests/golden/family_q<q>_<support>_uniform-1M-n64.json, for the full-size
GPU parity tests of the screen families.  Calls only the oracle
(oracle.adjoint.energy_forces with targets, pinned in
tests/test_oracle_screens27.py and tests/test_oracle_adjoint.py) on the
seeded inputs of workloads.py.

    python tests/golden/make_family_fixtures.py [q:support ...]   (default 1:27 2:27 3:27 4:27 2:one 4:one)

About 0.5, 1, 2, 3.5, 0.2 and 3 minutes on 8 cores."""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import adjoint, fep3m  # noqa: E402

WORKLOAD = "uniform-1M-n64"
NSAMPLE = 256


def make(q, support):
    x, Q = workloads.make(WORKLOAD)
    n = 64
    P = fep3m.Params(L=1.0, n=n, q=q, support=support)
    rng = np.random.default_rng(5000 + q)
    targets = np.sort(rng.choice(len(Q), NSAMPLE, replace=False))
    t0 = time.time()
    out = adjoint.energy_forces(x, Q, P, targets=targets)
    phi = out["phi"].ravel()
    nodes = np.sort(rng.choice(phi.size, 512, replace=False))
    rec = {"workload": WORKLOAD, "q": q, "support": support, "n": n, "n_sr": P.n_sr, "mesh_order": P.p,
           "oracle": "oracle.adjoint.energy_forces (targets)", "seconds": round(time.time() - t0, 1),
           "targets": targets.tolist(), "Phi": out["Phi"].tolist(), "F": out["F"].tolist(),
           "dUdQ": out["dUdQ"].tolist(), "nodes": nodes.tolist(), "phi": phi[nodes].tolist(),
           "phi_absmax": float(np.abs(phi).max())}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"family_q{q}_{support}_{WORKLOAD}.json")
    with open(path, "w") as f:
        json.dump(rec, f)
    print(f"wrote {path} ({rec['seconds']} s)", flush=True)


if __name__ == "__main__":
    for spec in (sys.argv[1:] or ["1:27", "2:27", "3:27", "4:27", "2:one", "4:one"]):
        q, support = spec.split(":")
        make(int(q), support)
