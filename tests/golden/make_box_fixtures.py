"""Write the oracle's potentials of sampled charges, and its mesh potential
at sampled nodes, for the uniform-1M-n64 workload (10^6 charges, 64^3
elements, one-element q = 3 screens, 7^3 near block) in the grounded and
the insulating box of Section 2.6, to tests/golden/box_<kind>_uniform-1M-n64.json,
for the full-size GPU parity tests.  Calls only the oracle's box forms
(oracle.dirichlet, oracle.neumann, pinned in tests/test_oracle_dirichlet.py
and tests/test_oracle_neumann.py) on the seeded inputs of workloads.py.

    python tests/golden/make_box_fixtures.py [grounded|insulated ...]

About 3 (grounded) and 6 (insulating) minutes on 8 cores."""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import dirichlet, fep3m, neumann  # noqa: E402

WORKLOAD = "uniform-1M-n64"
NSAMPLE = 512
SEEDS = {"grounded": 4004, "insulated": 4005}


def make(kind):
    x, Q = workloads.make(WORKLOAD)
    n = 64
    P = fep3m.Params(L=1.0, n=n)
    rng = np.random.default_rng(SEEDS[kind])
    targets = np.sort(rng.choice(len(Q), NSAMPLE, replace=False))
    Pn = P.p * n + 1
    nodes = np.sort(rng.choice(Pn ** 3, NSAMPLE, replace=False))
    t0 = time.time()
    form = dirichlet if kind == "grounded" else neumann
    out = form.run(x, Q, P, targets=targets, stages=True)
    phi = out["phi"].ravel()
    rec = {"workload": WORKLOAD, "kind": kind, "n": n, "q": P.q, "n_sr": P.n_sr,
           "oracle": f"oracle.{form.__name__.split('.')[-1]}.run", "seconds": round(time.time() - t0, 1),
           "targets": targets.tolist(), "Phi": out["Phi"].tolist(),
           "nodes": nodes.tolist(), "phi": phi[nodes].tolist(), "phi_absmax": float(np.abs(phi).max())}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"box_{kind}_{WORKLOAD}.json")
    with open(path, "w") as f:
        json.dump(rec, f)
    print(f"wrote {path} ({rec['seconds']} s)", flush=True)


if __name__ == "__main__":
    for kind in (sys.argv[1:] or ["grounded", "insulated"]):
        make(kind)
