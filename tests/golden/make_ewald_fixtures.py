"""Write the tin-foil Ewald potentials and forces of sampled charges of the
two 10^6-charge workloads (uniform-1M-n64, clustered-1M-n64) to
tests/golden/ewald_<workload>.json, for the method-error figures of the
benchmark and the GPU tests.  Calls only the oracle (oracle.ewald_sampled,
whose splitting is pinned against the paper's Ewald setting in
tests/test_oracle_ewald.py) on the seeded inputs of workloads.py.

    python tests/golden/make_ewald_fixtures.py [workload ...]

About 5 minutes per workload on 8 cores."""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import ewald, fep3m  # noqa: E402

NSAMPLE = 256


def targets_for(name, x, Q):
    """256 seeded charges; for the clustered workload half of them from the
    20 most populated elements of the 64^3 mesh."""
    rng = np.random.default_rng(7000 + len(name))
    if name.startswith("clustered"):
        _, e_lin, _ = fep3m.bin_particles(x, 1.0, 64)
        counts = np.bincount(e_lin, minlength=64**3)
        heavy = np.nonzero(np.isin(e_lin, np.argsort(counts)[-20:]))[0]
        t1 = rng.choice(heavy, NSAMPLE // 2, replace=False)
        rest = np.setdiff1d(np.arange(len(Q)), t1)
        return np.sort(np.concatenate([t1, rng.choice(rest, NSAMPLE - NSAMPLE // 2, replace=False)]))
    return np.sort(rng.choice(len(Q), NSAMPLE, replace=False))


def main(names):
    for name in names:
        x, Q = workloads.make(name)
        tg = targets_for(name, x, Q)
        t0 = time.time()
        ref = ewald.ewald_sampled(x, Q, tg, forces=True)
        out = {"workload": name, "reference": "tin-foil Ewald, oracle.ewald.ewald_sampled "
                                               "(alpha = 6/L, real space to r = L, |m_d| <= 12)",
               "targets": [int(t) for t in tg],
               "Phi": [float(v) for v in ref["Phi"]],
               "F": [[float(c) for c in row] for row in ref["F"]],
               "seconds": round(time.time() - t0, 1)}
        path = os.path.join(ROOT, "tests", "golden", f"ewald_{name}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=0)
        print(f"{name}: {len(tg)} targets, {out['seconds']} s -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["uniform-1M-n64", "clustered-1M-n64"])
