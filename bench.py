#!/usr/bin/env python3
"""Benchmark of the FE-P3M hot path on one MI355X.

One step = one full energy + force evaluation through the C ABI (bin and
sort, moments, load, multigrid-PCG mesh solve, near-screen field, near-pair
sum with pair forces, interpolation, energy; then the reverse pass: charge
deposit, second mesh solve, transposed near-screen correlation, forces) on
device-resident synthetic inputs.  Prints one JSON line: pair
interactions/s of the whole step, the step time (the N = 1e6 energy+force
time on the default workload), the
roofline position of the dominant kernel (device time from hipEvents the
library records on its stream), and the FP64 oracle's throughput on a
bounded sample of the same workload, timed on this host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair interactions/s + N=1M energy+force time at 1e-6 rel. RMS err vs Ewald"
PEAK_FP64_TFLOPS = 78.6     # MI355X vector FP64 (256 CU x 2.4 GHz x 128 FLOP/clk)
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="uniform-1M-n64")
    ap.add_argument("--cpu-sample", type=int, default=1000, help="oracle target sample for the CPU baseline")
    ap.add_argument("--outputs", choices=["forces", "energy"], default="forces",
                    help="forces: U and F (the metric's energy+force step); energy: Phi and U")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="fp64: float64 throughout; mixed: float32 multigrid preconditioner, near field and "
                         "interpolation with compensated sums, float64 reductions")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain device copy of 256 MiB (FETCH_SIZE/WRITE_SIZE calibration) and exit")
    return ap.parse_args()


def cpu_baseline(x, Q, w, sample, F_gpu):
    """The FP64 oracle's energy + force evaluation, stage by stage in the
    order the oracle computes it, on this host: every mesh-side stage in full
    (binning, moments, load, exact periodic solve; charge deposit, assembly,
    exact adjoint solve), the per-charge stages (near-screen field, moment
    adjoint, interpolation and its gradient, near pairs and pair forces) for
    `sample` charges, scaled to all N."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import adjoint as oadj, fep3m as ofe, mesh, screens, tables

    P = ofe.Params(L=w.L, n=w.n)
    n, p, q, d, h = P.n, P.p, P.q, P.d, P.h
    t0 = time.perf_counter()
    T = tables.screen_tables(p, q, P.n_sr, P.B, P.table_bc)
    t_tables = time.perf_counter() - t0
    t0 = time.perf_counter()
    e, e_lin, u = ofe.bin_particles(x, P.L, n)
    C = screens.element_moments(e_lin, u, Q, n**3, d)
    b = mesh.project_compatible(mesh.load_vector(C, n, p, q), p, n)
    phi = mesh.solve_periodic(b, p, n)
    phi = phi - mesh.mean_value(phi, p, n)
    gE = oadj.element_deposit(e_lin, u, Q, n, p)
    G = mesh.project_compatible(oadj.assemble(gE, n, p), p, n)
    lam = mesh.solve_periodic(G, p, n)
    lam = lam - mesh.mean_value(lam, p, n)
    t_fixed = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    tgt = np.sort(rng.choice(len(Q), min(sample, len(Q)), replace=False))
    t0 = time.perf_counter()
    uel, inv = np.unique(e_lin[tgt], return_inverse=True)
    W = ofe.element_phi(phi, p, n, uel) - ofe.near_field(C, T, n, P.n_sr, uel)
    A = oadj.moment_adjoint(lam, gE, T, n, p, q, P.n_sr, uel)
    ut, Qt = u[tgt], Q[tgt]
    mesh_grad = 0.5 * Qt[:, None] * (np.einsum("nkm,nm->nk", oadj.basis_gradients(p, ut), W[inv])
                                     + np.einsum("nka,na->nk", oadj.monomial_gradients(ut, d), A[inv]))
    Phi_m = np.sum(W[inv] * ofe.basis_values(p, ut), axis=1)
    Phi_p = ofe.pair_potential(e, e_lin, u, Q, n, P.n_sr, tgt)
    dUp = oadj.pair_forces(e, e_lin, u, Q, n, P.n_sr, tgt)
    F_s = -(dUp + mesh_grad) / h**2
    t_tgt = time.perf_counter() - t0
    t_step = t_fixed + t_tgt * len(Q) / len(tgt)
    counts = np.bincount(e_lin, minlength=n**3).reshape(n, n, n)
    block = np.zeros_like(counts)
    r = range(-P.n_sr, P.n_sr + 1)
    for dz in r:
        for dy in r:
            for dx in r:
                block += np.roll(counts, (dz, dy, dx), axis=(0, 1, 2))
    pairs = float(np.sum(counts * block) - len(Q))
    threads = max([dd.get("num_threads", 1) for dd in threadpool_info()] + [1])
    err = float(np.linalg.norm(F_gpu[tgt] - F_s) / np.linalg.norm(F_s))
    del Phi_m, Phi_p
    return {
        "value": pairs / t_step,
        "unit": "pair interactions/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"energy+forces; mesh side in full ({t_fixed:.1f} s: binning, moments, load, exact periodic "
                   f"solve, charge deposit, assembly, exact adjoint solve), per-charge side for {len(tgt)} of "
                   f"{len(Q)} charges ({t_tgt:.1f} s), scaled to all charges; tables precomputed once "
                   f"({t_tables:.1f} s, excluded); BLAS threads={threads}, per-charge loops single-threaded"),
        "step_seconds_extrapolated": t_step,
        "gpu_vs_oracle_force_rel_rms_on_sample": err,
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_calibration:
        a = torch.empty(2**25, dtype=torch.float64, device="cuda:0").fill_(1.0)
        torch.cuda.synchronize()
        c = a.clone()          # one copy kernel: reads and writes 2^25 doubles = 256 MiB each way
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": 2**25 * 8, "check": float(c[0].item())}))
        return

    import paper_1503_08509_amd as fp
    import workloads

    w = workloads.WORKLOADS[args.workload]
    x, Q = workloads.make(w)
    dev = torch.device("cuda:0")
    tx = torch.from_numpy(x).to(dev)
    tQ = torch.from_numpy(Q).to(dev)
    mixed = args.precision == "mixed"
    ctx = fp.Context(w.L, w.N, w.n, precision=fp.PRECISION_MIXED if mixed else fp.PRECISION_FP64)
    forces = args.outputs == "forces"

    def step():
        if forces:
            o = ctx.energy_forces(tx, tQ)
            return o["U"], o["F"]
        Phi_, U_ = ctx.energy(tx, tQ)
        return U_, None

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        U, F = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    st = ctx.stats()
    prof = ctx.profile()
    pairs = st["near_pairs"]

    def kern(slot, bound):
        s = prof[slot]
        if s["count"] == 0 or s["ms"] <= 0:
            return None
        sec = s["ms"] * 1e-3
        if bound == "hbm":
            ach = s["work"] / sec / 1e9
            return {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": ach / PEAK_HBM_GBS, "traffic": None,
                    "avg_launch_ms": s["ms"] / s["count"], "launches_per_step": s["count"] / args.steps}
        ach = s["work"] / sec / 1e12
        return {"bound": "alu", "achieved": ach, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_FP64_TFLOPS, "traffic": None,
                "avg_launch_ms": s["ms"] / s["count"], "launches_per_step": s["count"] / args.steps}

    kernels = {"k_psi (near-screen field)": kern("near", "alu"),
               "k_pair (near-pair sum)": kern("pair", "alu"),
               "k_apply p=5 (fine-level operator)": kern("fine_apply", "hbm")}
    if mixed:
        kernels["k_apply<float> p=5 (fine-level preconditioner operator)"] = kern("fine_apply_f32", "hbm")
    if forces:
        kernels["k_adj_moments (transposed near field)"] = kern("adj_near", "alu")
    dominant = max(kernels, key=lambda k: (kernels[k]["avg_launch_ms"] * kernels[k]["launches_per_step"])
                   if kernels[k] else -1)
    roof = dict(kernels[dominant])
    roof["kernel"] = dominant
    out = {
        "metric": METRIC,
        "value": pairs / (ms * 1e-3),
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "N": w.N, "elements": f"{w.n}^3", "L": w.L, "screen": "one-element q=3",
                   "mesh_order": 5, "near_block": "7^3", "outputs": "U, F" if forces else "Phi, U",
                   "precision": args.precision, "mg_rtol": ctx.options.mg_rtol, "near_pairs_per_step": pairs},
        "roofline": roof,
        "kernels": kernels,
        "stages_ms_per_step": {k: v["ms"] / args.steps for k, v in prof.items()
                               if not k.startswith("fine_apply")},
        "mg_iterations": st["mg_iterations"],
        "adj_mg_iterations": st["adj_iterations"] if forces else None,
        "mg_rel_residual": st["mg_rel_residual"],
        "U": float(U.item()),
    }
    if not args.no_cpu_baseline:
        if forces:
            out["cpu_baseline"] = cpu_baseline(x, Q, w, args.cpu_sample, F.cpu().numpy())
        else:
            out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
