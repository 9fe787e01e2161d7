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
PEAK_FP64_TFLOPS = 78.6     # MI355X vector FP64 (256 CU x 2.4 GHz x 128 FLOP/clk); also dense FP64 MFMA
PEAK_MFMA_FP32_TFLOPS = 157.3   # MI355X dense FP32 MFMA
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E
OPERATOR_FLOP_PER_DOF = 98.0


# screen family -> (support, degree q); mesh order p = q + 2
SCREENS = {"one-q2": ("one", 2), "one-q3": ("one", 3), "one-q4": ("one", 4),
           "27-q1": ("27", 1), "27-q2": ("27", 2), "27-q3": ("27", 3), "27-q4": ("27", 4)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="uniform-1M-n64")
    ap.add_argument("--cpu-sample", type=int, default=4000, help="oracle target sample for the CPU baseline")
    ap.add_argument("--cpu-baseline-child", nargs=3, metavar=("WORKLOAD", "SAMPLE", "OUT"),
                    help=argparse.SUPPRESS)
    ap.add_argument("--no-sweep", action="store_true", help="skip the screen-family sweep at full size")
    ap.add_argument("--outputs", choices=["forces", "energy"], default="forces",
                    help="forces: U and F (the metric's energy+force step); energy: Phi and U")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="fp64: float64 throughout; mixed: float32 multigrid preconditioner, near field and "
                         "interpolation with compensated sums, float64 reductions")
    ap.add_argument("--near", choices=["auto", "direct", "fft"], default="auto",
                    help="near-screen field and its transpose: FFTs where the mesh allows (auto), table sums, or FFTs")
    ap.add_argument("--solver", choices=["mg", "exact"], default="mg",
                    help="mesh solve: multigrid PCG (the method's default) or the exact periodic solve")
    ap.add_argument("--boundary", choices=["periodic", "grounded", "insulated"], default="periodic",
                    help="the periodic cube, or the boxes of Section 2.6 (with --solver exact)")
    ap.add_argument("--screen", choices=sorted(SCREENS), default="one-q3",
                    help="screen family: the one-element screens of degree 2..4 or the 27-element screens of degree "
                         "1..4 (one-q3 is the method's default; the others skip the variants and the CPU baseline)")
    ap.add_argument("--n-sr", type=int, choices=[1, 2, 3], default=3, help="near block radius (block of 2 n_sr + 1 "
                    "elements per axis)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the mixed-precision, clustered and batched measurements reported beside the FP64 line")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain device copy of 256 MiB (FETCH_SIZE/WRITE_SIZE calibration) and exit")
    return ap.parse_args()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# state shared with the oracle's worker processes (forked after it is set)
_CPU = {}


def _cpu_chunk(tgt):
    """Per-charge stages of the oracle for one chunk of target charges."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import adjoint as oadj, fep3m as ofe

    g = _CPU
    P = g["P"]
    n, p, q, d, h = P.n, P.p, P.q, P.d, P.h
    with threadpool_limits(1):
        e, e_lin, u, Q = g["e"], g["e_lin"], g["u"], g["Q"]
        uel, inv = np.unique(e_lin[tgt], return_inverse=True)
        W = ofe.element_phi(g["phi"], p, n, uel) - ofe.near_field(g["C"], g["T"], n, P.n_sr, uel)
        A = oadj.moment_adjoint(g["lam"], g["gE"], g["T"], n, p, q, P.n_sr, uel)
        ut, Qt = u[tgt], Q[tgt]
        mesh_grad = 0.5 * Qt[:, None] * (np.einsum("nkm,nm->nk", oadj.basis_gradients(p, ut), W[inv])
                                         + np.einsum("nka,na->nk", oadj.monomial_gradients(ut, d), A[inv]))
        Phi_m = np.sum(W[inv] * ofe.basis_values(p, ut), axis=1)
        Phi_p = ofe.pair_potential(e, e_lin, u, Q, n, P.n_sr, tgt)
        dUp = oadj.pair_forces(e, e_lin, u, Q, n, P.n_sr, tgt)
        F_s = -(dUp + mesh_grad) / h**2
    return tgt, F_s, (Phi_p + Phi_m) / h


def cpu_baseline_child(workload, sample, out_path):
    """The FP64 oracle's energy + force evaluation on this host, in a process
    that never touches the GPU: the mesh-side stages in full (binning,
    moments, load, exact periodic solve; charge deposit, assembly, exact
    adjoint solve) with BLAS on every core, then the per-charge stages
    (near-screen field, moment adjoint, interpolation and its gradient, near
    pairs and pair forces) for `sample` seeded charges, in chunks over one
    worker process per core."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_info

    import workloads
    from oracle import adjoint as oadj, fep3m as ofe, mesh, screens, tables

    w = workloads.WORKLOADS[workload]
    x, Q = workloads.make(w)
    P = ofe.Params(L=w.L, n=w.n)
    n, p, q, d = P.n, P.p, P.q, P.d
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
    blas_threads = max([dd.get("num_threads", 1) for dd in threadpool_info()] + [1])
    rng = np.random.default_rng(0)
    tgt = np.sort(rng.choice(len(Q), min(sample, len(Q)), replace=False))
    nproc = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    _CPU.update(P=P, e=e, e_lin=e_lin, u=u, Q=Q, C=C, T=T, phi=phi, lam=lam, gE=gE)
    chunks = [c for c in np.array_split(tgt, 4 * nproc) if len(c)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(nproc) as pool:
        parts = pool.map(_cpu_chunk, chunks)
    t_tgt = time.perf_counter() - t0
    F_s = np.concatenate([pp[1] for pp in parts])
    counts = np.bincount(e_lin, minlength=n**3).reshape(n, n, n)
    block = np.zeros_like(counts)
    r = range(-P.n_sr, P.n_sr + 1)
    for dz in r:
        for dy in r:
            for dx in r:
                block += np.roll(counts, (dz, dy, dx), axis=(0, 1, 2))
    pairs = float(np.sum(counts * block) - len(Q))
    t_step = t_fixed + t_tgt * len(Q) / len(tgt)
    out = {"value": pairs / t_step, "unit": "pair interactions/s", "cores": int(nproc),
           "blas_threads": int(blas_threads), "worker_processes": int(nproc), "nproc": int(os.cpu_count() or 1),
           "cpu_model": _cpu_model(), "kind": "oracle",
           "sample": (f"energy+forces; mesh side in full ({t_fixed:.1f} s: binning, moments, load, exact periodic "
                      f"solve, charge deposit, assembly, exact adjoint solve; BLAS threads {blas_threads}), "
                      f"per-charge side for {len(tgt)} of {len(Q)} charges over {nproc} worker processes "
                      f"({t_tgt:.1f} s), scaled to all charges; tables precomputed once ({t_tables:.1f} s, "
                      f"excluded)"),
           "step_seconds_extrapolated": t_step, "targets": [int(t) for t in tgt],
           "F_sample": F_s.tolist()}
    with open(out_path, "w") as f:
        json.dump(out, f)


def cpu_baseline(workload, sample, F_gpu):
    """Run the oracle's timing in a child process (no GPU there) and compare
    the GPU forces with its sampled ones."""
    import subprocess
    import tempfile

    import numpy as np

    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "cpu.json")
        subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", workload, str(sample),
                        path], check=True)
        with open(path) as f:
            out = json.load(f)
    tgt = np.array(out.pop("targets"))
    F_s = np.array(out.pop("F_sample"))
    out["gpu_vs_oracle_force_rel_rms_on_sample"] = _rel_rms(F_gpu[tgt], F_s)
    return out


BATCH_WORKLOAD = "batch-64-n16"

# Kernel -> (profile summary holding its measured HBM traffic, sources whose
# hash the summary records).  The summary's figure is used only while those
# sources are unchanged; otherwise traffic is reported as null.
TRAFFIC_FILES = {
    "k_apply p=5 (fine-level operator)": ("k_apply_p5_fp64", ["paper_1503_08509_amd/csrc/k_mesh.hip",
                                                               "paper_1503_08509_amd/csrc/device_common.hpp"]),
    "k_adj_moments (transposed near field)": ("k_adj_moments_fp64", ["paper_1503_08509_amd/csrc/k_adjoint.hip",
                                                                     "paper_1503_08509_amd/csrc/device_common.hpp"]),
    "k_psi (near-screen field)": ("k_psi_fp64", ["paper_1503_08509_amd/csrc/k_near.hip",
                                                 "paper_1503_08509_amd/csrc/device_common.hpp"]),
    "k_fft_axis (near-field FFT pass, 108 channels)": ("k_fft_axis_108_fp64", ["paper_1503_08509_amd/csrc/k_fft.hip"]),
    "k_spec_orbit (spectrum products, both)": ("k_spec_orbit_fp64", ["paper_1503_08509_amd/csrc/k_fft.hip"]),
}


def source_hash(paths):
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload):
    """Calibrated HBM traffic per launch (GB) of `kernel` on `workload` from
    profiles/traffic_<tag>_<workload>.txt (FETCH_SIZE and WRITE_SIZE of
    rocprofv3 --pmc runs scaled by the same counters on a plain copy), or
    None when no such summary exists or its kernel sources have changed."""
    if kernel not in TRAFFIC_FILES:
        return None
    tag, srcs = TRAFFIC_FILES[kernel]
    path = os.path.join(ROOT, "profiles", f"traffic_{tag}_{workload}.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != source_hash(srcs):
        return None
    try:
        return float(fields["hbm_gb_per_launch"])
    except (KeyError, ValueError):
        return None


def load_workload(name):
    """(label, L, counts, n, x, Q): one configuration, or the batch of 64
    independent 16^3 configurations with N log-uniform in [2000, 64000]."""
    import numpy as np

    import workloads

    if name == BATCH_WORKLOAD:
        xs, Qs = workloads.batch()
        return name, 1.0, [len(q) for q in Qs], 16, np.concatenate(xs), np.concatenate(Qs)
    w = workloads.WORKLOADS[name]
    x, Q = workloads.make(w)
    return name, w.L, [w.N], w.n, x, Q


def stream_copy_gbs():
    """Practical HBM rate on this device: a 1 GiB device-to-device copy
    (reads and writes 1 GiB), best of 5, timed with events on the current
    stream."""
    import torch
    a = torch.ones(2**27, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    return 2 * 2**30 / (best * 1e-3) / 1e9


def kernel_rooflines(prof, steps, mixed, near_fft=False, p=5, moments=8, default_screen=True):
    def kern(slot, bound):
        s = prof[slot]
        if s["count"] == 0 or s["ms"] <= 0:
            return None
        sec = s["ms"] * 1e-3
        if bound == "hbm":
            ach = s["work"] / sec / 1e9
            return {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": ach / PEAK_HBM_GBS, "traffic": None,
                    "avg_launch_ms": s["ms"] / s["count"], "launches_per_step": s["count"] / steps}
        ach = s["work"] / sec / 1e12
        # vector ALU: FP64 and unpacked FP32 share the 78.6 TFLOP/s rate;
        # matrix cores: FP64 78.6, FP32 157.3 TFLOP/s
        peak = PEAK_MFMA_FP32_TFLOPS if (bound == "mfma" and mixed) else PEAK_FP64_TFLOPS
        return {"bound": bound, "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": None,
                "avg_launch_ms": s["ms"] / s["count"], "launches_per_step": s["count"] / steps}

    if near_fft:   # transforms and spectrum products: bytes in and out of each launch
        kernels = {"near-screen field (FFTs + spectrum product)": kern("near", "hbm"),
                   "k_pair (near-pair sum)": kern("pair", "alu"),
                   "k_apply p=5 (fine-level operator)": kern("fine_apply", "hbm"),
                   "transposed near field (FFTs + spectrum product)": kern("adj_near", "hbm")}
    elif default_screen:
        kernels = {"k_psi (near-screen field)": kern("near", "mfma"),
                   "k_pair (near-pair sum)": kern("pair", "alu"),
                   "k_apply p=5 (fine-level operator)": kern("fine_apply", "hbm"),
                   "k_adj_moments (transposed near field)": kern("adj_near", "alu")}
    else:   # the other screen families: near field on the matrix cores from 8 moments, adjoint from 27
        kernels = {f"near-screen field, {moments} moments": kern("near", "mfma" if moments >= 8 else "alu"),
                   "k_pair (near-pair sum)": kern("pair", "alu"),
                   f"k_apply p={p} (fine-level operator)": kern("fine_apply", "hbm"),
                   f"moment adjoint, {moments} moments": kern("adj_near", "mfma" if moments >= 27 else "alu")}
    if mixed:
        kernels[f"k_apply<float> p={p} (fine-level preconditioner operator)"] = kern("fine_apply_f32", "hbm")
    return {k: v for k, v in kernels.items() if v}


def measure(name, precision, steps, warmup, forces=True, graph=False, solver=0, near_field=0, **opts):
    """Run `warmup` + `steps` evaluations of one workload; device-resident
    inputs; returns timings, per-stage device times, kernel rooflines, the
    outputs of the last step (host copies) and the context statistics."""
    import numpy as np
    import torch

    import paper_1503_08509_amd as fp

    label, L, counts, n, x, Q = load_workload(name)
    mixed = precision == "mixed"
    dev = torch.device("cuda:0")
    tx = torch.from_numpy(x).to(dev)
    tQ = torch.from_numpy(Q).to(dev)
    q = opts.pop("q", 3)
    sup = opts.get("support", fp.SUPPORT_ONE)
    nsr = opts.get("n_sr", 3)
    moments = (q + 1 if sup == fp.SUPPORT_27 else q - 1) ** 3
    ctx = fp.Context(L, counts if len(counts) > 1 else counts[0], n, q=q,
                     precision=fp.PRECISION_MIXED if mixed else fp.PRECISION_FP64, use_graph=1 if graph else 0,
                     solver=solver, near_field=near_field, **opts)

    def step():
        if forces:
            return ctx.energy_forces(tx, tQ, Phi=True)
        Phi_, U_ = ctx.energy(tx, tQ)
        return {"U": U_, "Phi": Phi_}

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if not graph:   # graph replays are timed by wall clock only (no per-stage events)
        ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / steps
    st = ctx.stats()
    prof = ctx.profile()
    res = {
        "workload": label, "precision": precision, "counts": counts, "n": n, "L": L, "ms_per_step": ms,
        "pairs": st["near_pairs"], "value": st["near_pairs"] / (ms * 1e-3), "stats": st,
        "kernels": kernel_rooflines(prof, steps, mixed, bool(st["near_fft"]), p=q + 2, moments=moments,
                                    default_screen=(sup == fp.SUPPORT_ONE and q == 3)),
        "stages_ms_per_step": {k: v["ms"] / steps for k, v in prof.items() if not k.startswith("fine_apply")},
        "out": {k: v.detach().cpu().numpy() for k, v in out.items()},
        "x": x, "Q": Q, "mg_rtol": ctx.options.mg_rtol, "prof": prof, "steps": steps,
    }
    ctx.close()
    return res


def method_error_vs_ewald():
    """The method's own accuracy (not the GPU's parity): FP64 GPU result on
    uniform-1k-n8 (N = 1000, 8^3 elements, same screen and near block)
    against classic Ewald summation from the oracle (alpha = 2.5, 2 image
    shells, 4 Fourier modes per direction, the paper's comparison settings),
    Phi shifted by the screen constant c before comparing.  Ewald at N = 1e6
    is beyond a bounded CPU sample, so the headline workload's own error is
    not evaluated; it depends on the screen and near block, not on N."""
    import numpy as np
    import torch

    import paper_1503_08509_amd as fp
    import workloads
    from oracle import ewald, fep3m as ofe

    x, Q = workloads.make("uniform-1k-n8")
    ctx = fp.Context(1.0, len(Q), 8)
    out = ctx.energy_forces(torch.from_numpy(x).cuda(), torch.from_numpy(Q).cuda(), Phi=True)
    ref = ewald.ewald(x, Q, forces=True)
    P = ofe.Params(L=1.0, n=8)
    _, _, u = ofe.bin_particles(x, P.L, P.n)
    Phi = out["Phi"].cpu().numpy() + ofe.ewald_constant(u, Q, P)
    F = out["F"].cpu().numpy()
    # U needs no shift: the charges are neutral, so the constant drops out
    return {"workload": "uniform-1k-n8", "reference": "Ewald (oracle)",
            "Phi_rel_rms": _rel_rms(Phi, ref["Phi"]), "F_rel_rms": _rel_rms(F, ref["F"]),
            "U_rel": float(abs(float(out["U"]) - ref["U"]) / abs(ref["U"]))}


def _rel_rms(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# algorithmic bytes per launch of these kernels are recorded by the library
# (fep3m.h, profile slots MOMENTS, LOAD, DEPOSIT, INTERP_KERNEL)
HBM_STAGES = {"moments": "k_moments (charge projection: element moments)",
              "load": "k_load (load-vector assembly)",
              "deposit": "k_deposit + k_assemble (charge deposit on the order-p basis)",
              "interp_kernel": "k_interp (mesh-to-charge interpolation)"}


def hbm_stage_rooflines(name="uniform-1M-n64", precision="fp64", steps=3):
    """HBM rate of the projection, load, deposit and interpolation kernels,
    measured with every launch on one stream (no pair sum running beside
    them): algorithmic bytes per launch / launch time (hipEvents)."""
    r = measure(name, precision, steps, 1, pair_stream=0)
    out = {}
    for slot, label in HBM_STAGES.items():
        s = r["prof"][slot]
        if s["count"] == 0 or s["ms"] <= 0:
            continue
        ach = s["work"] / (s["ms"] * 1e-3) / 1e9
        out[label] = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                      "frac": ach / PEAK_HBM_GBS, "avg_launch_ms": s["ms"] / s["count"],
                      "algorithmic_gb_per_launch": s["work"] / s["count"] / 1e9}
    return {"workload": name, "precision": precision, "pair_stream": 0, "kernels": out,
            "ms_per_step_single_stream": r["ms_per_step"]}


def ewald_fixture(name):
    path = os.path.join(ROOT, "tests", "golden", f"ewald_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def ewald_error_full_size(r, support="one", q=3, n_sr=3):
    """Method error of a full-size run against the committed Ewald reference
    of its workload's sampled charges (tests/golden/ewald_<workload>.json,
    written by the oracle): Phi shifted by the gauge constant c of the screen
    (zero once the x^2 moments are cancelled), F unshifted."""
    import numpy as np

    from oracle import fep3m as ofe

    fx = ewald_fixture(r["workload"])
    if fx is None:
        return None
    tg = np.array(fx["targets"])
    P = ofe.Params(L=r["L"], n=r["n"], q=q, support=support, n_sr=n_sr)
    _, _, u = ofe.bin_particles(r["x"], P.L, P.n)
    c = ofe.ewald_constant(u, r["Q"], P)
    Phi = r["out"]["Phi"][tg] + c
    F = r["out"]["F"][tg]
    return {"reference": fx["reference"], "sampled_charges": len(tg),
            "Phi_rel_rms": _rel_rms(Phi, np.array(fx["Phi"])), "F_rel_rms": _rel_rms(F, np.array(fx["F"])),
            "gauge_constant": c}


SCREEN_SWEEP = [("one", 3, 3), ("one", 4, 3), ("27", 1, 3), ("27", 2, 3), ("27", 3, 2), ("27", 3, 3), ("27", 4, 3)]


def screen_sweep(name="uniform-1M-n64"):
    """Time per energy+force step and method error against Ewald at full
    size for the screen families and near-block radii (the headline screen
    first)."""
    import paper_1503_08509_amd as fp

    rows = []
    for support, q, nsr in SCREEN_SWEEP:
        r = measure(name, "fp64", 2, 1, q=q, support=fp.SUPPORT_27 if support == "27" else fp.SUPPORT_ONE,
                    n_sr=nsr, table_box=2 * nsr + 9)
        err = ewald_error_full_size(r, support, q, nsr)
        rows.append({"screen": f"{'27-element' if support == '27' else 'one-element'} q={q}",
                     "near_block": f"{2 * nsr + 1}^3", "mesh_order": q + 2, "ms_per_step": r["ms_per_step"],
                     "pair_interactions_per_s": r["value"], "mg_iterations": r["stats"]["mg_iterations"],
                     "ewald": err})
        print(f"# sweep {rows[-1]['screen']} {rows[-1]['near_block']}: {r['ms_per_step']:.1f} ms, "
              f"Phi {err['Phi_rel_rms'] if err else float('nan'):.2e}", file=sys.stderr, flush=True)
        del r
    return {"workload": name, "rows": rows}


def variant_summary(r, ref=None):
    import numpy as np
    k = r["kernels"]
    v = {"ms_per_step": r["ms_per_step"], "value": r["value"], "unit": "pair interactions/s",
         "near_pairs_per_step": r["pairs"], "configurations": len(r["counts"]),
         "N": int(sum(r["counts"])), "elements": f"{r['n']}^3",
         "graph_replays": r["stats"]["graph_replays"],
         "mg_iterations": r["stats"]["mg_iterations"], "adj_mg_iterations": r["stats"]["adj_iterations"],
         "create_seconds": r["stats"]["create_seconds"],
         "stages_ms_per_step": {s: round(t, 4) for s, t in r["stages_ms_per_step"].items()},
         "pair_variant": {"kind": {0: "element", 1: "queue", 2: "rows"}[r["stats"]["pair_variant"]],
                          "item_targets": r["stats"]["pair_item_targets"], "waves": r["stats"]["pair_waves"],
                          "tuned_ms": r["stats"]["tune_ms_best"], "element_ms": r["stats"]["tune_ms_default"]}}
    if k:
        dom = max(k, key=lambda s: k[s]["avg_launch_ms"] * k[s]["launches_per_step"])
        v.update({"pair_kernel_ms": r["stages_ms_per_step"]["pair"],
                  "pair_interactions_per_s_pair_kernel": r["pairs"] / (r["stages_ms_per_step"]["pair"] * 1e-3),
                  "dominant_kernel": dom, "dominant_frac": k[dom]["frac"], "dominant_bound": k[dom]["bound"],
                  "kernel_fracs": {s: round(k[s]["frac"], 4) for s in k}})
    if ref is not None:
        v["accuracy_vs_fp64"] = {
            "Phi_rel_rms": _rel_rms(r["out"]["Phi"], ref["out"]["Phi"]),
            "F_rel_rms": _rel_rms(r["out"]["F"], ref["out"]["F"]),
            "U_rel": float(np.abs(r["out"]["U"] - ref["out"]["U"]).max() / np.abs(ref["out"]["U"]).max()),
        }
    return v


def main():
    args = parse()
    if args.cpu_baseline_child:   # the oracle's timing, in a process of its own (never touches the GPU)
        wl, sample, path = args.cpu_baseline_child
        cpu_baseline_child(wl, int(sample), path)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (one process, no collectives); --gpus must be 1"}))
        sys.exit(2)
    import numpy as np  # noqa: F401
    import torch

    if args.copy_calibration:
        a = torch.empty(2**25, dtype=torch.float64, device="cuda:0").fill_(1.0)
        torch.cuda.synchronize()
        c = a.clone()          # one copy kernel: reads and writes 2^25 doubles = 256 MiB each way
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": 2**25 * 8, "check": float(c[0].item())}))
        return

    forces = args.outputs == "forces"
    bc = {"periodic": 0, "grounded": 1, "insulated": 2}[args.boundary]
    if bc and args.solver != "exact":
        print(json.dumps({"error": "the boxes of Section 2.6 need --solver exact"}))
        sys.exit(2)
    support, q = SCREENS[args.screen]
    default_screen = args.screen == "one-q3" and args.n_sr == 3
    screen_opts = {} if default_screen else {"q": q, "support": 1 if support == "27" else 0, "n_sr": args.n_sr,
                                             "table_box": 2 * args.n_sr + 9}
    r = measure(args.workload, args.precision, args.steps, args.warmup, forces,
                solver={"mg": 0, "exact": 1}[args.solver], near_field={"auto": 0, "direct": 1, "fft": 2}[args.near],
                boundary=bc, **screen_opts)
    mixed = args.precision == "mixed"
    kernels = r["kernels"]
    practical = stream_copy_gbs() if not args.no_variants else None   # kept out of profiled runs
    for k, v in kernels.items():
        if v["bound"] == "hbm" and practical:
            v["practical_peak"] = practical
            v["frac_practical"] = v["achieved"] / practical
    op = kernels.get(f"k_apply p={q + 2} (fine-level operator)")
    if op:
        # the operator's own arithmetic: sum-factorised Kronecker-sum apply,
        # 7 one-dimensional band passes of 7 multiply-adds per node on average
        # (6 taps inside an element, 11 at a vertex) = 98 FLOP per DOF
        # with forces every fine-level launch covers the forward and the adjoint system
        dofs = ((q + 2) * r["n"]) ** 3 * len(r["counts"]) * (2 if forces else 1)
        tf = OPERATOR_FLOP_PER_DOF * dofs / (op["avg_launch_ms"] * 1e-3) / 1e12
        op["flop_achieved"] = tf
        op["flop_peak"] = PEAK_FP64_TFLOPS   # the PCG operator is float64 in both precisions
        op["flop_frac"] = tf / op["flop_peak"]
        op["flop_unit"] = "TFLOP/s (98 FLOP per DOF)"
    if not mixed:   # counter-measured HBM bytes per launch where a current summary exists
        for k in kernels:
            kernels[k]["traffic"] = traffic_for(k, r["workload"])
    dominant = max(kernels, key=lambda k: kernels[k]["avg_launch_ms"] * kernels[k]["launches_per_step"])
    roof = dict(kernels[dominant])
    roof["kernel"] = dominant
    roof["traffic"] = traffic_for(dominant, r["workload"]) if not mixed else None
    roof["traffic_unit"] = "GB per launch (calibrated FETCH_SIZE + WRITE_SIZE)"
    if roof["bound"] == "hbm":
        roof["algorithmic_gb_per_launch"] = roof["achieved"] * roof["avg_launch_ms"] * 1e-3
    st = r["stats"]
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "pair interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": r["workload"], "N": int(sum(r["counts"])), "configurations": len(r["counts"]),
                   "elements": f"{r['n']}^3", "L": r["L"],
                   "screen": f"{'27-element' if support == '27' else 'one-element'} q={q}", "mesh_order": q + 2,
                   "near_block": f"{2 * args.n_sr + 1}^3", "outputs": "U, F" if forces else "Phi, U", "precision": args.precision,
                   "mg_rtol": r["mg_rtol"], "solver": "multigrid PCG" if args.solver == "mg" else "exact",
                   "boundary": args.boundary,
                   "near_pairs_per_step": r["pairs"]},
        "roofline": roof,
        "kernels": kernels,
        "stages_ms_per_step": r["stages_ms_per_step"],
        "mg_iterations": st["mg_iterations"],
        "adj_mg_iterations": st["adj_iterations"] if forces else None,
        "mg_rel_residual": st["mg_rel_residual"],
        "create_seconds": st["create_seconds"],
        "practical_hbm_gbs": practical,
        "pair_variant": variant_summary(r)["pair_variant"],
        "U": [float(u) for u in np.atleast_1d(r["out"]["U"])][:4],
    }
    if not args.no_variants and forces and args.workload == "uniform-1M-n64" and not mixed and not bc \
            and default_screen:
        variants = {}
        m = measure("uniform-1M-n64", "mixed", 3, 1)
        variants["mixed uniform-1M-n64"] = variant_summary(m, r)
        del m
        c64 = measure("clustered-1M-n64", "fp64", 3, 1)
        variants["fp64 clustered-1M-n64"] = variant_summary(c64)
        variants["fp64 clustered-1M-n64"]["method_error_vs_ewald"] = ewald_error_full_size(c64)
        cm = measure("clustered-1M-n64", "mixed", 3, 1)
        variants["mixed clustered-1M-n64"] = variant_summary(cm, c64)
        del c64, cm
        b64 = measure(BATCH_WORKLOAD, "fp64", 3, 1)
        variants["fp64 " + BATCH_WORKLOAD] = variant_summary(b64)
        bm = measure(BATCH_WORKLOAD, "mixed", 3, 1)
        variants["mixed " + BATCH_WORKLOAD] = variant_summary(bm, b64)
        bg = measure(BATCH_WORKLOAD, "fp64", 3, 2, graph=True)
        variants["fp64 " + BATCH_WORKLOAD + " hipGraph"] = variant_summary(bg, b64)
        bmg = measure(BATCH_WORKLOAD, "mixed", 3, 2, graph=True)
        variants["mixed " + BATCH_WORKLOAD + " hipGraph"] = variant_summary(bmg, b64)
        del b64, bm, bg, bmg
        ug = measure("uniform-1M-n64", "fp64", 3, 2, graph=True)
        variants["fp64 uniform-1M-n64 hipGraph"] = variant_summary(ug, r)
        del ug
        # the near field and its transpose as direct table sums instead of FFTs
        for prec in ("fp64", "mixed"):
            dn = measure("uniform-1M-n64", prec, 3, 1, near_field=1)
            variants[f"{prec} uniform-1M-n64 direct near field"] = variant_summary(dn, r)
            del dn
        # the smaller configurations: 1000 charges on 8^3, 1e5 on 32^3 (FP64 and mixed side by side)
        for wl in ("uniform-1k-n8", "uniform-100k-n32"):
            s64 = measure(wl, "fp64", 5, 2)
            variants["fp64 " + wl] = variant_summary(s64)
            sm = measure(wl, "mixed", 5, 2)
            variants["mixed " + wl] = variant_summary(sm, s64)
            sg = measure(wl, "fp64", 5, 2, graph=True)   # small problems: launches and host reads dominate
            variants["fp64 " + wl + " hipGraph"] = variant_summary(sg, s64)
            del s64, sm, sg
        # the exact periodic mesh solve (Fourier analysis over the element lattice) in place of multigrid
        for prec, wl in (("fp64", "uniform-1M-n64"), ("mixed", "uniform-1M-n64"), ("fp64", BATCH_WORKLOAD)):
            fd = measure(wl, prec, 3, 1, solver=1)
            variants[f"{prec} {wl} exact mesh solver"] = variant_summary(
                fd, r if wl == "uniform-1M-n64" else None)
            del fd
        # the boxes of Section 2.6 (exact solve of the box pencil): grounded with forces, insulated
        gb = measure("uniform-1M-n64", "fp64", 3, 1, solver=1, boundary=1)
        variants["fp64 uniform-1M-n64 grounded box (energy + forces)"] = variant_summary(gb)
        del gb
        ib = measure("uniform-1M-n64", "fp64", 3, 1, solver=1, boundary=2)
        variants["fp64 uniform-1M-n64 insulated box (energy + forces)"] = variant_summary(ib)
        del ib
        out["variants"] = variants
        out["hbm_stages"] = hbm_stage_rooflines()
        if not args.no_sweep:
            out["screen_sweep"] = screen_sweep()
    if not default_screen and args.boundary == "periodic" and forces and not mixed \
            and args.workload in ("uniform-1M-n64", "clustered-1M-n64"):
        out["method_error_vs_ewald_full_size"] = ewald_error_full_size(r, support, q, args.n_sr)
    if not args.no_cpu_baseline and args.boundary == "periodic" and default_screen:
        out["method_error_vs_ewald"] = method_error_vs_ewald()
        if args.workload in ("uniform-1M-n64", "clustered-1M-n64") and forces and not mixed:
            out["method_error_vs_ewald_full_size"] = ewald_error_full_size(r)
        if forces and len(r["counts"]) == 1:
            import workloads
            out["cpu_baseline"] = cpu_baseline(r["workload"], args.cpu_sample, r["out"]["F"])
        else:
            out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
