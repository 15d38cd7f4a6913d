#!/usr/bin/env python3
"""Throughput benchmark of the FR x conservative-DVM hot path on one MI355X.

A step is one explicit time step (three RK stages) over the whole phase space
of the workload; the metric counts DOF-updates per second, one DOF-update
being one of the N_e * N_s * N_u values advanced by one RK stage.

    python bench.py [--workload NAME] [--steps K] [--warmup W]

Prints one JSON line (see the keys below).  The roofline object describes
the fused FR stage kernel (HBM bound): algorithmic bytes per launch over its
average HIP-event duration on the library's stream.  The cpu_baseline object
times the FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def stage_bytes_per_dof(p: int, es: int, rk: int) -> float:
    """Algorithmic HBM bytes per DOF of one fused stage launch, averaged over
    the three stages of a step (the compulsory traffic of the fused design):
    read the stage value f, write the result, read the neighbours' outflow
    traces (3/(p+1) values per DOF) and write the own outflow traces of the
    result (3/(p+1)); SSP-RK3 also reads f^n in stages 2 and 3, the low-storage
    scheme reads dF in stages 2 and 3 and writes it in every stage."""
    n = p + 1
    tr = 3.0 / n
    if rk == 0:
        vals = 1 + 1 + 2 * tr + 2.0 / 3.0
    else:
        vals = 1 + 1 + 2 * tr + 1 + 2.0 / 3.0
    return vals * es


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="box16_p3_v16")
    ap.add_argument("--precision", type=int, default=None, help="0 FP64, 1 FP32 (default: the workload's)")
    ap.add_argument("--rk", type=int, default=None)
    ap.add_argument("--guess", type=int, default=None)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; multi-GPU sharding is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2312_06567_amd.frdvm import FrDvm

    w = W.workload(args.workload)
    prec = w["precision"] if args.precision is None else args.precision
    rk = w["rk"] if args.rk is None else args.rk
    steps = args.steps if args.steps is not None else 10
    mesh = W.box_mesh(w["N"])
    params = W.physics_params(w)
    params.update(precision=prec, rk=rk)
    if args.guess is not None:
        params["guess"] = args.guess
    print(f"[bench] workload {w['name']}: building handle", file=sys.stderr, flush=True)
    s = FrDvm(mesh, w["p"], w["grid"], params)
    ne, ns, nu = s.shape
    dof = ne * ns * nu
    dt = s.dt(0.2)
    prim = W.initial_prim(mesh, w["p"], w)
    print(f"[bench] generating f0 ({dof:.3e} DOFs) on the GPU", file=sys.stderr, flush=True)
    f = W.maxwellian(prim, w["grid"], dtype=s.dtype, device="cuda").reshape(ne, ns, nu)
    torch.cuda.synchronize()

    for i in range(args.warmup):
        s.rk_step(f, dt)
        torch.cuda.synchronize()
        print(f"[bench] warmup step {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    s.newton_stats(reset=True)
    s.profile(True)
    s.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        s.rk_step(f, dt)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = s.profile_read(reset=True)
    s.profile(False)
    stats = s.newton_stats(reset=True)
    print(f"[bench] {steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    updates = dof * 3 * steps
    value = updates / elapsed
    es = 8 if prec == 0 else 4
    ms_stage, n_stage = prof["stage"]
    avg_stage_s = ms_stage / 1e3 / max(n_stage, 1)
    bpd = stage_bytes_per_dof(w["p"], es, rk)
    achieved = bpd * dof / avg_stage_s / 1e9
    hist = stats["hist"]
    n_solves = int(hist.sum())
    mean_it = float((hist * np.arange(64)).sum() / max(n_solves, 1))

    out = {
        "metric": "DOF-updates/s (N_e*N_s*N_u per RK stage)",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32 (FP64 moments and Newton)",
        "data": "synthetic (seeded initial Maxwellian of the workload's macroscopic field)",
        "config": {"workload": w["name"], "n_elem": ne, "p": w["p"], "ns": ns, "nu": nu, "dof": dof,
                   "model": ["BGK", "ES-BGK", "free"][w["model"]], "rk": ["SSP-RK3", "LSRK3-2N"][rk],
                   "guess": params.get("guess", 0), "parallelism": "single GPU"},
        "kernels_ms_per_step": {k: v[0] / steps for k, v in prof.items()},
        "newton": {"mean_iters": mean_it, "fallback": stats["n_fallback"], "max_resid": stats["max_resid"]},
        "roofline": {"kernel": "k_fr_axis (fused FR stage)", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "algorithmic_bytes_per_dof": bpd,
                     "avg_launch_ms": avg_stage_s * 1e3},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, params, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline(w: dict, params: dict, budget_s: float) -> dict:
    """The FP64 CPU oracle (unchanged, OpenMP over elements) on a bounded
    sample of the workload: same order, velocity grid and physics on a smaller
    periodic box, one SSP-RK3 step, DOF-updates per second."""
    import numpy as np

    import oracle
    import workloads as W

    oracle.build(force=False)
    # sample size: elements chosen so one step takes roughly budget_s
    nsample = 2
    mesh = W.box_mesh(nsample)
    par = dict(params)
    par["model"] = w["model"]
    P = oracle.Problem(mesh, w["p"], w["grid"], par)
    prim = W.initial_prim(mesh, w["p"], dict(w))
    f0 = W.maxwellian(prim, w["grid"]).numpy()
    dt = P.dt(0.2)
    t0 = time.perf_counter()
    P.rk_step(f0, dt, scheme=0, nsteps=1)
    el = time.perf_counter() - t0
    dof = P.ne * P.ns * P.nu
    # grow the sample once if the first one was far below the budget
    if el < budget_s / 8:
        nsample = max(2, min(8, int(nsample * (budget_s / max(el, 1e-3)) ** (1 / 3))))
        mesh = W.box_mesh(nsample)
        P = oracle.Problem(mesh, w["p"], w["grid"], par)
        prim = W.initial_prim(mesh, w["p"], dict(w))
        f0 = W.maxwellian(prim, w["grid"]).numpy()
        t0 = time.perf_counter()
        P.rk_step(f0, P.dt(0.2), scheme=0, nsteps=1)
        el = time.perf_counter() - t0
        dof = P.ne * P.ns * P.nu
    return {"value": dof * 3 / el, "unit": "DOF-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one SSP-RK3 step on a {nsample}^3-element periodic box, p={w['p']}, "
                      f"{P.nu} velocities ({dof:.3e} DOFs), FP64, {el:.1f} s"}


if __name__ == "__main__":
    main()
