#!/usr/bin/env python3
"""Throughput benchmark of the FR x conservative-DVM hot path on one MI355X.

A step is one explicit time step (three RK stages) over the whole phase space
of the workload; the metric counts DOF-updates per second, one DOF-update
being one of the N_e * N_s * N_u values advanced by one RK stage.

Default (``--mode compare``, workload box24_p3_v20_es: 24^3 periodic hexes,
p = 3, 20^3 velocities on [-8, 8]^3, ES-BGK Pr 0.71, Kn 2e-4, Taylor-Green
U0 = 0.5 with a 1 % seeded perturbation):
  * plain FP64: FP64 storage and arithmetic, SSP-RK3, cold-start Newton;
  * mixed + learned: FP32 storage and FR/RK arithmetic with FP64 moments and
    Newton, low-storage RK, Newton started from the learned guess (MLP trained
    first, untimed, on states of this grid including the solver's own initial
    states) and warm afterwards;
  both timed over the same K steps from the same initial state.  ``value`` is
  the mixed + learned throughput.  Equal error: the relative L2 difference of
  the conserved moments between the two runs is compared with the FP64 run's
  own time-discretisation error, estimated by a dt / 2 FP64 run.
``--mode single`` times one configuration (flags choose precision, RK scheme,
guess, model) and is what the profiler runs.

Prints one JSON line.  ``roofline`` describes the fused FR stage kernel of the
reported configuration (HBM bound): algorithmic bytes per launch over its
average HIP-event duration on the library's stream.  ``cpu_baseline`` times
the FP64 CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stage_bytes_per_dof(p: int, es: int, rk: int) -> float:
    """Algorithmic HBM bytes per DOF of one fused stage launch, averaged over
    the three stages of a step (the compulsory traffic of the fused design):
    read the stage value f, write the result, read the neighbours' outflow
    traces (3/(p+1) values per DOF) and write the own outflow traces of the
    result (3/(p+1)); SSP-RK3 also reads f^n in stages 2 and 3, the low-storage
    scheme reads dF in stages 2 and 3 and writes it in every stage."""
    tr = 3.0 / (p + 1)
    vals = 1 + 1 + 2 * tr + 2.0 / 3.0 + (1.0 if rk == 1 else 0.0)
    return vals * es


def run_config(W, w, mesh, params, steps, warmup, label, weights=None, keep_moments=False, dt_scale=1.0,
               nsteps_override=None):
    """Build a handle, generate f0 on the GPU, warm up, time `steps` steps.
    Returns a dict with timing, kernel times and (optionally) final moments."""
    import numpy as np
    import torch

    from paper_2312_06567_amd.frdvm import FrDvm
    s = FrDvm(mesh, w["p"], w["grid"], params)
    if weights is not None:
        s.mlp_set_weights(weights)
    ne, ns, nu = s.shape
    dof = ne * ns * nu
    dt = s.dt(0.2) * dt_scale
    prim = W.initial_prim(mesh, w["p"], w)
    log(f"{label}: generating f0 ({dof:.3e} DOFs, {s.dtype})")
    f = W.maxwellian(prim, w["grid"], dtype=s.dtype, device="cuda").reshape(ne, ns, nu)
    torch.cuda.synchronize()
    for i in range(warmup):
        s.rk_step(f, dt)
        torch.cuda.synchronize()
        log(f"{label}: warmup step {i + 1}/{warmup} done")
    n_timed = nsteps_override if nsteps_override is not None else steps
    s.newton_stats(reset=True)
    s.profile(True)
    s.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_timed):
        s.rk_step(f, dt)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = s.profile_read(reset=True)
    s.profile(False)
    stats = s.newton_stats(reset=True)
    log(f"{label}: {n_timed} steps in {elapsed:.3f} s")
    out = {"label": label, "dof": dof, "steps": n_timed, "elapsed": elapsed, "dt": dt,
           "value": dof * 3 * n_timed / elapsed, "ms_per_step": elapsed / n_timed * 1e3, "prof": prof,
           "stats": stats, "precision": params.get("precision", 0), "rk": params.get("rk", 0)}
    hist = stats["hist"]
    nsol = max(int(hist.sum()), 1)
    out["newton"] = {"mean_iters": float((hist * np.arange(64)).sum() / nsol),
                     "mean_evals": float(stats["n_evals"] / nsol),
                     "fallback": int(stats["n_fallback"]), "es_guard": int(stats["n_guard"]),
                     "max_resid": float(stats["max_resid"])}
    if keep_moments:
        Q = torch.empty(ne * ns * 5, dtype=torch.float64, device="cuda")
        tot = s.moments(f, Q, totals=True)
        out["Q"] = Q.cpu().numpy().reshape(-1, 5)
        out["totals"] = tot
    out["totals_finite"] = bool(torch.isfinite(f).all().item())
    del f
    s.destroy()
    torch.cuda.empty_cache()
    return out


def roofline(r, p):
    es = 8 if r["precision"] == 0 else 4
    ms, n = r["prof"]["stage"]
    avg_s = ms / 1e3 / max(n, 1)
    bpd = stage_bytes_per_dof(p, es, r["rk"])
    ach = bpd * r["dof"] / avg_s / 1e9
    return {"kernel": "k_fr_layer (fused FR stage)", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None, "algorithmic_bytes_per_dof": bpd,
            "avg_launch_ms": avg_s * 1e3}


def rel_moments(Qa, Qb):
    import numpy as np
    out = {}
    for name, sl in (("rho", slice(0, 1)), ("rhoU", slice(1, 4)), ("E", slice(4, 5))):
        out[name] = float(np.linalg.norm(Qa[:, sl] - Qb[:, sl]) / np.linalg.norm(Qb[:, sl]))
    return out


def train_guess(W, w, log_fn):
    """Learned Newton start for this workload's grid: states sampled over the
    grid's attainable range plus the solver's own initial states, targets from
    the library's FP64 Newton, training by the library's MLP kernels."""
    import numpy as np
    import torch

    from paper_2312_06567_amd import learned
    umax = float(w["grid"]["umax"][0])
    nv = int(w["grid"]["n"][0])
    mesh = W.box_mesh(w["N"])
    prim = W.initial_prim(mesh, w["p"], w).reshape(-1, 5)
    rng = np.random.default_rng(7)
    pick = rng.choice(prim.shape[0], min(20000, prim.shape[0]), replace=False)
    extra = {"rho": prim[pick, 0], "U": prim[pick, 1:4], "theta": prim[pick, 4],
             "umax": np.full(len(pick), umax)}
    t0 = time.perf_counter()
    wts, info = learned.fit_guess(n_states=20000, nv=nv, steps=3000, seed=4, umax_choices=(umax,), extra=extra)
    torch.cuda.synchronize()
    info["train_seconds"] = time.perf_counter() - t0
    log_fn(f"learned guess trained in {info['train_seconds']:.1f} s on {info['n_converged']} states")
    return wts, info


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="box24_p3_v20_es")
    ap.add_argument("--mode", choices=("compare", "single"), default="compare")
    ap.add_argument("--precision", type=int, default=None, help="single mode: 0 FP64, 1 FP32")
    ap.add_argument("--rk", type=int, default=None, help="single mode: 0 SSP-RK3, 1 low-storage")
    ap.add_argument("--guess", type=int, default=None, help="single mode: 0 cold, 1 warm, 2 MLP, 3 MLP then warm")
    ap.add_argument("--model", type=int, default=None, help="0 BGK, 1 ES-BGK, 2 collisionless")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-error", action="store_true", help="compare mode: skip the dt/2 error estimate")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="instead of the benchmark, copy this many GiB with the library's plain copy kernel "
                         "(calibration of the HBM byte counters) and print its bandwidth")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; multi-GPU sharding is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import workloads as W
    from paper_2312_06567_amd import frdvm

    if args.copy_probe > 0:
        nbytes = int(args.copy_probe * 2 ** 30) // 16 * 16
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        frdvm.hbm_copy(b, a, nbytes)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            frdvm.hbm_copy(b, a, nbytes)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        print(json.dumps({"copy_probe_bytes": nbytes, "read_plus_write_GBps": 2 * nbytes / el / 1e9,
                          "ms": el * 1e3, "launches": reps + 1}))
        return

    w = W.workload(args.workload)
    mesh = W.box_mesh(w["N"])
    base = W.physics_params(w)
    if args.model is not None:
        base["model"] = args.model
    cfg = {"workload": w["name"], "n_elem": int(mesh["n_elem"]), "p": w["p"], "ns": (w["p"] + 1) ** 3,
           "nu": int(w["grid"]["n"][0] * w["grid"]["n"][1] * w["grid"]["n"][2]),
           "model": ["BGK", "ES-BGK", "free"][base["model"]], "prandtl": base["prandtl"], "kn": w["kn"],
           "parallelism": "single GPU"}

    if args.mode == "single":
        par = dict(base)
        par["precision"] = w["precision"] if args.precision is None else args.precision
        par["rk"] = w["rk"] if args.rk is None else args.rk
        par["guess"] = 0 if args.guess is None else args.guess
        weights = None
        if par["guess"] in (2, 3):
            weights, _ = train_guess(W, w, log)
        r = run_config(W, w, mesh, par, args.steps, args.warmup, "single", weights=weights)
        cfg.update(precision=["FP64", "FP32"][par["precision"]], rk=["SSP-RK3", "LSRK3-2N"][par["rk"]],
                   guess=["cold", "warm", "learned", "learned+warm"][par["guess"]])
        out = {"metric": "DOF-updates/s (N_e*N_s*N_u per RK stage)", "value": r["value"], "unit": "DOF-updates/s",
               "n_gpus": 1, "steps": r["steps"], "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64" if par["precision"] == 0 else "f32 (FP64 moments and Newton)",
               "data": "synthetic (seeded initial Maxwellian of the workload's macroscopic field)", "config": cfg,
               "kernels_ms_per_step": {k: v[0] / r["steps"] for k, v in r["prof"].items()},
               "newton": r["newton"], "roofline": roofline(r, w["p"])}
        if not args.no_cpu:
            out["cpu_baseline"] = cpu_baseline(w, par, args.cpu_seconds)
        print(json.dumps(out), flush=True)
        return

    # compare mode: plain FP64 against mixed precision + learned Newton start
    p64 = dict(base, precision=0, rk=0, guess=0)
    pmx = dict(base, precision=1, rk=1, guess=3)
    r64 = run_config(W, w, mesh, p64, args.steps, args.warmup, "fp64-plain", keep_moments=True)
    err_t = None
    if not args.no_error:
        # FP64 time-discretisation error over the same horizon: dt/2, twice the steps
        rh = run_config(W, w, mesh, p64, args.steps, 0, "fp64-half-dt", keep_moments=True, dt_scale=0.5,
                        nsteps_override=2 * (args.steps + args.warmup))
        r64_long = run_config(W, w, mesh, p64, args.steps, 0, "fp64-ref", keep_moments=True,
                              nsteps_override=args.steps + args.warmup)
        err_t = rel_moments(r64_long["Q"], rh["Q"])
    weights, tinfo = train_guess(W, w, log)
    rmx = run_config(W, w, mesh, pmx, args.steps, args.warmup, "mixed-learned", weights=weights, keep_moments=True)
    err_m = rel_moments(rmx["Q"], r64["Q"])
    holds = None if err_t is None else all(err_m[k] <= err_t[k] for k in err_m)
    cfg.update(mixed="FP32 f, FP32 FR/RK arithmetic, FP64 moments + Newton; LSRK3-2N; learned then warm Newton start",
               plain="FP64 everything; SSP-RK3; cold Newton start")
    out = {"metric": "DOF-updates/s (N_e*N_s*N_u per RK stage), mixed+learned vs FP64 at equal error",
           "value": rmx["value"], "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": rmx["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 (FP64 moments and Newton)",
           "data": "synthetic (seeded initial Maxwellian of the workload's macroscopic field)", "config": cfg,
           "fp64_plain": {"value": r64["value"], "ms_per_step": r64["ms_per_step"],
                          "kernels_ms_per_step": {k: v[0] / r64["steps"] for k, v in r64["prof"].items()},
                          "newton": r64["newton"], "roofline": roofline(r64, w["p"])},
           "speedup_vs_fp64": rmx["value"] / r64["value"],
           "equal_error": {"mixed_vs_fp64_rel_l2": err_m, "fp64_dt_vs_half_dt_rel_l2": err_t, "holds": holds,
                           "horizon_steps": args.steps + args.warmup},
           "kernels_ms_per_step": {k: v[0] / rmx["steps"] for k, v in rmx["prof"].items()},
           "newton": rmx["newton"], "learned_guess": {k: tinfo[k] for k in ("n_converged", "train_seconds")},
           "roofline": roofline(rmx, w["p"])}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, p64, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def cpu_baseline(w: dict, params: dict, budget_s: float) -> dict:
    """The FP64 CPU oracle (unchanged, OpenMP over elements) on a bounded
    sample of the workload: same order, velocity grid and physics on a smaller
    periodic box, one SSP-RK3 step, DOF-updates per second."""
    import oracle
    import workloads as W

    oracle.build(force=False)
    par = dict(params)
    nsample = 2

    def one(n):
        mesh = W.box_mesh(n)
        P = oracle.Problem(mesh, w["p"], w["grid"], par)
        prim = W.initial_prim(mesh, w["p"], dict(w))
        f0 = W.maxwellian(prim, w["grid"]).numpy()
        t0 = time.perf_counter()
        P.rk_step(f0, P.dt(0.2), scheme=0, nsteps=1)
        return time.perf_counter() - t0, P.ne * P.ns * P.nu

    el, dof = one(nsample)
    if el < budget_s / 8:
        nsample = max(2, min(8, int(nsample * (budget_s / max(el, 1e-3)) ** (1 / 3))))
        el, dof = one(nsample)
    return {"value": dof * 3 / el, "unit": "DOF-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one SSP-RK3 step on a {nsample}^3-element periodic box, p={w['p']}, "
                      f"{w['grid']['n'][0]}^3 velocities ({dof:.3e} DOFs), FP64, {el:.1f} s"}


if __name__ == "__main__":
    main()
