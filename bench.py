#!/usr/bin/env python3
"""Throughput benchmark of the FR x conservative-DVM hot path on one MI355X.

A step is one explicit time step (three RK stages) over the whole phase space
of the workload; the metric counts DOF-updates per second, one DOF-update
being one of the N_e * N_s * N_u values advanced by one RK stage.

Default (``--mode compare``, workload box24_p3_v20_es: 24^3 periodic hexes,
p = 3, 20^3 velocities on [-8, 8]^3, ES-BGK Pr 0.71, Kn 2e-4, Taylor-Green
U0 = 0.5 with a 1 % seeded perturbation):
  * plain FP64: FP64 storage and arithmetic, SSP-RK3, warm-start Newton;
  * mixed + learned: the mixed storage form (see ``MIXED``), the low-storage
    RK scheme (the configuration's), FP64 moments and Newton, Newton started from the learned guess where no
    previous solution exists (MLP trained first, untimed, on states of this
    grid including the solver's own initial states) and warm afterwards;
  both timed over the same K steps from the same initial state after the
  same warm-up, so both timed runs use the warm start and the speed-up is
  that of the storage form.  The learned start acts where no previous
  solution exists: the first solve of a run, reported separately (cold vs
  learned start on the initial state).  ``value`` is the mixed throughput,
  reported under the equal-error metric only when equal error holds.  Equal
  error (untimed runs over the workload's horizon, 200 steps at 24^3): the
  relative L2 difference of the conserved moments between the two forms is
  compared with the FP64 solution's own discretisation error, temporal from
  a dt / 2 FP64 run and spatial by Richardson from an N / 2 FP64 run; the
  conservation drift of both runs is reported too.
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
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = {0: 78.6, 1: 157.3}  # MI355X vector FP64 / FP32

# The mixed storage form of the compare mode (precision code of fr_dvm_params):
# FR_DVM_FP32_DEV, f held in FP32 as its deviation from an element reference
# equilibrium between stages, FP32 stage arithmetic on the deviations.
MIXED = 2
MIXED_LABEL = ("FP32 storage and FP32 FR/RK arithmetic of the deviation of f from an element reference "
               "equilibrium (FP32 f at call boundaries), FP32 traces and RK register, FP64 moments and Newton")
MIXED_DTYPE = "f32 (deviation from an element reference), FP64 moments and Newton"
# RK scheme of the compare mode's reduced-precision forms: the low-storage
# scheme the configuration names; the mixed storage form is also run with
# SSP-RK3 (as the FP64 run; 20 % fewer register bytes per step) and reported
# beside it
MIXED_RK = 1


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def value_sizes(precision: int):
    """Bytes of a state value and of a trace value: FP64 (0) 8 / 8, FP32 (1)
    and FP32 deviation storage (2) 4 / 4."""
    return (8, 8) if precision == 0 else (4, 4)


def stage_values_per_dof(p: int, rk: int, stage: int, last: bool):
    """Algorithmic HBM traffic of one fused stage launch per DOF, as (state
    values, trace values): read the stage value f and write the result; read
    the neighbours' outflow traces (3/(p+1) values per DOF) and, unless it is
    the last stage of the call, write the result's own outflow traces
    (3/(p+1)); SSP-RK3 reads f^n in stages 2 and 3; the low-storage scheme
    reads dF in stages 2 and 3 and writes it in stages 1 and 2 (after stage 3
    it is dead).  (Moments and equilibrium records are per solution point,
    not per DOF: below 0.1 % at 20^3 velocities.)"""
    tr = 3.0 / (p + 1)
    v = 2.0
    if stage > 0:
        v += 1.0
    if rk == 1 and stage < 2:
        v += 1.0
    return v, tr + (0.0 if last else tr)


def gen_stage_values_per_dof(p: int, rk: int, stage: int, last: bool):
    """The same for a stage on a general hexahedral mesh (stage kernel plus
    the moment pass over its result): read f, write the result; read the
    neighbour traces where the velocity enters (half of the 6/(p+1) full
    traces per DOF) and, unless last, write the result's full traces
    (6/(p+1)) and read the result once more for its moments; the second RK
    register as for the box kernel."""
    full = 6.0 / (p + 1)
    v = 2.0 + (0.0 if last else 1.0)
    if stage > 0:
        v += 1.0
    if rk == 1 and stage < 2:
        v += 1.0
    return v, 0.5 * full + (0.0 if last else full)


def stage_bytes(p: int, precision: int, rk: int, nsteps: int, general: bool = False) -> float:
    """Algorithmic bytes per DOF summed over the stage launches of one
    rk_steps call of nsteps steps."""
    per = gen_stage_values_per_dof if general else stage_values_per_dof
    es, te = value_sizes(precision)
    tot = 0.0
    for k in range(nsteps):
        for st in range(3):
            sv, tv = per(p, rk, st, k == nsteps - 1 and st == 2)
            tot += sv * es + tv * te
    return tot


KERNEL_SOURCES = ("frdvm_fr.hip", "frdvm_dev.h", "frdvm_common.h")
GEN_KERNEL_SOURCES = ("frdvm_gen.hip", "frdvm_dev.h", "frdvm_common.h")


def kernel_source_hash(general: bool = False) -> str:
    """Hash of the sources the stage kernel (box meshes, or with general=True
    the general-mesh stage, wall and moment kernels) is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in (GEN_KERNEL_SOURCES if general else KERNEL_SOURCES):
        with open(os.path.join(ROOT, "paper_2312_06567_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, precision: int, rk: int, delta: float = 0.0, general: bool = False):
    """HBM bytes per stage launch from the committed rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE, calibrated on a copy kernel), or None when
    no run matches this configuration or the kernel source has changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        recs = json.load(fh)
    src = kernel_source_hash(general)
    for r in recs:
        if (r["workload"] == workload and r["precision"] == precision and r["rk"] == rk
                and r.get("delta", 0.0) == delta and r["source"] == src):
            return r
    return None


def run_config(W, w, mesh, params, steps, warmup, label, weights=None, keep_moments=False, dt_scale=1.0,
               nsteps_override=None, dt_override=None, keep_f=False):
    """Build a handle, generate f0 on the GPU, warm up, time `steps` steps.
    Returns a dict with timing, kernel times and (optionally) final moments."""
    import numpy as np
    import torch

    from paper_2312_06567_amd.frdvm import FrDvm
    delta = float(w.get("delta", 0.0))
    s = FrDvm(mesh, w["p"], w["grid"], params, delta=delta)
    if weights is not None:
        s.mlp_set_weights(weights)
    ne, ns, nu = s.shape  # nu: state values per point (both components of a pair)
    dof = ne * ns * s.nu  # N_e N_s N_u: velocity nodes, once for the pair (F, G)
    dt = (s.dt(0.2) if dt_override is None else dt_override) * dt_scale
    prim = W.initial_prim(mesh, w["p"], w)
    log(f"{label}: generating f0 ({dof:.3e} DOFs, {s.dtype})")
    if delta > 0:
        # the pair in equilibrium: G = delta theta / 2 F
        Fm = W.maxwellian(prim, w["grid"], dtype=s.dtype, device="cuda").reshape(ne, ns, nu // 2)
        th = torch.as_tensor(prim[..., 4], dtype=s.dtype, device="cuda").reshape(ne, ns, 1)
        f = torch.cat([Fm, 0.5 * delta * th * Fm], -1).contiguous()
        del Fm
    else:
        f = W.maxwellian(prim, w["grid"], dtype=s.dtype, device="cuda").reshape(ne, ns, nu)
    torch.cuda.synchronize()
    tot0 = None
    if keep_moments:
        Q0 = torch.empty(ne * ns * 5, dtype=torch.float64, device="cuda")
        tot0 = s.moments(f, Q0, totals=True)
        del Q0
    if warmup:
        s.rk_steps(f, dt, warmup)
        torch.cuda.synchronize()
        log(f"{label}: {warmup} warmup step(s) done")
    n_timed = nsteps_override if nsteps_override is not None else steps
    s.newton_stats(reset=True)
    s.profile(True)
    s.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if n_timed <= 500:
        s.rk_steps(f, dt, n_timed)
    else:
        # long horizons in calls of 100 steps, each reported
        done = 0
        while done < n_timed:
            k = min(100, n_timed - done)
            s.rk_steps(f, dt, k)
            torch.cuda.synchronize()
            done += k
            log(f"{label}: {done}/{n_timed} steps")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = s.profile_read(reset=True)
    s.profile(False)
    stats = s.newton_stats(reset=True)
    log(f"{label}: {n_timed} steps in {elapsed:.3f} s")
    out = {"label": label, "dof": dof, "ncomp": s.ncomp, "steps": n_timed, "elapsed": elapsed, "dt": dt,
           "value": dof * 3 * n_timed / elapsed, "state_values_per_s": dof * s.ncomp * 3 * n_timed / elapsed,
           "ms_per_step": elapsed / n_timed * 1e3, "prof": prof,
           "stats": stats, "precision": params.get("precision", 0), "rk": params.get("rk", 0), "delta": delta}
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
        out["totals"] = [float(x) for x in tot]
        out["totals0"] = [float(x) for x in tot0]
    out["totals_finite"] = bool(torch.isfinite(f).all().item())
    if keep_f:
        out["f"] = f
        out["f_min"] = float(f.min().item())
    del f
    s.destroy()
    torch.cuda.empty_cache()
    return out


def roofline(r, p, workload, general=False):
    """The fused stage kernel against HBM bandwidth: algorithmic bytes of all
    its launches in the timed call over their summed HIP-event durations (on
    the library's stream).  General meshes: the stage kernel with its wall
    and moment passes."""
    ms, n = r["prof"]["stage"]
    tot_bytes = stage_bytes(p, r["precision"], r["rk"], r["steps"], general) * r["dof"] * r.get("ncomp", 1)
    ach = tot_bytes / (ms / 1e3) / 1e9
    name = "k_gen_stage + k_gen_wall + k_gen_moments (general hexes)" if general else "k_fr_layer (fused FR stage)"
    avg_ms = ms / max(n, 1)
    out = {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
           "algorithmic_bytes_per_launch": tot_bytes / max(n, 1), "avg_launch_ms": avg_ms}
    # the same launches priced with the unfused per-DOF traffic of the FR x
    # DVM stage (read f twice, the RK register, traces at both ends): p = 3
    # SSP FP64 56 B, FP32 28 B, low-storage FP32 32 B per DOF and stage
    ub = unfused_bytes_per_dof(p, r["precision"], r["rk"]) * r["dof"] * r.get("ncomp", 1)
    out["unfused_bytes_per_dof"] = unfused_bytes_per_dof(p, r["precision"], r["rk"])
    out["frac_unfused_bytes"] = ub / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS
    t = measured_traffic(workload, r["precision"], r["rk"], r.get("delta", 0.0), general)
    if t is not None:
        out["traffic"] = t["bytes_per_launch"]
        out["traffic_source"] = t["profile"]
        # bandwidth the launches actually drew: counted bytes over the live time
        out["counted_GBps"] = t["bytes_per_launch"] / (avg_ms / 1e3) / 1e9
        out["frac_counted"] = out["counted_GBps"] / HBM_PEAK_GBS
    # the FR operators (interpolation, derivative, correction) as flops: the
    # sum-factorised algorithm the kernel runs, and the dense-operator form
    # (derivative, lifting and face interpolation as dense products) that an
    # MFMA formulation would execute
    fpd = fr_operator_flops_per_dof(p)
    dofs = r["dof"] * r.get("ncomp", 1)
    out["fr_operator_flops"] = {
        "sum_factorised_per_dof": fpd, "dense_per_dof": fr_dense_flops_per_dof(p),
        "achieved_TFLOPs": fpd * dofs / (avg_ms / 1e3) / 1e12,
        "frac_of_vector_peak": fpd * dofs / (avg_ms / 1e3) / 1e12 / VALU_PEAK_TFLOPS[0 if r["precision"] == 0 else 1]}
    return out


def fr_operator_flops_per_dof(p: int) -> float:
    """Flops per DOF of the sum-factorised FR operators on a hexahedron of
    N = p + 1 points per direction: per direction the derivative along the
    point's line (N multiply-adds) and its metric scaling (one), the lifting
    of the line's inflow jump (one), and per line the inflow-side trace (N)
    and the jump (two flops), shared by the line's N points."""
    n = p + 1
    return 3.0 * (2 * n + 2 + 2 + (2 * n + 2) / n)


def fr_dense_flops_per_dof(p: int) -> float:
    """Flops per DOF of the same operators as dense products: per point
    three [N_s x N_s] derivative rows, one [N_s x N_f] lifting row, and its
    share of the [N_f x N_s] interpolation to the face points (N_s = N^3,
    N_f = 6 N^2)."""
    n = p + 1
    return 2.0 * (3 * n ** 3 + 2 * 6 * n ** 2)


# solution points and face points of each mixed-mesh element type at order p
# (hexahedron, prism, tetrahedron)
MIXED_SIZES = {1: ((8, 24), (6, 18), (4, 12)), 2: ((27, 54), (18, 39), (10, 24)),
               3: ((64, 96), (40, 68), (20, 40))}


def mixed_row_madds(t: int, p: int) -> int:
    """Multiply-adds per solution point and velocity of the operator rows of
    element type t (0 hexahedron, 1 prism, 2 tetrahedron): hexahedra and
    tetrahedra dense (three derivative rows of N_s entries, a lifting row of
    N_ft); the prism's rows hold only its layer / column structure (two
    in-plane rows of N_s / (p + 1) entries and an axial one of p + 1; lifting
    from the two end-face points of its column and the 3 (p + 1) side-face
    points of its layer)."""
    ns, nft = MIXED_SIZES[p][t]
    if t == 1:
        nl = p + 1
        return 2 * (ns // nl) + nl + 2 + 3 * nl
    return 3 * ns + nft


def mixed_flops_per_dof(mesh, p: int) -> float:
    """Algorithmic flops per DOF of a mixed-mesh stage: 2 x the operator
    multiply-adds per point (mixed_row_madds), averaged over the mesh's
    points."""
    import numpy as np
    counts = np.bincount(np.asarray(mesh["elem_type"]), minlength=3)
    pts = sum(int(counts[t]) * MIXED_SIZES[p][t][0] for t in range(3))
    fl = sum(int(counts[t]) * MIXED_SIZES[p][t][0] * 2 * mixed_row_madds(t, p) for t in range(3))
    return fl / pts


def mixed_roofline(r, p, mesh):
    """The mixed-mesh stage (dense element operators, VALU) against the
    vector ALU peak of its precision: algorithmic flops of the stage launches
    over their summed HIP-event durations."""
    ms, n = r["prof"]["stage"]
    fpd = mixed_flops_per_dof(mesh, p)
    ach = fpd * r["dof"] * 3 * r["steps"] / (ms / 1e3) / 1e12
    peak = VALU_PEAK_TFLOPS[0 if r["precision"] == 0 else 1]
    # HBM: read f, write the result, the low-storage register (read in 2 of 3
    # stages, written in 2 of 3), read the neighbour traces where the velocity
    # enters (half the face points), write the result's traces, read the
    # result again for its moments
    import numpy as np
    counts = np.bincount(np.asarray(mesh["elem_type"]), minlength=3)
    pts = sum(int(counts[t]) * MIXED_SIZES[p][t][0] for t in range(3))
    fpts = sum(int(counts[t]) * MIXED_SIZES[p][t][1] for t in range(3))
    vals = 3.0 + (4.0 / 3.0 if r["rk"] == 1 else 2.0 / 3.0) + 1.5 * fpts / pts
    bpd = vals * (8 if r["precision"] == 0 else 4)
    gbs = bpd * r["dof"] * 3 * r["steps"] / (ms / 1e3) / 1e9
    return {"kernel": "k_mix_stage (+ k_gen_moments), element operators (prisms: layer/column structure)", "bound": "alu", "achieved": ach,
            "peak": peak, "unit": "TFLOP/s", "frac": ach / peak, "traffic": None,
            "flops_per_dof": fpd, "avg_launch_ms": ms / max(n, 1),
            "hbm_bytes_per_dof": bpd, "hbm_GBps": gbs, "frac_hbm": gbs / HBM_PEAK_GBS}


def unfused_bytes_per_dof(p: int, precision: int, rk: int) -> float:
    """Per-DOF traffic of one RK stage when its parts are separate passes
    (moments read f, the residual reads f and writes traces of r = 6/(p+1)
    face values and reads them back, the update reads the RK register and
    writes f): 4 state values plus 2 r trace values for SSP-RK3, one more
    state value for the low-storage register's second access.  p = 3: FP64
    SSP 56 B, FP32 SSP 28 B, FP32 low-storage 32 B."""
    es, te = value_sizes(precision)
    r = 6.0 / (p + 1)
    return es * (4.0 + (1.0 if rk == 1 else 0.0)) + te * 2.0 * r


def coarse_to_fine(Qc, Nc, p):
    """Evaluate the degree-p element polynomials of a field given at the Gauss
    points of the periodic Nc^3 box mesh at the Gauss points of the 2Nc^3
    mesh of the same box (element id ix + N (iy + N iz), point i + n (j + n l)).
    Qc: [Nc^3 * n^3, k] -> [(2Nc)^3 * n^3, k]."""
    import numpy as np

    import workloads as W
    n = p + 1
    xi = W.gauss_points(p)
    k = Qc.shape[-1]
    # 1-D Lagrange basis of the coarse nodes at the fine nodes of half s
    B = np.empty((2, n, n))
    for s_ in range(2):
        xc = -1.0 + s_ + (xi + 1.0) / 2.0
        for m in range(n):
            others = [xi[o] for o in range(n) if o != m]
            B[s_, :, m] = np.prod([(xc - xo) / (xi[m] - xo) for xo in others], axis=0)
    Q6 = Qc.reshape(Nc, Nc, Nc, n, n, n, k)  # [iz, iy, ix, l, j, i, k]
    F = np.empty((2 * Nc, 2 * Nc, 2 * Nc, n, n, n, k))
    for sz in range(2):
        for sy in range(2):
            for sx in range(2):
                F[sz::2, sy::2, sx::2] = np.einsum("cl,bj,ai,ZYXljiq->ZYXcbaq", B[sz], B[sy], B[sx], Q6)
    return F.reshape(-1, k)


def f_rel_l2(fa, fb):
    """Relative L2 difference of two distributions on the GPU, in FP64,
    taken in slabs (fa may be FP32)."""
    num = 0.0
    den = 0.0
    for a, b in zip(fa.reshape(-1, fa.shape[-1]).split(4096), fb.reshape(-1, fb.shape[-1]).split(4096)):
        num += float((a.double() - b.double()).pow(2).sum().item())
        den += float(b.double().pow(2).sum().item())
    return math.sqrt(num / den)


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


def first_solve(W, w, mesh, params, weights):
    """The learned start where it acts: the first conservative-equilibrium
    solve of a run (no previous solution at any point), on the workload's
    initial state, from the cold start and from the learned start.  Newton
    linear solves and grid passes per point, fallbacks, the largest final
    residual and the Newton kernel time (HIP events)."""
    import numpy as np
    import torch

    from paper_2312_06567_amd.frdvm import FrDvm
    out = {}
    for label, guess in (("cold", 0), ("learned", 2)):
        s = FrDvm(mesh, w["p"], w["grid"], dict(params, guess=guess))
        if guess == 2:
            s.mlp_set_weights(weights)
        ne, ns, nu = s.shape
        f = W.maxwellian(W.initial_prim(mesh, w["p"], w), w["grid"], dtype=s.dtype, device="cuda").reshape(ne, ns, nu)
        S = torch.empty_like(f)
        s.collide(f, S)  # compiles / warms the kernels
        s.newton_stats(reset=True)
        s.profile(True)
        s.profile_read(reset=True)
        s.collide(f, S)
        prof = s.profile_read(reset=True)
        st = s.newton_stats(reset=True)
        hist = st["hist"]
        nsol = max(int(hist.sum()), 1)
        out[label] = {"mean_solves": float((hist * np.arange(64)).sum() / nsol),
                      "mean_passes": float(st["n_evals"] / nsol), "fallback": int(st["n_fallback"]),
                      "max_resid": float(st["max_resid"]), "newton_ms": prof["newton"][0],
                      "mlp_ms": prof["other"][0]}
        del f, S
        s.destroy()
        torch.cuda.empty_cache()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="box24_p3_v20_es")
    ap.add_argument("--mode", choices=("compare", "single", "kn", "horizon"), default="compare")
    ap.add_argument("--precision", type=int, default=None,
                    help="single and horizon modes: 0 FP64, 1 FP32, 2 FP32 deviation storage")
    ap.add_argument("--rk", type=int, default=None, help="single mode: 0 SSP-RK3, 1 low-storage")
    ap.add_argument("--guess", type=int, default=None, help="single mode: 0 cold, 1 warm, 2 MLP, 3 MLP then warm")
    ap.add_argument("--model", type=int, default=None, help="0 BGK, 1 ES-BGK, 2 collisionless")
    ap.add_argument("--delta", type=float, default=None,
                    help="single mode: internal degrees of freedom (> 0: the reduced pair F, G)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-error", action="store_true",
                    help="compare mode: skip the error runs at the workload's horizon")
    ap.add_argument("--horizon", type=int, default=None,
                    help="compare mode: steps of the error runs (default: the workload's, 200 at 24^3)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="instead of the benchmark, copy this many GiB with the library's plain copy kernel "
                         "(calibration of the HBM byte counters) and print its bandwidth")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on exactly one GPU; multi-GPU sharding is not implemented",
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
    if args.delta is not None:
        w["delta"] = args.delta
    mesh = W.workload_mesh(w)
    base = W.physics_params(w)
    if args.model is not None:
        base["model"] = args.model
    cfg = {"workload": w["name"], "n_elem": int(mesh["n_elem"]), "p": w["p"], "ns": (w["p"] + 1) ** 3,
           "nu": int(w["grid"]["n"][0] * w["grid"]["n"][1] * w["grid"]["n"][2]),
           "model": ["BGK", "ES-BGK", "free"][base["model"]], "prandtl": base["prandtl"], "kn": w["kn"],
           "parallelism": "single GPU"}

    if args.mode == "kn":
        print(json.dumps(kn_bench(W, w, mesh, base, args, cfg)), flush=True)
        return

    if args.mode == "horizon":
        print(json.dumps(horizon_compare(W, w, mesh, base, args, cfg)), flush=True)
        return

    if args.mode == "single":
        par = dict(base)
        par["precision"] = w["precision"] if args.precision is None else args.precision
        par["rk"] = w["rk"] if args.rk is None else args.rk
        par["guess"] = 0 if args.guess is None else args.guess
        weights = None
        if par["guess"] in (2, 3):
            weights, _ = train_guess(W, w, log)
        r = run_config(W, w, mesh, par, args.steps, args.warmup, "single", weights=weights)
        if w.get("delta", 0.0) > 0:
            cfg.update(delta=w["delta"], state="reduced pair (F, G): 2 values per velocity node")
        cfg.update(precision=["FP64", "FP32", "FP32 deviation storage"][par["precision"]],
                   rk=["SSP-RK3", "LSRK3-2N"][par["rk"]],
                   guess=["cold", "warm", "learned", "learned+warm"][par["guess"]])
        out = {"metric": "DOF-updates/s (N_e*N_s*N_u per RK stage)", "value": r["value"], "unit": "DOF-updates/s",
               "n_gpus": 1, "steps": r["steps"], "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": ["f64", "f32 (FP64 moments and Newton)", MIXED_DTYPE][par["precision"]],
               "data": "synthetic (seeded initial Maxwellian of the workload's macroscopic field)", "config": cfg,
               "kernels_ms_per_step": {k: v[0] / r["steps"] for k, v in r["prof"].items()},
               "newton": r["newton"],
               "roofline": mixed_roofline(r, w["p"], mesh) if "elem_type" in mesh
               else roofline(r, w["p"], w["name"], w.get("mesh") == "cylinder")}
        if "elem_type" in mesh:
            import numpy as np
            cnt = np.bincount(np.asarray(mesh["elem_type"]), minlength=3)
            cfg.update(elements={"hexahedra": int(cnt[0]), "prisms": int(cnt[1]), "tetrahedra": int(cnt[2])},
                       points=int(r["dof"] // cfg["nu"]), ns=None)
        if not args.no_cpu:
            out["cpu_baseline"] = cpu_baseline(w, par, args.cpu_seconds)
        print(json.dumps(out), flush=True)
        return

    # compare mode: plain FP64 against the mixed form + learned Newton start;
    # both timed with the warm start (the learned start acts at the first
    # solve only, reported by first_solve)
    p64 = dict(base, precision=0, rk=0, guess=1)
    pmx = dict(base, precision=MIXED, rk=MIXED_RK, guess=3)
    r64 = run_config(W, w, mesh, p64, args.steps, args.warmup, "fp64-plain", keep_moments=True)
    weights, tinfo = train_guess(W, w, log)
    rmx = run_config(W, w, mesh, pmx, args.steps, args.warmup, "mixed-learned", weights=weights, keep_moments=True)
    # the plain FP32 form (FP32 state, stochastic rounding, FP32 stage
    # arithmetic) timed beside them
    p32 = dict(base, precision=1, rk=MIXED_RK, guess=3)
    r32 = run_config(W, w, mesh, p32, args.steps, args.warmup, "fp32-learned", weights=weights, keep_moments=True)
    # the mixed storage form with SSP-RK3
    psp = dict(base, precision=MIXED, rk=0, guess=3)
    rsp = run_config(W, w, mesh, psp, args.steps, args.warmup, "mixed-ssp", weights=weights, keep_moments=True)
    err = None
    f_err = None
    if args.no_error:
        # moment difference after the timed runs only
        horizon = args.steps + args.warmup
        a64, amx, a32, asp = r64, rmx, r32, rsp
    else:
        # the error comparison runs the workload's own horizon (untimed):
        # FP64 and mixed + learned from the same initial state, and the
        # discretisation error of the FP64 solution at that horizon:
        # temporal from a dt/2 run, spatial from the N/2 mesh at the same dt
        # (Richardson with order p+1: e_N ~ |Q_N - I Q_N/2| / (2^(p+1) - 1))
        horizon = args.horizon if args.horizon is not None else int(w.get("steps", args.steps + args.warmup))
        a64 = run_config(W, w, mesh, p64, 0, 0, "fp64-horizon", keep_moments=True, nsteps_override=horizon,
                         keep_f=True)
        amx = run_config(W, w, mesh, pmx, 0, 0, "mixed-horizon", weights=weights, keep_moments=True,
                         nsteps_override=horizon, keep_f=True)
        a32 = run_config(W, w, mesh, p32, 0, 0, "fp32-horizon", weights=weights, keep_moments=True,
                         nsteps_override=horizon, keep_f=True)
        # relative L2 difference of f itself from the FP64 run
        f_err = {"mixed": f_rel_l2(amx.pop("f"), a64["f"]), "fp32": f_rel_l2(a32.pop("f"), a64["f"])}
        asp = run_config(W, w, mesh, psp, 0, 0, "mixed-ssp-horizon", weights=weights, keep_moments=True,
                         nsteps_override=horizon, keep_f=True)
        f_err["mixed_ssp"] = f_rel_l2(asp.pop("f"), a64["f"])
        del a64["f"]
        import torch
        torch.cuda.empty_cache()
        rh = run_config(W, w, mesh, p64, 0, 0, "fp64-half-dt", keep_moments=True, dt_scale=0.5,
                        nsteps_override=2 * horizon)
        mesh_c = W.box_mesh(w["N"] // 2)
        rc = run_config(W, w, mesh_c, p64, 0, 0, "fp64-coarse", keep_moments=True, dt_override=a64["dt"],
                        nsteps_override=horizon)
        e_t = rel_moments(a64["Q"], rh["Q"])
        e_s = {k: v / (2 ** (w["p"] + 1) - 1)
               for k, v in rel_moments(coarse_to_fine(rc["Q"], w["N"] // 2, w["p"]), a64["Q"]).items()}
        err = {"temporal": e_t, "spatial": e_s, "total": {k: e_t[k] + e_s[k] for k in e_t}}
    err_m = rel_moments(amx["Q"], a64["Q"])
    # equal error: the mixed run differs from the FP64 run by less than a
    # tenth of the FP64 run's own discretisation error, field by field
    holds = None if err is None else all(err_m[k] <= 0.1 * err["total"][k] for k in err_m)
    # drift of each conserved total over the run; momentum totals are near
    # zero, so momentum is scaled by sqrt(2 * mass * energy), a momentum of
    # the flow's own thermal-plus-bulk speed
    def drift_of(r):
        t0, t1 = r["totals0"], r["totals"]
        ref = [abs(t0[0]), *[math.sqrt(2.0 * abs(t0[0] * t0[4]))] * 3, abs(t0[4])]
        return {k: abs(t1[i] - t0[i]) / max(ref[i], 1e-300)
                for i, k in enumerate(("rho", "rhoUx", "rhoUy", "rhoUz", "E"))}
    drift = {lab: drift_of(r) for lab, r in (("fp64", a64), ("mixed", amx), ("fp32", a32), ("mixed_ssp", asp))}
    err_32 = rel_moments(a32["Q"], a64["Q"])
    err_sp = rel_moments(asp["Q"], a64["Q"])
    first = first_solve(W, w, mesh, dict(base, precision=MIXED, rk=MIXED_RK), weights)
    rk_name = ["SSP-RK3", "LSRK3-2N"][MIXED_RK]
    cfg.update(mixed=MIXED_LABEL + f"; {rk_name}; learned then warm Newton start",
               plain="FP64 everything; SSP-RK3; warm Newton start")
    metric = "DOF-updates/s (N_e*N_s*N_u per RK stage), mixed+learned vs FP64 at equal error"
    if holds is not True:
        metric = "DOF-updates/s (N_e*N_s*N_u per RK stage), mixed precision; equal error NOT reached"
    out = {"metric": metric, "equal_error_holds": holds,
           "value": rmx["value"], "unit": "DOF-updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": rmx["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": MIXED_DTYPE,
           "data": "synthetic (seeded initial Maxwellian of the workload's macroscopic field)", "config": cfg,
           "fp64_plain": {"value": r64["value"], "ms_per_step": r64["ms_per_step"],
                          "kernels_ms_per_step": {k: v[0] / r64["steps"] for k, v in r64["prof"].items()},
                          "newton": r64["newton"], "roofline": roofline(r64, w["p"], w["name"])},
           "speedup_vs_fp64": rmx["value"] / r64["value"],
           "equal_error": {"mixed_vs_fp64_rel_l2": err_m, "fp64_discretisation_rel_l2": err, "holds": holds,
                           "f_vs_fp64_rel_l2": f_err,
                           "criterion": "mixed_vs_fp64 <= 0.1 * (temporal + spatial) per conserved field",
                           "horizon_steps": horizon, "conservation_drift": drift},
           "kernels_ms_per_step": {k: v[0] / rmx["steps"] for k, v in rmx["prof"].items()},
           "newton": rmx["newton"], "learned_guess": {k: tinfo[k] for k in ("n_converged", "train_seconds")},
           "learned_start_first_solve": first,
           "fp32_form": {"label": "FP32 f (stochastic rounding), FP32 FR/RK arithmetic, FP64 moments + Newton; "
                                  f"{rk_name}; learned then warm Newton start",
                         "value": r32["value"], "ms_per_step": r32["ms_per_step"],
                         "speedup_vs_fp64": r32["value"] / r64["value"],
                         "kernels_ms_per_step": {k: v[0] / r32["steps"] for k, v in r32["prof"].items()},
                         "mixed_vs_fp64_rel_l2": err_32,
                         "ratio_to_fp64_discretisation": None if err is None else
                         {k: err_32[k] / err["total"][k] for k in err_32},
                         "equal_error_holds": None if err is None else
                         all(err_32[k] <= 0.1 * err["total"][k] for k in err_32),
                         "roofline": roofline(r32, w["p"], w["name"])},
           "ssp_form": {"label": MIXED_LABEL + "; SSP-RK3 (as the FP64 run); learned then warm Newton start",
                        "value": rsp["value"], "ms_per_step": rsp["ms_per_step"],
                        "speedup_vs_fp64": rsp["value"] / r64["value"],
                        "kernels_ms_per_step": {k: v[0] / rsp["steps"] for k, v in rsp["prof"].items()},
                        "mixed_vs_fp64_rel_l2": err_sp,
                        "ratio_to_fp64_discretisation": None if err is None else
                        {k: err_sp[k] / err["total"][k] for k in err_sp},
                        "equal_error_holds": None if err is None else
                        all(err_sp[k] <= 0.1 * err["total"][k] for k in err_sp),
                        "roofline": roofline(rsp, w["p"], w["name"])},
           "roofline": roofline(rmx, w["p"], w["name"])}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, p64, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def horizon_compare(W, w, mesh, base, args, cfg):
    """The mixed form against FP64 after the workload's horizon (2000 steps
    on the Mach-8 O-grid) from the same initial state: relative L2
    differences of rho, rho U, E and f, the domain totals of both runs and
    their Newton outcomes; both runs timed (HIP-event kernel times)."""
    import numpy as np
    import torch
    H = args.horizon if args.horizon is not None else int(w.get("steps", 100))
    r64 = run_config(W, w, mesh, dict(base, precision=0, rk=0, guess=1), 0, 0, "fp64-horizon", keep_moments=True,
                     nsteps_override=H, keep_f=True)
    # the reduced-precision form: --precision / --rk when given, else the
    # deviation storage on box meshes (FP32 elsewhere) with the low-storage RK
    mprec = args.precision if args.precision is not None else (MIXED if w.get("mesh") != "cylinder" else 1)
    mrk = args.rk if args.rk is not None else 1
    rmx = run_config(W, w, mesh, dict(base, precision=mprec, rk=mrk, guess=1), 0, 0, "mixed-horizon",
                     keep_moments=True, nsteps_override=H, keep_f=True)
    f64, fmx = r64.pop("f"), rmx.pop("f")
    ferr = f_rel_l2(fmx, f64)
    del f64, fmx
    torch.cuda.empty_cache()
    err = bench_rel = rel_moments(rmx["Q"], r64["Q"])
    err["f"] = ferr
    cfg = dict(cfg, mixed=(MIXED_LABEL if mprec == MIXED else "FP32 f, FP32 FR/RK arithmetic, FP64 moments + Newton")
               + "; " + ["SSP-RK3", "LSRK3-2N"][mrk] + "; warm Newton start",
               plain="FP64 everything; SSP-RK3; warm Newton start", positivity=base.get("positivity", 0))
    return {"metric": "mixed vs FP64 relative L2 difference at the horizon", "horizon_steps": H,
            "mixed_vs_fp64_rel_l2": bench_rel, "config": cfg,
            "fp64": {k: r64[k] for k in ("value", "ms_per_step", "newton", "totals0", "totals", "f_min")},
            "mixed": {k: rmx[k] for k in ("value", "ms_per_step", "newton", "totals0", "totals", "f_min")},
            "speedup_vs_fp64": rmx["value"] / r64["value"]}


def kn_bench(W, w, mesh, base, args, cfg):
    """Local Knudsen number of the whole field: the moment pass over f plus
    the per-element gradient kernel, timed with HIP events over `steps`
    calls.  Algorithmic bytes: read f once, write and read the moments, write
    Kn."""
    import torch

    from paper_2312_06567_amd.frdvm import FrDvm
    par = dict(base, precision=w["precision"] if args.precision is None else args.precision)
    s = FrDvm(mesh, w["p"], w["grid"], par)
    ne, ns, nu = s.shape
    f = W.maxwellian(W.initial_prim(mesh, w["p"], w), w["grid"], dtype=s.dtype, device="cuda").reshape(ne, ns, nu)
    kn = torch.empty(ne * ns, dtype=torch.float64, device="cuda")
    for _ in range(max(args.warmup, 1)):
        s.kn_gll(f, kn)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        s.kn_gll(f, kn)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    es = 8 if par["precision"] == 0 else 4
    nbytes = ne * ns * (nu * es + (10 if par["model"] == 1 else 5) * 8 * 2 + 8)
    ach = nbytes / (ms / 1e3) / 1e9
    kmax = float(kn.max().item())
    cfg = dict(cfg, precision=["FP64", "FP32", "FP32 (deviation storage: plain FP32 here)"][par["precision"]])
    return {"metric": "local Knudsen number field evaluations/s", "value": 1e3 / ms, "unit": "fields/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_call": ms, "higher_is_better": True,
            "dtype": "f64" if par["precision"] == 0 else "f32 (FP64 moments and gradient)", "data": "synthetic",
            "config": cfg, "kn_max": kmax,
            "roofline": {"kernel": "moment pass + k_kn_gll", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                         "algorithmic_bytes_per_call": nbytes}}


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
    # the same oracle on one thread (a child process: OpenMP reads the
    # thread count at start-up), on the 2^3-element sample
    one_thread = None
    import subprocess
    code = ("import sys, time, json; sys.path.insert(0, %r); import workloads as W, oracle; "
            "w = W.workload(%r); p = json.loads(%r); mesh = W.box_mesh(2); "
            "P = oracle.Problem(mesh, w['p'], w['grid'], p); "
            "f0 = W.maxwellian(W.initial_prim(mesh, w['p'], w), w['grid']).numpy(); "
            "t0 = time.perf_counter(); P.rk_step(f0, P.dt(0.2), scheme=0, nsteps=1); "
            "print(json.dumps([time.perf_counter() - t0, P.ne * P.ns * P.nu]))") % (ROOT, w["name"], json.dumps(par))
    try:
        r = subprocess.run([sys.executable, "-c", code], env=dict(os.environ, OMP_NUM_THREADS="1"),
                           capture_output=True, text=True, timeout=600)
        el1, dof1 = json.loads(r.stdout.strip().splitlines()[-1])
        one_thread = {"value": dof1 * 3 / el1, "seconds": el1,
                      "sample": f"one SSP-RK3 step on the 2^3-element box ({dof1:.3e} DOFs)"}
    except Exception as exc:  # reported, not fatal
        one_thread = {"error": str(exc)[:200]}
    return {"value": dof * 3 / el, "unit": "DOF-updates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(), "one_thread": one_thread,
            "sample": f"one SSP-RK3 step on a {nsample}^3-element periodic box, p={w['p']}, "
                      f"{w['grid']['n'][0]}^3 velocities ({dof:.3e} DOFs), FP64, {el:.1f} s"}


if __name__ == "__main__":
    main()
