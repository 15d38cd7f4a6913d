"""Learned initial guess for the conservative-equilibrium Newton solve.

Training data are states the solver itself produces: for each macroscopic
state the library's FP64 Newton (``fr_dvm_equilibrium``, cold start) gives the
converged unknowns z*; the network learns dz = z* - z_cold from the features
[ln rho, U/u_max, ln theta, u_max/10, n_v/32].  Forward, backward and Adam
run in the library's HIP kernels (``fr_mlp_*``); this module only batches
tensors and calls them.  At use, ``FrDvm.mlp_set_weights`` loads the network
into the Newton kernel, which starts from z_cold + dz and still iterates to
the FP64 tolerance (falling back to the cold start if the guess fails).
"""
from __future__ import annotations

import math
import sys

import numpy as np

from . import frdvm

Z_COLD = np.array([-1.5 * math.log(2 * math.pi), 0.0, 0.0, 0.0, 1.0])


def _grid(umax: float, nv: int) -> dict:
    return {"n": (nv, nv, nv), "umin": (-umax,) * 3, "umax": (umax,) * 3}


def handle_for_grid(umax: float, nv: int, tol=1e-13, max_iter=100):
    """A one-element handle whose only purpose is its velocity grid."""
    import workloads as W
    return frdvm.FrDvm(W.box_mesh(1), 1, _grid(umax, nv),
                       {"model": frdvm.BGK, "mu_ref": 1.0, "newton_tol": tol, "newton_max_iter": max_iter})


def features(rho, U, theta, umax, nv):
    """Network inputs as float32, the formula of the library's feature kernel
    for the grid [-u_max, u_max]^3 with nv nodes per axis: [ln rho, U/u_max,
    ln theta, u_max/10, n_v/32, sin phi, cos phi] with the grid phase
    phi = 2 pi (U + u_max)/du of the bulk velocity."""
    import torch
    rho = torch.as_tensor(rho, dtype=torch.float64)
    U = torch.as_tensor(U, dtype=torch.float64)
    th = torch.as_tensor(theta, dtype=torch.float64)
    um = torch.as_tensor(umax, dtype=torch.float64).reshape(-1, 1).expand(rho.shape[0], 1)
    du = 2.0 * um / (nv - 1)
    ph = 2.0 * math.pi * (U + um) / du
    X = torch.cat([rho.log()[:, None], U / um, th.log()[:, None], um / 10.0,
                   torch.full_like(um, nv / 32.0), ph.sin(), ph.cos()], 1)
    return X.float()


def envelope(U, theta, umax, nv):
    """Size of the discrete-velocity error of the continuous equilibrium on
    the closed grid [-u_max, u_max]^3 with nv nodes per axis: trapezoid
    aliasing exp(-2 pi^2 theta / du^2) plus truncation by the box
    max_d exp(-(u_max - |U_d|)^2 / (2 theta)).  The network predicts the
    Newton correction in units of this envelope (the same formula runs in the
    feature kernel of the library)."""
    U = np.asarray(U, np.float64)
    th = np.asarray(theta, np.float64)
    um = np.asarray(umax, np.float64)
    du = 2.0 * um / (nv - 1)
    gap = np.clip(um[:, None] - np.abs(U), 0.0, None)
    tr = np.exp(-gap ** 2 / (2.0 * th[:, None])).max(1)
    s = np.exp(-2.0 * math.pi ** 2 * th / du ** 2) + tr
    return np.clip(s, 1e-10, 1.0)  # below 1e-10 the correction is Newton round-off


def solve_targets(states: dict, nv: int = 32, guess=frdvm.GUESS_COLD, handles=None, weights=None):
    """FP64 Newton on the GPU for every state (grouped by u_max).  Returns a
    dict of numpy arrays: z* [n,5], iters (linear solves), evals (sum
    passes), status, resid."""
    import torch
    import workloads as W
    n = len(states["rho"])
    out = {"z": np.zeros((n, 5)), "iters": np.zeros(n, np.int32), "evals": np.zeros(n, np.int32),
           "status": np.zeros(n, np.int32), "resid": np.zeros(n)}
    Q = W.state_moments(states["rho"], states["U"], states["theta"])
    for um in np.unique(states["umax"]):
        idx = np.nonzero(states["umax"] == um)[0]
        h = handles[float(um)] if handles else handle_for_grid(float(um), nv)
        if weights is not None:
            h.mlp_set_weights(weights)
        Qd = torch.as_tensor(Q[idx], dtype=torch.float64, device="cuda").contiguous()
        res = h.equilibrium(Qd, guess)
        for key, t in zip(("z", "iters", "evals", "status", "resid"), res):
            out[key][idx] = t.cpu().numpy()
    return out


def train(X, T, H=64, steps=3000, batch=4096, lr=1e-3, seed=4, log_every=0, verbose=False):
    """Adam on the GPU with cosine learning-rate decay.  X [n,7], T [n,5]
    (unnormalised dz) float32 CUDA tensors.  Returns the flat weights (CUDA
    float32, with the target z-score folded into the output affine) and the
    loss history."""
    import torch
    mean = T.mean(0)
    std = T.std(0).clamp_min(1e-12)
    Tn = ((T - mean) / std).contiguous()
    net = frdvm.Mlp(H)
    rng = np.random.default_rng(seed)
    w0 = np.zeros(net.n, np.float32)
    o = 0
    for (m, k) in [(H, frdvm.MLP_INPUTS), (H, H), (H, H), (5, H)]:
        lim = math.sqrt(6.0 / k)
        w0[o:o + m * k] = rng.uniform(-lim, lim, m * k)
        o += m * k + m
    w0[o:o + 5] = std.cpu().numpy()
    w0[o + 5:o + 10] = mean.cpu().numpy()
    w = torch.as_tensor(w0, device="cuda")
    m1 = torch.zeros_like(w)
    m2 = torch.zeros_like(w)
    n = X.shape[0]
    B = min(batch, n)
    work = net.workspace(B)
    g = torch.empty_like(w)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    hist = []
    for step in range(1, steps + 1):
        idx = torch.randint(0, n, (B,), generator=gen, device="cuda")
        xb = X[idx].contiguous()
        tb = Tn[idx].contiguous()
        net.grad(w, xb, tb, g, loss, work)
        lr_t = lr * 0.5 * (1 + math.cos(math.pi * (step - 1) / steps))
        net.adam(w, g, m1, m2, step, lr_t)
        if log_every and (step % log_every == 0 or step == 1):
            hist.append((step, float(loss.item())))
            if verbose:
                print(f"[learned] step {step}/{steps} loss {hist[-1][1]:.4e}", file=sys.stderr, flush=True)
    return w, hist


def fit_guess(n_states=100_000, nv=32, H=64, steps=3000, seed=4, umax_choices=(6.0, 10.0, 14.0), extra=None,
              verbose=False):
    """Generate states, solve them, train the network.  `extra` may add
    solver-harvested states (dict of arrays rho, U, theta, umax).  Returns
    (weights as numpy float32, info dict)."""
    import torch
    import workloads as W
    st = W.sample_states(n_states, seed=seed, umax_choices=umax_choices, nv=nv)
    if extra is not None:
        for k in ("rho", "U", "theta", "umax"):
            st[k] = np.concatenate([st[k], extra[k]])
    sol = solve_targets(st, nv=nv)
    ok = sol["status"] == frdvm.NEWTON_OK
    if verbose:
        print(f"[learned] {int(ok.sum())} of {len(ok)} training states solved", file=sys.stderr, flush=True)
    X = features(st["rho"][ok], st["U"][ok], st["theta"][ok], st["umax"][ok], nv).cuda()
    env = envelope(st["U"][ok], st["theta"][ok], st["umax"][ok], nv)
    T = torch.as_tensor((sol["z"][ok] - Z_COLD) / env[:, None], dtype=torch.float32, device="cuda")
    w, hist = train(X, T, H=H, steps=steps, seed=seed, log_every=max(steps // 10, 1), verbose=verbose)
    info = {"n_states": int(len(ok)), "n_converged": int(ok.sum()), "reject_rate": float(st["reject_rate"]),
            "cold_mean_iters": float(sol["iters"][ok].mean()), "loss_history": hist}
    return w.cpu().numpy(), info


def evaluate(weights, n_states=100_000, nv=32, seed=99, umax_choices=(6.0, 10.0, 14.0)):
    """Newton from the cold start and from the learned start on held-out
    states: mean linear solves and sum passes, both overall and on the states
    the cold start needs >= 5 solves for, fallbacks, largest final residual
    and the largest difference of the converged unknowns."""
    st = W_sample(n_states, seed, umax_choices, nv)
    a = solve_targets(st, nv=nv, guess=frdvm.GUESS_COLD)
    b = solve_targets(st, nv=nv, guess=frdvm.GUESS_MLP, weights=weights)
    ok = (a["status"] == frdvm.NEWTON_OK) & (b["status"] == frdvm.NEWTON_OK)
    hard = ok & (a["iters"] >= 5)
    return {"n_states": int(n_states), "both_converged": int(ok.sum()),
            "cold_solves": float(a["iters"][ok].mean()), "learned_solves": float(b["iters"][ok].mean()),
            "cold_passes": float(a["evals"][ok].mean()), "learned_passes": float(b["evals"][ok].mean()),
            "hard_states": int(hard.sum()), "cold_solves_hard": float(a["iters"][hard].mean()),
            "learned_solves_hard": float(b["iters"][hard].mean()),
            "fallback_cold": int((a["status"] == frdvm.NEWTON_FALLBACK).sum()),
            "fallback_learned": int((b["status"] == frdvm.NEWTON_FALLBACK).sum()),
            "max_resid_cold": float(a["resid"][ok].max()), "max_resid_learned": float(b["resid"][ok].max()),
            "max_dz_between_roots": float(np.abs(a["z"][ok] - b["z"][ok]).max())}


def W_sample(n, seed, umax_choices, nv):
    import workloads as W
    return W.sample_states(n, seed=seed, umax_choices=umax_choices, nv=nv)


if __name__ == "__main__":
    # Learned-start study on the 32^3 grids with u_max in {6, 10, 14}: train on
    # solver-solved states, evaluate on held-out ones; prints one JSON line.
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=1_000_000)
    ap.add_argument("--test", type=int, default=200_000)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--hidden", type=int, default=64)
    args = ap.parse_args()
    t0 = time.perf_counter()
    w, info = fit_guess(n_states=args.train, H=args.hidden, steps=args.steps, seed=4, verbose=True)
    t1 = time.perf_counter()
    print(f"[learned] trained in {t1 - t0:.1f} s; evaluating on {args.test} held-out states", file=sys.stderr,
          flush=True)
    ev = evaluate(w, n_states=args.test)
    out = {"train_states": args.train, "train_steps": args.steps, "hidden": args.hidden,
           "train_seconds": t1 - t0, "final_loss": info["loss_history"][-1][1] if info["loss_history"] else None,
           "reject_rate": info["reject_rate"], **ev}
    print(json.dumps(out), flush=True)
