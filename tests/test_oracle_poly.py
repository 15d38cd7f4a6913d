"""Pins of the oracle's reduced distribution pair (F, G) for a gas with
delta internal degrees of freedom (Section "Governing equations": F and G
are advected alike; they relax to g and delta theta / 2 g with the same
tau; rho and rho U come from F, the energy from F and G)."""
import numpy as np
import pytest

import workloads as W

DELTA = 2.0
BGK = {"model": 0, "prandtl": 1.0, "mu_ref": 0.05, "newton_tol": 1e-13, "newton_max_iter": 50, "delta": DELTA}
ES = dict(BGK, model=1, prandtl=0.71)
FREE = {"model": 2, "prandtl": 1.0, "mu_ref": 1.0, "delta": DELTA}


def _pair(F, th_t, th_i, delta=DELTA):
    """G = delta theta_i / 2 F (internal energy at temperature theta_i)."""
    return np.concatenate([F, 0.5 * delta * th_i * F], -1)


def test_both_components_are_advected_alike(orc):
    mesh = W.box_mesh((3, 2, 2), length=(1.0, 0.8, 0.6))
    grid = W.grid_spec((5, 4, 3), 3.0)
    P2 = orc.Problem(mesh, 2, grid, FREE)
    P1 = orc.Problem(mesh, 2, grid, dict(FREE, delta=0.0))
    F = np.random.default_rng(0).uniform(0.5, 1.5, size=P1.shape)
    G = np.random.default_rng(1).uniform(0.5, 1.5, size=P1.shape)
    R = P2.residual(np.concatenate([F, G], -1))
    assert np.abs(R[..., :P1.nu] - P1.residual(F)).max() < 1e-14 * np.abs(R).max()
    assert np.abs(R[..., P1.nu:] - P1.residual(G)).max() < 1e-14 * np.abs(R).max()


@pytest.mark.parametrize("par", [BGK, ES], ids=["bgk", "es"])
def test_collision_conserves_total_energy(orc, par):
    grid = W.grid_spec(9, 6.0)
    P = orc.Problem.points_only(grid, par)
    xs = np.random.default_rng(2).uniform(0, 1, size=(6, 3))
    prim = W.prim_random_modes(xs, seed=3, U_amp=0.4)
    F = W.maxwellian(prim, grid).numpy() * (1 + 0.3 * np.random.default_rng(4).uniform(-1, 1, size=(6, P.nu)))
    f = _pair(F, 1.0, 0.6) * (1 + 0.2 * np.random.default_rng(5).uniform(-1, 1, size=(6, 2 * P.nu)))
    S, prim_eq, _, st, _ = P.collide(f)
    assert np.all(st == 0)
    u, w = P.u, P.w
    SF, SG = S[:, :P.nu], S[:, P.nu:]
    mom = np.stack([SF @ w, (SF * w) @ u[:, 0], (SF * w) @ u[:, 1], (SF * w) @ u[:, 2],
                    (SF * w) @ (0.5 * (u ** 2).sum(1)) + SG @ w], -1)
    scale = np.abs(S).max() * w.sum() * 20
    assert np.abs(mom).max() < 1e-13 * scale


@pytest.mark.parametrize("th_t,th_i", [(1.2, 0.6), (0.8, 1.1)])
def test_relaxation_temperature_closed_form(orc, th_t, th_i):
    """F a Maxwellian at theta_t and internal energy at theta_i: the total
    energy is rho (|U|^2/2 + 3/2 theta_t + delta/2 theta_i) and the
    equilibrium temperature (3 theta_t + delta theta_i)/(3 + delta); energy
    flows from the hotter mode into the colder."""
    grid = W.grid_spec(40, 12.0)  # trapezoid error far below the tolerances
    P = orc.Problem.points_only(grid, BGK)
    prim = np.array([[1.3, 0.4, -0.2, 0.1, th_t]])
    f = _pair(W.maxwellian(prim, grid).numpy(), th_t, th_i)
    Q = P.moments(f.reshape(1, 1, -1))[0, 0]
    rho, U = 1.3, np.array([0.4, -0.2, 0.1])
    assert Q[4] == pytest.approx(rho * (0.5 * U @ U + 1.5 * th_t + 0.5 * DELTA * th_i), rel=1e-11)
    S, prim_eq, *_ = P.collide(f)
    th = (3 * th_t + DELTA * th_i) / (3 + DELTA)
    assert prim_eq[0, 4] == pytest.approx(th, rel=1e-10)
    gain = S[0, P.nu:] @ P.w
    assert (gain > 0) == (th_i < th_t)


def test_equilibrium_pair_is_steady(orc):
    grid = W.grid_spec(40, 12.0)
    P = orc.Problem.points_only(grid, ES)
    prim = np.array([[0.9, -0.3, 0.2, 0.5, 1.4]])
    F = W.maxwellian(prim, grid).numpy()
    f = _pair(F, 1.4, 1.4)
    S, *_ = P.collide(f)
    assert np.abs(S).max() < 1e-9 * np.abs(f).max() / BGK["mu_ref"]


def test_pair_wall_and_farfield(orc):
    """Walled box holding the wall pair at rest is steady and, for any
    state, keeps its mass; a uniform farfield pair is steady on curved
    elements."""
    tw = 1.3
    mesh = W.box_mesh((2, 2, 2), periodic=False)
    mesh = dict(mesh, bc=np.where(mesh["nbr_elem"] < 0, 2, 0).astype(np.int8))
    grid = W.grid_spec(8, 6.0)
    P = orc.Problem(mesh, 2, grid, dict(FREE, theta_wall=tw))
    Mw = W.maxwellian(np.array([0.7, 0.0, 0.0, 0.0, tw]), grid).numpy()
    f = np.broadcast_to(_pair(Mw, tw, tw), P.shape)
    assert np.abs(P.residual(f)).max() < 1e-12 * f.max() * 100
    g = f * (1 + 0.3 * np.random.default_rng(7).uniform(-1, 1, size=P.shape))
    tot, scale = P.totals(P.residual(g)), P.totals(np.abs(P.residual(g)))
    assert abs(tot[0]) < 1e-13 * scale[0]
    qm = W.quadratic_map_mesh(2, eps=0.15, bc_all=1)
    finf = _pair(W.maxwellian(np.array([1.1, 0.5, -0.3, 0.2, 0.9]), grid).numpy(), 0.9, 0.9)
    Pq = orc.Problem(qm, 2, grid, dict(FREE, f_inf=finf))
    assert np.abs(Pq.residual(np.broadcast_to(finf, Pq.shape))).max() < 1e-11 * finf.max()
