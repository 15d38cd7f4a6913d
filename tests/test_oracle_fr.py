"""Pins of the oracle's flux-reconstruction residual and time stepping.

Section "Numerical method": each velocity node is advected independently by
an FR scheme (element-wise degree-p polynomial at solution nodes, corrected
flux with correction functions h_i that recover nodal DG, upwind common
interface flux).  The scheme is conservative, exact on polynomials, reduces to
first-order upwind finite volumes at p = 0 and converges at order p+1.  The
paper integrates explicitly in time; the three-stage schemes used here are
third order, so one step applies 1 + z + z^2/2 + z^3/6 on a linear problem.
"""
import numpy as np
import pytest

import workloads as W

FREE = {"model": 2, "prandtl": 1.0, "mu_ref": 1.0}
BGK = {"model": 0, "prandtl": 1.0, "mu_ref": 0.04, "omega": 0.81, "newton_tol": 1e-13,
       "newton_max_iter": 50}


def one_velocity(u):
    return {"n": (1, 1, 1), "umin": tuple(u), "umax": tuple(u)}


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8])
def test_gauss_legendre_matches_numpy(orc, n):
    xi, w = orc.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(xi, xr, atol=1e-15) and np.allclose(w, wr, atol=1e-15)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_operators_exact_on_polynomials(orc, p):
    o = orc.fr_ops(p)
    xi = o["xi"]
    for q in range(p + 1):
        assert np.allclose(o["D"] @ xi ** q, q * xi ** max(q - 1, 0) if q else 0 * xi, atol=1e-12)
        assert o["lamL"] @ xi ** q == pytest.approx((-1.0) ** q, abs=1e-13)
        assert o["lamR"] @ xi ** q == pytest.approx(1.0, abs=1e-13)


@pytest.mark.parametrize("p", [0, 1, 2, 3, 4])
def test_correction_recovers_nodal_dg(orc, p):
    """With Gauss points the DG mass matrix is diag(w) and the DG lifting of a
    face jump is M^-1 l(+-1); FR recovers DG iff the correction derivatives
    at the solution points equal that lifting.  l_j(+-1) is evaluated here
    with numpy's polynomial fit, independently of the oracle."""
    o = orc.fr_ops(p)
    xi, w = np.polynomial.legendre.leggauss(p + 1)
    lR = np.array([np.polyval(np.polyfit(xi, np.eye(p + 1)[j], p), 1.0) for j in range(p + 1)])
    lL = np.array([np.polyval(np.polyfit(xi, np.eye(p + 1)[j], p), -1.0) for j in range(p + 1)])
    assert np.allclose(o["cP"], lR / w, atol=1e-11)
    assert np.allclose(o["cM"], lL / w, atol=1e-11)


def test_p0_is_first_order_upwind_finite_volume(orc):
    N = 6
    mesh = W.box_mesh((N, 1, 1), length=(1.0, 0.5, 0.25))
    for a in (1.3, -0.7):
        P = orc.Problem(mesh, 0, one_velocity((a, 0.0, 0.0)), FREE)
        rng = np.random.default_rng(0)
        f = rng.uniform(size=(N, 1, 1))
        R = P.residual(f)[:, 0, 0]
        fe = f[:, 0, 0]
        h = 1.0 / N
        ref = -a * (fe - np.roll(fe, 1)) / h if a > 0 else -a * (np.roll(fe, -1) - fe) / h
        assert np.allclose(R, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_uniform_state_and_conservation(orc, p):
    """A uniform state has zero residual, and sum_e sum_s w_s |J| R = 0 per
    velocity on a periodic box (FR-DG conservation)."""
    mesh = W.box_mesh((3, 2, 2), length=(1.0, 0.8, 0.6))
    grid = W.grid_spec(4, 3.0)
    P = orc.Problem(mesh, p, grid, FREE)
    R0 = P.residual(np.full(P.shape, 0.7))
    assert np.abs(R0).max() < 1e-12
    rng = np.random.default_rng(1)
    f = rng.uniform(size=P.shape)
    R = P.residual(f)
    _, wq = np.polynomial.legendre.leggauss(p + 1)
    ws = np.einsum("i,j,k->kji", wq, wq, wq).reshape(-1)
    tot = np.einsum("s,es,esk->k", ws, P.geo["detJ"], R)
    assert np.abs(tot).max() < 1e-12 * np.abs(R).max()


def _distorted_box(N, amp, seed=0):
    """Periodic box whose interior nodes are displaced (trilinear, non-affine
    elements); boundary nodes move consistently with their periodic images."""
    mesh = W.box_mesh(N)
    rng = np.random.default_rng(seed)
    nodes = mesh["nodes"].copy()
    n1 = N + 1
    disp = rng.uniform(-amp, amp, size=(N, N, N, 3)) / N
    for k in range(n1):
        for j in range(n1):
            for i in range(n1):
                nodes[i + n1 * (j + n1 * k)] += disp[i % N, j % N, k % N]
    mesh["nodes"] = nodes
    return mesh


@pytest.mark.parametrize("p", [2, 3])
def test_free_stream_preservation_on_distorted_mesh(orc, p):
    """On trilinear (non-affine) elements the pointwise metrics are exact
    polynomials of degree <= 2 per direction, so for p >= 2 a uniform state
    stays uniform."""
    mesh = _distorted_box(3, 0.2)
    P = orc.Problem(mesh, p, W.grid_spec(3, 2.0), FREE)
    R = P.residual(np.full(P.shape, 1.3))
    assert np.abs(R).max() < 1e-11


def _advect_error(orc, N, p, cfl, T, u=(1.0, 0.5, 0.25)):
    u = np.array(u)
    mesh = W.box_mesh(N)
    P = orc.Problem(mesh, p, one_velocity(u), FREE)
    xs = P.geo["xs"]
    f0 = np.sin(2 * np.pi * (xs[..., 0] + xs[..., 1] + xs[..., 2]))[..., None]
    dt0 = P.dt(cfl)
    nst = int(np.ceil(T / dt0))
    dt = T / nst
    f = P.rk_step(f0, dt, scheme=0, nsteps=nst)
    ex = np.sin(2 * np.pi * ((xs - u * T) @ np.ones(3)))[..., None]
    _, wq = np.polynomial.legendre.leggauss(p + 1)
    ws = np.einsum("i,j,k->kji", wq, wq, wq).reshape(-1)
    return np.sqrt(np.einsum("s,es,es->", ws, P.geo["detJ"], (f - ex)[..., 0] ** 2))


@pytest.mark.parametrize("p,cfl,minrate", [(1, 0.2, 1.7), (2, 0.1, 2.8), (3, 0.03, 3.8)])
def test_single_velocity_advection_order(orc, p, cfl, minrate):
    """Pure advection of sin(2 pi (x+y+z)) on a periodic box, compared with the
    exact translate: the L2 error falls at order p+1."""
    for u in ((1.0, 0.5, 0.25), (-0.5, 0.75, -1.0)):
        e1 = _advect_error(orc, 6, p, cfl, 0.1, u)
        e2 = _advect_error(orc, 12, p, cfl, 0.1, u)
        rate = np.log2(e1 / e2)
        assert rate > minrate, (u, e1, e2, rate)


@pytest.mark.parametrize("scheme", [0, 1])
def test_rk_step_is_third_order_polynomial_on_linear_problem(orc, scheme):
    """Collisionless transport is linear, L(f) = A f, and both three-stage
    schemes advance it by 1 + dt A + dt^2 A^2/2 + dt^3 A^3/6."""
    mesh = W.box_mesh((2, 2, 2))
    P = orc.Problem(mesh, 2, W.grid_spec(3, 2.0), FREE)
    rng = np.random.default_rng(3)
    f0 = rng.uniform(size=P.shape)
    dt = 0.01
    A1 = P.residual(f0)
    A2 = P.residual(A1)
    A3 = P.residual(A2)
    ref = f0 + dt * A1 + dt ** 2 / 2 * A2 + dt ** 3 / 6 * A3
    f1 = P.rk_step(f0, dt, scheme=scheme)
    assert np.abs(f1 - ref).max() < 1e-13 * np.abs(f0).max()


def test_dt_rule_on_box(orc):
    mesh = W.box_mesh(4)
    P = orc.Problem(mesh, 1, W.grid_spec(8, 6.0), FREE)
    assert P.dt(0.2) == pytest.approx(0.2 * 0.25 / (3 * 18.0), rel=1e-14)


@pytest.mark.parametrize("scheme", [0, 1])
def test_full_step_conserves_totals(orc, scheme):
    """Advection (FR-DG on a periodic box) and the conservative collision both
    conserve mass, momentum and energy: the global totals are unchanged by a
    full BGK step to 1e-12 relative."""
    w = W.workload("box4_p1_v8")
    mesh = W.box_mesh(2)
    grid = W.grid_spec(6, 5.0)
    P = orc.Problem(mesh, 1, grid, dict(BGK))
    prim = W.prim_random_modes(P.geo["xs"], seed=w["seed"])
    f = W.maxwellian(prim, grid).numpy()
    t0 = P.totals(f)
    f1 = P.rk_step(f, P.dt(0.2), scheme=scheme, nsteps=2)
    t1 = P.totals(f1)
    scale = np.abs(t0).max()
    assert np.abs(t1 - t0).max() < 1e-12 * scale
    assert np.abs(f1 - f).max() > 1e-6  # something happened
