"""Pins of the oracle's density gradient-length local Knudsen number
(Section "Results"): zero for a uniform state; for a density linear in x,
which the element polynomials represent exactly on box and on trilinear
(distorted) elements, the closed form lambda |grad rho| / rho with
lambda = mu(theta) / rho sqrt(pi / (2 theta)), mu = mu_ref (theta/theta_ref)^omega."""
import numpy as np
import pytest

import workloads as W

PAR = {"model": 0, "prandtl": 1.0, "mu_ref": 0.02, "theta_ref": 1.0, "omega": 0.81}


def _distorted_box(N, amp, seed=0):
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


def _maxwellian_field(P, grid, grad, rho0=1.0, theta=1.2):
    xs = P.geo["xs"].reshape(P.ne, P.ns, 3)
    prim = np.zeros((P.ne, P.ns, 5))
    prim[..., 0] = rho0 + xs @ np.asarray(grad, dtype=float)
    prim[..., 4] = theta
    return prim, W.maxwellian(prim, grid).numpy()


def test_uniform_state_has_zero_kn(orc):
    mesh = W.box_mesh((2, 2, 2))
    grid = W.grid_spec(12, 7.0)
    P = orc.Problem(mesh, 2, grid, PAR)
    _, f = _maxwellian_field(P, grid, (0.0, 0.0, 0.0))
    assert np.abs(P.kn_gll(f)).max() < 1e-13


@pytest.mark.parametrize("distorted", [False, True])
@pytest.mark.parametrize("p", [1, 3])
def test_linear_density_matches_closed_form(orc, p, distorted):
    mesh = _distorted_box(3, 0.2) if distorted else W.box_mesh((3, 2, 2), length=(1.0, 0.8, 0.6))
    grid = W.grid_spec(24, 10.0)  # trapezoid error of the moments ~1e-14
    P = orc.Problem(mesh, p, grid, PAR)
    grad, theta = np.array([0.3, 0.2, -0.1]), 1.2
    prim, f = _maxwellian_field(P, grid, grad, theta=theta)
    rho = prim[..., 0]
    mu = PAR["mu_ref"] * (theta / PAR["theta_ref"]) ** PAR["omega"]
    ref = mu / rho * np.sqrt(np.pi / (2.0 * theta)) * np.linalg.norm(grad) / rho
    got = P.kn_gll(f)
    assert np.abs(got - ref).max() < 1e-10 * ref.max()


def test_nonrealizable_point_gets_zero(orc):
    mesh = W.box_mesh((2, 2, 2))
    grid = W.grid_spec(8, 6.0)
    P = orc.Problem(mesh, 1, grid, PAR)
    _, f = _maxwellian_field(P, grid, (0.3, 0.0, 0.0))
    f[0, 3] = 0.0
    kn = P.kn_gll(f)
    assert kn[0, 3] == 0.0 and np.all(np.isfinite(kn))
