"""Pins of the oracle's velocity grid, moments and pressure tensor against
closed forms, a library quadrature and exact rational arithmetic.

Section "Governing equations", eq. (moments): Q = [rho, rho U, E] are the
moments of f against psi = (1, u, |u|^2/2) (monatomic).  Section "Numerical
method": the velocity integral is the trapezoid rule on a uniform grid.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import trapezoid

import workloads as W


def test_vgrid_nodes_and_weights_match_library_trapezoid(orc):
    n, umin, umax = (5, 4, 3), (-2.0, -1.0, 0.5), (2.0, 3.0, 1.5)
    u, w = orc.vgrid(n, umin, umax)
    ax = [np.linspace(umin[d], umax[d], n[d]) for d in range(3)]
    # node ordering k = i + n0 (j + n1 l): x fastest
    k = 1 + 5 * (2 + 4 * 1)
    assert np.allclose(u[k], [ax[0][1], ax[1][2], ax[2][1]], atol=0, rtol=0)
    # the weights integrate any grid function exactly like scipy's trapezoid rule
    rng = np.random.default_rng(0)
    g = rng.standard_normal((n[2], n[1], n[0]))
    ref = trapezoid(trapezoid(trapezoid(g, ax[0], axis=2), ax[1], axis=1), ax[2], axis=0)
    assert abs(np.dot(w, g.reshape(-1)) - ref) < 1e-13
    assert np.all(w > 0)


@pytest.mark.parametrize("U,theta,rho", [((0.3, -0.2, 0.1), 1.0, 1.3), ((1.5, 0.0, -0.7), 0.5, 0.4)])
def test_moments_of_maxwellian_match_closed_form(orc, U, theta, rho):
    """On a fine grid the trapezoid rule is spectrally accurate for a Gaussian,
    so the discrete moments reach the continuous ones: rho, rho U,
    E = rho |U|^2 / 2 + 3/2 rho theta."""
    grid = W.grid_spec(61, 12.0)
    u, w = orc.vgrid(grid["n"], grid["umin"], grid["umax"])
    prim = np.array([[rho, *U, theta]])
    f = W.maxwellian(prim, grid).numpy()
    Q = orc.moments(f, u, w)[0]
    Uv = np.array(U)
    ref = [rho, *(rho * Uv), 0.5 * rho * Uv @ Uv + 1.5 * rho * theta]
    assert np.allclose(Q, ref, rtol=1e-12, atol=1e-12)
    Pi = orc.pressure_tensor(f, u, w)[0]
    assert np.allclose(Pi, [rho * theta] * 3 + [0, 0, 0], atol=1e-12)


def test_moments_brute_force_exact_rationals(orc):
    """Tiny 2x3x2 grid with dyadic rational f: the moments are computed exactly
    with Fractions and must agree to the last bit of the rounded result."""
    n, umin, umax = (2, 3, 2), (-1.0, -2.0, 0.0), (1.0, 2.0, 0.5)
    u, w = orc.vgrid(n, umin, umax)
    rng = np.random.default_rng(3)
    f = rng.integers(1, 64, size=(4, u.shape[0])) / 16.0
    Q = orc.moments(f, u, w)
    for p in range(f.shape[0]):
        acc = [Fraction(0)] * 5
        for k in range(u.shape[0]):
            wf = Fraction(w[k]) * Fraction(f[p, k])
            ux, uy, uz = (Fraction(x) for x in u[k])
            acc[0] += wf
            acc[1] += wf * ux
            acc[2] += wf * uy
            acc[3] += wf * uz
            acc[4] += wf * (ux * ux + uy * uy + uz * uz) / 2
        assert np.array_equal(Q[p], np.array([float(a) for a in acc]))


def test_pressure_tensor_of_anisotropic_gaussian(orc):
    """Pi_ij = int f (u_i - U_i)(u_j - U_j): for a Gaussian with covariance C
    this is rho C (closed form, fine grid)."""
    grid = W.grid_spec(71, 14.0)
    u, w = orc.vgrid(grid["n"], grid["umin"], grid["umax"])
    Cm = np.array([[1.2, 0.3, -0.1], [0.3, 0.8, 0.2], [-0.1, 0.2, 1.0]])
    U = np.array([0.4, -0.3, 0.2])
    rho = 0.9
    d = u - U
    Ci = np.linalg.inv(Cm)
    f = rho / np.sqrt(np.linalg.det(2 * np.pi * Cm)) * np.exp(-0.5 * np.einsum("ki,ij,kj->k", d, Ci, d))
    Pi = orc.pressure_tensor(f[None], u, w)[0]
    ref = rho * np.array([Cm[0, 0], Cm[1, 1], Cm[2, 2], Cm[0, 1], Cm[0, 2], Cm[1, 2]])
    assert np.allclose(Pi, ref, atol=1e-11)


def test_viscosity_laws(orc):
    """Power law mu_ref (theta/theta_ref)^omega and Sutherland's law."""
    assert orc.viscosity(2.0, 0.1, 1.0, 0.81, 0, 0.0) == pytest.approx(0.1 * 2 ** 0.81, rel=1e-15)
    ts = 110.4 / 203
    mu = orc.viscosity(3.0, 0.05, 1.0, 0.0, 1, ts)
    assert mu == pytest.approx(0.05 * 3.0 ** 1.5 * (1 + ts) / (3.0 + ts), rel=1e-15)


def test_knudsen_to_reference_viscosity():
    """lambda = (mu/rho) sqrt(pi/(2 theta)) with lambda = Kn, rho = theta = 1."""
    for kn in (0.05, 1e-3, 2e-4):
        mu = W.mu_ref_from_knudsen(kn)
        assert mu * np.sqrt(np.pi / 2) == pytest.approx(kn, rel=1e-15)


def _uniform_moments(rho, U, theta):
    U = np.asarray(U, float)
    return np.array([rho, *(rho * U), 0.5 * rho * U @ U + 1.5 * rho * theta])


@pytest.mark.parametrize("p,nodes", [(1, 0), (3, 0), (2, 1)])
def test_totals_of_uniform_maxwellian_are_volume_times_moments(orc, p, nodes):
    """Domain totals of a uniform sampled Maxwellian on a box of side lengths
    (0.7, 1.3, 0.9): V (rho, rho U, E) with V = 0.819 and the closed-form
    moments (fine velocity grid: trapezoid aliasing below 1e-20)."""
    mesh = W.box_mesh((1, 2, 1), length=(0.7, 1.3, 0.9))
    grid = W.grid_spec(31, 9.0)
    P = orc.Problem(mesh, p, grid, {"model": 2, "mu_ref": 1.0, "nodes": nodes})
    rho, U, th = 1.3, (0.3, -0.2, 0.1), 0.9
    prim = np.tile([rho, *U, th], (P.ne, P.ns, 1))
    f = W.maxwellian(prim, grid).numpy()
    V = 0.7 * 1.3 * 0.9
    ref = V * _uniform_moments(rho, U, th)
    assert np.allclose(P.totals(f), ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("p", [2, 3])
def test_totals_of_linear_density_on_curved_mesh(orc, p):
    """rho(X) = 1 + a . X on the image of the unit cube under the quadratic
    map X = x + eps (y^2, z^2, x^2), with U and theta uniform: the mass total
    is the integral of rho over the image, computed here by a 12-point Gauss
    rule on the unit cube with the map's Jacobian 1 + 8 eps^3 x y z, and the
    other totals follow from the uniform U and theta."""
    eps = 0.2
    N = (2, 1, 2)
    mesh = W.quadratic_map_mesh(N, eps=eps)
    grid = W.grid_spec(31, 10.0)
    P = orc.Problem(mesh, p, grid, {"model": 2, "mu_ref": 1.0})
    a = np.array([0.3, -0.2, 0.25])
    U, th = np.array([0.2, 0.1, -0.3]), 1.1
    n = p + 1
    xi = np.polynomial.legendre.leggauss(n)[0]
    rho = np.zeros((P.ne, P.ns))
    for e in range(P.ne):
        idx = np.array((e % N[0], (e // N[0]) % N[1], e // (N[0] * N[1])))
        for s in range(P.ns):
            r = np.array([xi[s % n], xi[(s // n) % n], xi[s // (n * n)]])
            x = (idx + 0.5 * (r + 1.0)) / np.array(N)
            X = x + eps * np.array([x[1] ** 2, x[2] ** 2, x[0] ** 2])
            rho[e, s] = 1.0 + a @ X
    prim = np.concatenate([rho[..., None], np.broadcast_to(U, rho.shape + (3,)), np.full(rho.shape + (1,), th)], -1)
    f = W.maxwellian(prim, grid).numpy()
    g, wg = np.polynomial.legendre.leggauss(12)
    g, wg = 0.5 * (g + 1.0), 0.5 * wg
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    wt = wg[:, None, None] * wg[None, :, None] * wg[None, None, :]
    X = np.stack([x + eps * y ** 2, y + eps * z ** 2, z + eps * x ** 2])
    mass = float(np.sum(wt * (1.0 + np.tensordot(a, X, 1)) * (1.0 + 8.0 * eps ** 3 * x * y * z)))
    ref = mass * _uniform_moments(1.0, U, th)
    assert np.allclose(P.totals(f), ref, rtol=1e-13, atol=1e-14)
