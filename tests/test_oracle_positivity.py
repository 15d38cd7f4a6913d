"""Pins of the oracle's positivity limiter (the scheme the paper builds on,
Section "Numerical method", is a positivity-preserving and conservative FR
method; the limiter scales each element's polynomial of each velocity node
about its element mean, after Zhang and Shu).

* a linear state in one element: the limited values follow in closed form;
* a state whose element polynomials are positive at the solution and face
  points is left unchanged, to the last bit;
* on curved elements (Jacobian varying inside each element) the limiter
  keeps every element integral (Gauss weights x |J|, computed here from
  numpy's Gauss rule) and makes the polynomial nonnegative at the solution
  points and at the face points (traces evaluated here with numpy's Lagrange
  basis), and the change is a pure scaling about the mean;
* the impulsive Mach-8 start against the diffuse wall: without the limiter f
  turns negative and the conservative-equilibrium Newton fails at the wall;
  with it, f stays nonnegative and every solve converges.
"""
import math

import numpy as np
import pytest

import workloads as W

FREE = {"model": 2, "mu_ref": 1.0}


def _one_node(u=(0.3, 0.2, 0.1)):
    return {"n": (1, 1, 1), "umin": tuple(u), "umax": tuple(u)}


@pytest.mark.parametrize("b", [-3.0, 3.0])
def test_linear_state_closed_form(orc, b):
    """f = 1 + b xi_x on one p = 1 element: mean 1, smallest value 1 - |b| at
    a face, so theta = 1/|b| and the limited polynomial is 1 + sign(b) xi_x,
    zero on one face."""
    mesh = W.box_mesh(1)
    P = orc.Problem(mesh, 1, _one_node(), FREE)
    xi = np.polynomial.legendre.leggauss(2)[0]
    f = np.array([1.0 + b * xi[s % 2] for s in range(8)]).reshape(1, 8, 1)
    got = P.positivity(f)
    ref = np.array([1.0 + math.copysign(1.0, b) * xi[s % 2] for s in range(8)]).reshape(1, 8, 1)
    assert np.allclose(got, ref, rtol=0, atol=1e-15)


def test_nonnegative_state_unchanged(orc):
    """f = M(u) (1 + 0.3 s(x)) with s linear in x and |s| <= 1 on the box:
    every element polynomial is the same linear function, at least 0.7 M > 0
    at the solution and face points, so the limiter changes no bit.  (A
    sampled Maxwellian field is not such a state: in the far tails its
    element polynomials dip below zero between and beyond the nodes.)"""
    mesh = W.box_mesh((2, 1, 2))
    grid = W.grid_spec(6, 4.0)
    P = orc.Problem(mesh, 2, grid, dict(FREE, positivity=1))
    xs = W.box_solution_points(mesh, 2)
    s = (2.0 * xs[..., 0] - 1.0) * 0.5 + (2.0 * xs[..., 2] - 1.0) * 0.5
    prim = np.tile([1.0, 0.3, -0.2, 0.1, 0.9], xs.shape[:2] + (1,))
    f = W.maxwellian(prim, grid).numpy() * (1.0 + 0.3 * s)[..., None]
    assert np.array_equal(P.positivity(f), f)


def _lagrange(x, nodes):
    return np.array([np.prod([(x - nodes[o]) / (nodes[m] - nodes[o]) for o in range(len(nodes)) if o != m])
                     for m in range(len(nodes))])


@pytest.mark.parametrize("p", [1, 2, 3])
def test_curved_elements_keep_integrals_and_reach_nonnegative(orc, p):
    mesh = W.quadratic_map_mesh((2, 1, 2), eps=0.2)
    grid = W.grid_spec((3, 2, 2), 2.0)
    P = orc.Problem(mesh, p, grid, FREE)
    rng = np.random.default_rng(11)
    f = rng.uniform(-0.5, 1.0, size=P.shape)
    f[0, :, 0] = rng.uniform(-1.0, -0.1, size=P.ns)  # an element value with a negative mean
    g = P.positivity(f)
    n = p + 1
    xi, wq = np.polynomial.legendre.leggauss(n)
    W3 = np.einsum("i,j,l->lji", wq, wq, wq).reshape(-1) * P.geo["detJ"]  # [e][s], s = i + n (j + n l)
    integ = np.einsum("es,esk->ek", W3, f)
    assert np.allclose(np.einsum("es,esk->ek", W3, g), integ, rtol=0, atol=1e-14 * np.abs(f).max() * W3.sum())
    # values at the faces: the element polynomial at xi_d = -1 / +1 on every line
    lam = [_lagrange(-1.0, xi), _lagrange(1.0, xi)]
    g4 = g.reshape(P.ne, n, n, n, -1)  # [e][l][j][i][k]
    faces = [np.einsum("m,ezyxk->ezyk", lam[s], g4) for s in (0, 1)] + \
            [np.einsum("m,ezxyk->ezyk", lam[s], g4.transpose(0, 1, 3, 2, 4)) for s in (0, 1)] + \
            [np.einsum("m,exyzk->exyk", lam[s], g4.transpose(0, 3, 2, 1, 4)) for s in (0, 1)]
    mean = integ / W3.sum(1)[:, None]
    pos = mean > 0
    tol = 1e-14 * np.abs(f).max()
    assert (g.min(1)[pos] >= -tol).all()
    for fc in faces:
        assert (fc.reshape(P.ne, -1, f.shape[-1]).min(1)[pos] >= -tol).all()
    # a scaling about the mean: g - mean = theta (f - mean), 0 <= theta <= 1
    d0, d1 = f - mean[:, None, :], g - mean[:, None, :]
    th = (d0 * d1).sum(1) / np.maximum((d0 * d0).sum(1), 1e-300)
    assert np.allclose(d1, th[:, None, :] * d0, rtol=0, atol=1e-13)
    assert (th >= -1e-15).all() and (th <= 1 + 1e-15).all()
    assert abs(th[0, 0]) < 1e-15  # negative mean: the element value becomes its mean


def test_impulsive_wall_start_stays_realizable(orc):
    """The Mach-8 O-grid configuration (24^3 velocities on [-14, 14]^3,
    ES-BGK Pr 2/3, wall at theta_w = 2) on a small O-grid, started
    impulsively from the seeded farfield state; three SSP-RK3 steps."""
    w = W.workload("cyl48x24x2_p2_v24_es")
    mesh = W.cylinder_mesh(n_theta=8, n_r=2, n_z=1, r1=1.5)
    par = W.physics_params(w)
    finf = W.maxwellian(np.array(par["farfield"]), w["grid"]).numpy()
    out = {}
    for pos in (0, 1):
        P = orc.Problem(mesh, 2, w["grid"], dict(par, f_inf=finf, positivity=pos))
        rng = np.random.default_rng(31)
        prim = np.tile(par["farfield"], (P.ne, P.ns, 1))
        prim[..., 0] *= 1.0 + 0.01 * rng.uniform(-1.0, 1.0, (P.ne, P.ns))
        f = P.rk_step(W.maxwellian(prim, w["grid"]).numpy(), P.dt(0.2), scheme=0, nsteps=3)
        st = P.collide(f)[3]
        out[pos] = (f.min() / f.max(), np.bincount(st.ravel(), minlength=4))
    assert out[0][0] < -1e-3 and out[0][1][1:].sum() > 0  # unlimited: negative f, failed solves
    assert out[1][0] > -1e-14 and out[1][1][1:].sum() == 0  # limited: f >= 0, every solve converges
