"""Pins of the oracle with Gauss-Lobatto solution points (the point set the
paper uses on tensor-product elements, Section "Implementation & problem
setup").  The
correction functions are still the DG-recovering ones, so the scheme is
nodal DG with the exact mass matrix on these points."""
import numpy as np
import pytest

import workloads as W

FREE = {"model": 2, "prandtl": 1.0, "mu_ref": 1.0, "nodes": 1}
L = np.polynomial.legendre


@pytest.mark.parametrize("n", [2, 3, 4, 5, 8])
def test_gauss_lobatto_nodes_and_exactness(orc, n):
    """Nodes: +-1 and the roots of P'_{n-1} (numpy); the rule integrates
    x^k exactly for k <= 2n - 3."""
    xi, w = orc.gauss_lobatto(n)
    inner = np.sort(L.Legendre.basis(n - 1).deriv().roots().real)
    assert np.allclose(xi, np.concatenate([[-1.0], inner, [1.0]]), atol=1e-14)
    for k in range(2 * n - 2):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert w @ xi ** k == pytest.approx(exact, abs=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_lobatto_operators_and_dg_lifting(orc, p):
    """D differentiates polynomials of degree p exactly, the traces are the
    end values, and the correction derivatives equal the DG lifting
    M^-1 l(+-1) with the exact mass matrix (not diagonal on these points),
    M from a 2p+2-point Gauss rule and numpy polynomial fits."""
    o = orc.fr_ops(p, nodes=1)
    xi = o["xi"]
    n = p + 1
    for q in range(n):
        assert np.allclose(o["D"] @ xi ** q, q * xi ** max(q - 1, 0) if q else 0 * xi, atol=1e-12)
    assert np.allclose(o["lamL"], np.eye(n)[0], atol=1e-15) and np.allclose(o["lamR"], np.eye(n)[-1], atol=1e-15)
    xg, wg = L.leggauss(2 * n + 2)
    coef = [np.polyfit(xi, np.eye(n)[j], p) for j in range(n)]
    V = np.array([np.polyval(c, xg) for c in coef])
    M = (V * wg) @ V.T
    lR = np.array([np.polyval(c, 1.0) for c in coef])
    lL = np.array([np.polyval(c, -1.0) for c in coef])
    assert np.allclose(o["cP"], np.linalg.solve(M, lR), atol=1e-10)
    assert np.allclose(o["cM"], np.linalg.solve(M, lL), atol=1e-10)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_lobatto_uniform_state_and_conservation(orc, p):
    mesh = W.box_mesh((3, 2, 2), length=(1.0, 0.8, 0.6))
    grid = W.grid_spec(4, 3.0)
    P = orc.Problem(mesh, p, grid, FREE)
    assert np.abs(P.residual(np.full(P.shape, 0.7))).max() < 1e-12
    f = np.random.default_rng(1).uniform(size=P.shape)
    R = P.residual(f)
    _, wq = orc.gauss_lobatto(p + 1)
    ws = np.einsum("i,j,k->kji", wq, wq, wq).reshape(-1)
    tot = np.einsum("s,es,esk->k", ws, P.geo["detJ"], R)
    assert np.abs(tot).max() < 1e-12 * np.abs(R).max()


def test_lobatto_points_on_faces(orc):
    """Gauss-Lobatto elements carry points on their faces: the solution point
    coordinates of a box element include its corners."""
    mesh = W.box_mesh(1)
    P = orc.Problem(mesh, 2, W.grid_spec(1, 0.0), FREE)
    xs = P.geo["xs"][0]
    assert np.allclose(xs[0], [0, 0, 0]) and np.allclose(xs[-1], [1, 1, 1])


@pytest.mark.parametrize("p,cfl,minrate", [(1, 0.2, 1.7), (2, 0.1, 2.8), (3, 0.03, 3.8)])
def test_lobatto_advection_order(orc, p, cfl, minrate):
    u = np.array([1.0, 0.5, 0.25])
    errs = []
    for N in (6, 12):
        mesh = W.box_mesh(N)
        P = orc.Problem(mesh, p, {"n": (1, 1, 1), "umin": tuple(u), "umax": tuple(u)}, FREE)
        xs = P.geo["xs"]
        f0 = np.sin(2 * np.pi * xs.sum(-1))[..., None]
        nst = int(np.ceil(0.1 / P.dt(cfl)))
        f = P.rk_step(f0, 0.1 / nst, scheme=0, nsteps=nst)
        ex = np.sin(2 * np.pi * (xs - u * 0.1).sum(-1))[..., None]
        _, wq = orc.gauss_lobatto(p + 1)
        ws = np.einsum("i,j,k->kji", wq, wq, wq).reshape(-1)
        errs.append(np.sqrt(np.einsum("s,es,es->", ws, P.geo["detJ"], (f - ex)[..., 0] ** 2)))
    assert np.log2(errs[0] / errs[1]) > minrate, errs
