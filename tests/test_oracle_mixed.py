"""Pins of the mixed-mesh oracle (hexahedra, prisms, tetrahedra; Section
"Implementation & problem setup": alpha-optimised points on simplices,
Gauss-Lobatto points on tensor-product elements; Section "Numerical method":
FR with the DG-recovering correction and the upwind flux), against what the
mathematics fixes:

* the point sets are those of the published warp & blend construction
  (p <= 3, with the published alpha values), and that construction puts
  Gauss-Lobatto points on every edge at any order;
* the rational monomial integrals equal an independent Gauss rule;
* the derivative matrices differentiate every polynomial of the element's
  space exactly; the face lifting integrates 1 and x over each face exactly
  (face area, face centroid);
* a uniform state has zero residual, the residual of any state conserves
  the domain integral (periodic mesh), and on an all-hexahedron mesh the
  residual equals the (independently pinned) Gauss-Lobatto FR oracle's;
* the residual of a smooth advected field converges to -u . grad f at
  order p under refinement, and RK steps with the conservative BGK
  collision conserve mass, momentum and energy.
"""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import mixed as M


def _bary(P, dim):
    V = M.REF_VERTS[M.TET][:dim + 1, :dim]
    T = np.stack([V[a] - V[0] for a in range(1, dim + 1)], 1)
    lam = np.linalg.solve(T, (P - V[0]).T).T
    return np.concatenate([1.0 - lam.sum(1, keepdims=True), lam], 1)


def _same_set(A, B, tol=1e-12):
    A = np.array(sorted(map(tuple, np.round(A, 11))))
    B = np.array(sorted(map(tuple, np.round(B, 11))))
    return A.shape == B.shape and np.abs(A - B).max() < tol


@pytest.mark.parametrize("p", [1, 2, 3])
def test_simplex_points_are_the_warp_blend_points(p):
    assert _same_set(_bary(M.simplex_points(p, 2), 2), M.warp_blend_tri(p))
    assert _same_set(_bary(M.simplex_points(p, 3), 3), M.warp_blend_tet(p))
    assert len(M.simplex_points(p, 2)) == (p + 1) * (p + 2) // 2
    assert len(M.simplex_points(p, 3)) == (p + 1) * (p + 2) * (p + 3) // 6


@pytest.mark.parametrize("p", [4, 5, 6])
def test_warp_blend_edges_are_gauss_lobatto_and_sets_symmetric(p):
    gl = M.gauss_lobatto_points(p)
    for lam, dim in ((M.warp_blend_tri(p), 2), (M.warp_blend_tet(p), 3)):
        on_edge = lam[(lam > 1e-12).sum(1) <= 2]
        # the points of the edge between vertices 0 and 1, by their coordinate along it
        e01 = np.sort(on_edge[(on_edge[:, 2:] < 1e-12).all(1)][:, 1])
        assert np.allclose(2.0 * e01 - 1.0, gl, atol=1e-12)
        # invariant under every permutation of the vertices
        for perm in itertools.permutations(range(dim + 1)):
            assert _same_set(lam[:, perm], lam, 1e-10)
    # alpha matters above p = 3: the interior points move
    assert not _same_set(M.warp_blend_tri(4), M.warp_blend_tri(4, 0.0), 1e-6)


def _gauss_integral(etype, a, b, c, n=8):
    g, w = np.polynomial.legendre.leggauss(n)
    tot = 0.0
    for i, j, k in itertools.product(range(n), repeat=3):
        x, y, z = g[i], g[j], g[k]
        if etype == M.HEX:
            r, s, t, jac = x, y, z, 1.0
        elif etype == M.PRISM:  # collapse the square onto the triangle
            r, s, t, jac = x, 0.5 * (1 + y) * (1 - x) - 1, z, 0.5 * (1 - x)
        else:  # collapse the cube onto the tetrahedron
            t = z
            s = 0.5 * (1 + y) * (1 - t) - 1
            r = 0.5 * (1 + x) * (-s - t) - 1
            jac = 0.5 * (1 - t) * 0.5 * (-s - t)
        tot += w[i] * w[j] * w[k] * jac * r ** a * s ** b * t ** c
    return tot


@pytest.mark.parametrize("etype", [M.HEX, M.PRISM, M.TET])
def test_monomial_integrals_against_gauss(etype):
    vol = {M.HEX: 8.0, M.PRISM: 4.0, M.TET: 4.0 / 3.0}[etype]
    assert float(M.mono_integral(etype, 0, 0, 0)) == pytest.approx(vol, rel=1e-15)
    for a, b, c in itertools.product(range(5), repeat=3):
        assert float(M.mono_integral(etype, a, b, c)) == pytest.approx(_gauss_integral(etype, a, b, c), abs=1e-13)


@pytest.mark.parametrize("etype", [M.HEX, M.PRISM, M.TET])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_derivatives_exact_and_lifting_integrates_the_face(etype, p):
    R = M.ref_element(etype, p)
    rng = np.random.default_rng(etype * 10 + p)
    coef = rng.normal(size=len(R.ex))
    x = R.x
    q = sum(cf * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c for cf, (a, b, c) in zip(coef, R.ex))
    for d in range(3):
        dq = np.zeros(len(x))
        for cf, e in zip(coef, R.ex):
            if e[d]:
                e2 = list(e)
                e2[d] -= 1
                dq += cf * e[d] * x[:, 0] ** e2[0] * x[:, 1] ** e2[1] * x[:, 2] ** e2[2]
        assert np.abs(R.D[d] @ q - dq).max() < 1e-12 * (1 + np.abs(dq).max())
    for fc in R.faces:
        verts = M.REF_VERTS[etype][fc["verts"]]
        # the face's integrals of l_j: 1^T M LIFT; their sum is the face area and
        # their first moments the face centroid times the area
        ints = np.ones(R.ns) @ R.M @ fc["lift"]
        area = 0.5 * np.linalg.norm(np.cross(verts[1] - verts[0], verts[2] - verts[0])) if len(verts) == 3 else \
            np.linalg.norm(np.cross(*M._quad_edges(verts)[1:]))
        assert ints.sum() == pytest.approx(area, rel=1e-13)
        assert np.allclose(ints @ x[fc["nodes"]], area * verts.mean(0), atol=1e-13)



@pytest.mark.parametrize("p", [1, 2, 3])
def test_prism_operators_have_the_layer_structure(p):
    """The prism's points are the triangle's points on every Gauss-Lobatto
    layer (point m + nt k) and its space is P_p(triangle) x P_p(line), so its
    Lagrange basis is a product: the in-plane derivatives couple only points
    of one layer, the axial one only points of one column, an end-face point
    lifts onto its own column and a side-face point onto its own layer.  The
    GPU prism kernel skips every other entry; here the oracle's operators,
    formed without that assumption, show them to vanish."""
    R = M.ref_element(M.PRISM, p)
    nl = p + 1
    nt = R.ns // nl
    i, j = np.meshgrid(np.arange(R.ns), np.arange(R.ns), indexing="ij")
    scale = max(np.abs(d).max() for d in R.D)
    assert np.abs(R.D[0][i // nt != j // nt]).max() < 1e-14 * scale
    assert np.abs(R.D[1][i // nt != j // nt]).max() < 1e-14 * scale
    assert np.abs(R.D[2][i % nt != j % nt]).max() < 1e-14 * scale
    for fc in R.faces:
        L, nodes = fc["lift"], fc["nodes"]
        end = len(fc["verts"]) == 3
        for c, node in enumerate(nodes):
            onto = (np.arange(R.ns) % nt == node % nt) if end else (np.arange(R.ns) // nt == node // nt)
            assert np.abs(L[~onto, c]).max() < 1e-14 * np.abs(L).max()
            assert np.abs(L[onto, c]).max() > 1e-3 * np.abs(L).max()

def _params():
    return {"model": 0, "mu_ref": 0.05, "prandtl": 1.0, "theta_ref": 1.0, "omega": 0.81}


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mixed_mesh_free_stream_and_conservation(p):
    mesh = W.mixed_box_mesh(3)
    P = M.MixedProblem(mesh, p, W.grid_spec(6, 4.0), _params())
    assert np.bincount(mesh["elem_type"]).tolist() == [20, 12, 6]
    assert np.abs(P.residual(np.ones(P.shape))).max() < 1e-12
    f = np.random.default_rng(p).uniform(0.5, 1.5, P.shape)
    R = P.residual(f)
    tot = (P.point_weights()[:, None] * R).sum(0)
    assert np.abs(tot).max() < 1e-14 * np.abs(R).max()
    assert P.point_weights().sum() == pytest.approx(1.0, rel=1e-13)  # the unit box


@pytest.mark.parametrize("p", [1, 2, 3])
def test_all_hexahedra_equal_the_gauss_lobatto_oracle(p, orc):
    box = W.box_mesh(3)
    hexmesh = dict(box, elem_type=np.zeros(box["n_elem"], np.int8), period=(1.0, 1.0, 1.0))
    grid = W.grid_spec(6, 4.0)
    P = M.MixedProblem(hexmesh, p, grid, _params())
    Q = orc.Problem(box, p, grid, dict(_params(), nodes=1))
    f = np.random.default_rng(7 + p).uniform(0.5, 1.5, P.shape)
    Rm = P.residual(f)
    Rc = Q.residual(f.reshape(Q.shape)).reshape(P.shape)
    assert np.abs(Rm - Rc).max() < 1e-13 * np.abs(Rc).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_residual_converges_to_the_advection_derivative(p):
    u = np.array([[0.7, -0.4, 0.3]])
    k = 2.0 * np.pi * np.array([1.0, 1.0, 1.0])
    errs = []
    for N in (3, 6):
        mesh = W.mixed_box_mesh(N)
        P = M.MixedProblem(mesh, p, W.grid_spec(2, 1.0), _params())
        P.u, P.nu = u, 1
        xs = P.mm.xs
        f = np.sin(xs @ k)[:, None]
        exact = -(u @ k) * np.cos(xs @ k)[:, None]
        errs.append(np.sqrt(np.mean((P.residual(f) - exact) ** 2)))
    order = np.log2(errs[0] / errs[1])
    assert order > p - 0.3, (errs, order)


@pytest.mark.parametrize("scheme", [0, 1])
def test_rk_steps_conserve_with_bgk_collision(scheme):
    mesh = W.mixed_box_mesh(3)
    grid = W.grid_spec(8, 5.0)
    P = M.MixedProblem(mesh, 2, grid, dict(_params(), newton_tol=1e-13, newton_max_iter=50))
    xs = P.mm.xs
    prim = np.stack([1 + 0.1 * np.sin(2 * np.pi * xs[:, 0]), 0.2 * np.cos(2 * np.pi * xs[:, 1]),
                     0.1 * np.sin(2 * np.pi * xs[:, 2]), np.zeros(len(xs)), 1 + 0.05 * np.cos(2 * np.pi * xs[:, 0])], 1)
    f0 = W.maxwellian(prim, grid).numpy()
    t0 = P.totals(f0)
    f = P.rk_step(f0, P.dt(0.2), scheme=scheme, nsteps=2)
    t1 = P.totals(f)
    assert np.abs(t1 - t0).max() < 1e-13 * np.abs(t0).max()
    assert np.abs(f - f0).max() > 1e-4 * np.abs(f0).max()  # it moved


@pytest.mark.parametrize("p", [1, 2, 3])
def test_input_points_follow_the_documented_order(p):
    # the input builder's solution points (its own closed form) are the
    # oracle's, point for point
    mesh = W.mixed_box_mesh(3)
    mm = M.MixedMesh(mesh, p)
    assert np.abs(W.mixed_solution_points(mesh, p) - mm.xs).max() < 1e-14


def test_prism_tetrahedron_box_conserves():
    # the prism / tetrahedron workload mesh: conforming faces, free stream, conservation
    mesh = W.prism_tet_box_mesh(3)
    assert np.bincount(mesh["elem_type"], minlength=3).tolist() == [0, 18, 108]
    P = M.MixedProblem(mesh, 2, W.grid_spec(4, 3.0), _params())
    assert np.abs(P.residual(np.ones(P.shape))).max() < 1e-12
    f = np.random.default_rng(11).uniform(0.5, 1.5, P.shape)
    R = P.residual(f)
    assert np.abs((P.point_weights()[:, None] * R).sum(0)).max() < 1e-14 * np.abs(R).max()
