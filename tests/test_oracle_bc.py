"""Pins of the oracle on general hexahedral meshes: curved (27-node)
elements, element frames that differ across a face, and the two boundary
conditions of the paper's external flows plus its symmetry plane (Section
"Implementation & problem setup": the farfield exterior is the freestream
Maxwellian; the wall is diffuse and isothermal, its exterior a wall
Maxwellian whose density makes the net mass flux through the wall vanish;
the symmetry plane reflects specularly)."""
import math

import numpy as np
import pytest

import workloads as W

FREE = {"model": 2, "prandtl": 1.0, "mu_ref": 1.0}


def _ws(p):
    _, wq = np.polynomial.legendre.leggauss(p + 1)
    return np.einsum("i,j,k->kji", wq, wq, wq).reshape(-1)


def _walls(mesh, tag):
    m = dict(mesh)
    m["bc"] = np.where(mesh["nbr_elem"] < 0, tag, 0).astype(np.int8)
    return m


def _noisy(P, grid, seed, amp=0.3):
    xs = P.geo["xs"]
    prim = W.prim_random_modes(xs, seed=seed, U_amp=0.3)
    f = W.maxwellian(prim, grid).numpy()
    rng = np.random.default_rng(seed)
    return f * (1.0 + amp * rng.uniform(-1, 1, size=f.shape))


@pytest.mark.parametrize("p", [1, 2])
def test_reoriented_elements_give_the_same_residual(orc, p):
    """Giving every element its own local frame (axes permuted and reversed,
    faces met under all eight orientation codes) only relabels points: the
    residual, mapped back, is unchanged."""
    mesh = W.box_mesh((3, 3, 2), length=(1.0, 0.9, 0.7))
    grid = W.grid_spec((4, 3, 5), 3.0)
    P0 = orc.Problem(mesh, p, grid, FREE)
    f0 = _noisy(P0, grid, 2)
    R0 = P0.residual(f0)
    rmesh, frames = W.reorient_elements(mesh, seed=3)
    assert len(set(rmesh["nbr_orient"].reshape(-1).tolist())) >= 6
    P1 = orc.Problem(rmesh, p, grid, FREE)
    R1 = P1.residual(W.reindex_points(f0, frames, p, to_new=True))
    back = W.reindex_points(R1, frames, p, to_new=False)
    assert np.abs(back - R0).max() < 1e-12 * np.abs(R0).max()


def test_wall_maxwellian_at_rest_is_steady(orc):
    """A box closed by walls at theta_w holding the wall Maxwellian at rest
    (any density) is steady: on a symmetric grid the wall density equals the
    interior density."""
    tw = 1.4
    mesh = _walls(W.box_mesh((2, 2, 2), periodic=False), 2)
    grid = W.grid_spec(6, 5.0)
    P = orc.Problem(mesh, 2, grid, {**FREE, "theta_wall": tw})
    f = W.maxwellian(np.array([[[1.7, 0.0, 0.0, 0.0, tw]]]), grid).numpy()
    f = np.broadcast_to(f, P.shape)
    R = P.residual(f)
    assert np.abs(R).max() < 1e-13 * f.max() * 10


def test_closed_wall_box_conserves_mass(orc):
    """With walls on every side no mass leaves: the integral of the mass
    moment of R vanishes for any state, while the energy flux through a wall
    hotter than the gas does not."""
    mesh = _walls(W.box_mesh((2, 3, 2), periodic=False, length=(1.0, 1.2, 0.8)), 2)
    grid = W.grid_spec(7, 6.0)
    P = orc.Problem(mesh, 2, grid, {**FREE, "theta_wall": 2.0})
    f = _noisy(P, grid, 4)
    R = P.residual(f)
    tot = P.totals(R)
    scale = P.totals(np.abs(R))
    assert abs(tot[0]) < 1e-13 * scale[0]
    assert tot[4] > 1e-3 * scale[4]


@pytest.mark.parametrize("p", [2, 3])
def test_farfield_free_stream_on_curved_elements(orc, p):
    """A uniform drifting Maxwellian equal to the farfield state stays
    uniform on curved elements: the quadratic map's metric terms are
    polynomials of degree <= 2 per direction, exact for p >= 2."""
    mesh = W.quadratic_map_mesh(2, eps=0.15, bc_all=1)
    grid = W.grid_spec(5, 4.0)
    finf = W.maxwellian(np.array([1.1, 0.5, -0.3, 0.2, 0.9]), grid).numpy()
    P = orc.Problem(mesh, p, grid, {**FREE, "f_inf": finf})
    R = P.residual(np.broadcast_to(finf, P.shape))
    assert np.abs(R).max() < 1e-11 * finf.max()


@pytest.mark.parametrize("p", [1, 2])
def test_quadratic_map_volume_and_normals(orc, p):
    """x -> x + eps (y^2, z^2, x^2) has det = 1 + 8 eps^3 x y z, so the
    volume of the image of the unit cube is 1 + eps^3; and the outward
    area-scaled normals satisfy the divergence theorem for F = x,
    sum over boundary points of x . n dA = 3 V."""
    eps = 0.2
    mesh = W.quadratic_map_mesh((2, 2, 3), eps=eps)
    P = orc.Problem(mesh, p, W.grid_spec(1, 0.0), FREE)
    V = float(np.einsum("s,es->", _ws(p), P.geo["detJ"]))
    assert abs(V - (1.0 + eps ** 3)) < 1e-13
    xi, wq = np.polynomial.legendre.leggauss(p + 1)
    n = p + 1
    N = (2, 2, 3)
    flux = 0.0
    for e in range(mesh["n_elem"]):
        idx = (e % N[0], (e // N[0]) % N[1], e // (N[0] * N[1]))
        for f in range(6):
            if mesh["nbr_elem"][e, f] >= 0:
                continue
            d, side = divmod(f, 2)
            t = [a for a in range(3) if a != d]
            for b in range(n):
                for a in range(n):
                    r = np.zeros(3)
                    r[d] = 1.0 if side else -1.0
                    r[t[0]], r[t[1]] = xi[a], xi[b]
                    x = (np.array(idx) + 0.5 * (r + 1.0)) / np.array(N)
                    X = x + eps * np.array([x[1] ** 2, x[2] ** 2, x[0] ** 2])
                    flux += wq[a] * wq[b] * X @ P.geo["nf"][e, f, a + n * b]
    assert abs(flux - 3.0 * (1.0 + eps ** 3)) < 1e-12


def test_cylinder_mesh_geometry(orc):
    """The O-grid's Jacobians are positive and its volume approaches the
    annulus pi (r1^2 - r0^2) lz (16 quadratic arcs: relative error 5e-5)."""
    m = W.cylinder_mesh(n_theta=16, n_r=4, n_z=1, r1=2.0)
    P = orc.Problem(m, 2, W.grid_spec(1, 0.0), FREE)
    V = float(np.einsum("s,es->", _ws(2), P.geo["detJ"]))
    exact = math.pi * (m["r1"] ** 2 - m["r0"] ** 2) * m["lz"]
    assert (P.geo["detJ"] > 0).all()
    assert abs(V - exact) < 1e-4 * exact


def _specular_half_and_mirror(p, grid):
    """Half box [0,1] x [0,0.8] x [0,0.6] with specular walls at x = 0 and
    x = 1 (periodic in y, z), and the periodic box of twice the length in x
    that holds the mirrored state."""
    half = W.box_mesh((2, 2, 2), length=(1.0, 0.8, 0.6))
    nb = half["nbr_elem"].copy()
    bc = half["bc"].copy()
    for e in range(half["n_elem"]):
        ix = e % 2
        if ix == 0:
            nb[e, 0], bc[e, 0] = -1, 3
        if ix == 1:
            nb[e, 1], bc[e, 1] = -1, 3
    half = dict(half, nbr_elem=nb, bc=bc)
    full = W.box_mesh((4, 2, 2), length=(2.0, 0.8, 0.6))
    return half, full


def _mirror_state(fh, p, grid):
    """f on the doubled box: elements ix = 0, 1 hold fh, ix = 2, 3 the image
    under x -> 2 - x, u_x -> -u_x."""
    n = p + 1
    nx = grid["n"][0]
    ne_h, ns, nu = fh.shape
    ff = np.zeros((2 * ne_h, ns, nu))
    fr = fh.reshape(ne_h, n, n, n, -1, nx)  # [e][l][j][i][k_yz][k_x]
    mir = fr[:, :, :, ::-1, :, ::-1].reshape(ne_h, ns, nu)
    for e in range(ne_h):
        ix, rest = e % 2, e // 2
        ff[0 + 4 * rest + ix] = fh[e]
        ff[3 - ix + 4 * rest] = mir[e]
    return ff


@pytest.mark.parametrize("p", [1, 2])
def test_specular_wall_is_a_mirror_plane(orc, p):
    """Specular walls at x = 0 and x = 1 give the residual of the periodic
    box of twice the length holding the mirrored state, restricted to the
    original half."""
    grid = W.grid_spec((6, 3, 4), 4.0)
    half, full = _specular_half_and_mirror(p, grid)
    Ph = orc.Problem(half, p, grid, FREE)
    fh = _noisy(Ph, grid, 9)
    Pf = orc.Problem(full, p, grid, FREE)
    Rf = Pf.residual(_mirror_state(fh, p, grid))
    Rh = Ph.residual(fh)
    keep = [e for e in range(full["n_elem"]) if e % 4 < 2]
    assert np.abs(Rh - Rf[keep]).max() < 1e-12 * np.abs(Rh).max()


def test_specular_box_conserves_mass_and_energy(orc):
    mesh = _walls(W.box_mesh((2, 2, 2), periodic=False, length=(1.0, 1.2, 0.8)), 3)
    grid = W.grid_spec(6, 5.0)
    P = orc.Problem(mesh, 2, grid, FREE)
    R = P.residual(_noisy(P, grid, 10))
    tot, scale = P.totals(R), P.totals(np.abs(R))
    assert abs(tot[0]) < 1e-13 * scale[0] and abs(tot[4]) < 1e-13 * scale[4]


def test_specular_wall_needs_an_axis_plane(orc):
    mesh = W.quadratic_map_mesh(2, eps=0.15, bc_all=3)
    P = orc.Problem(mesh, 2, W.grid_spec(4, 3.0), FREE)
    with pytest.raises(ValueError):
        P.residual(np.ones(P.shape))
