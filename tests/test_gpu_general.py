"""GPU parity on general hexahedral meshes (curved 27-node elements, element
frames that meet under any orientation code, farfield and diffuse-wall
boundaries) against the FP64 oracle on the same seeded inputs: relative L2
<= 1e-12 in FP64 unless stated.  Velocity grids span two blocks of 256
velocities with a ragged tail."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FAR = [1.0, 1.5, 0.0, 0.0, 1.0]  # rho, U, theta of the farfield
TW = 1.5                          # wall temperature


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_06567_amd import frdvm
    frdvm.lib()
    return frdvm


def _params(model=2, **kw):
    d = {"model": model, "prandtl": 1.0, "mu_ref": 0.05, "theta_ref": 1.0, "omega": 0.81,
         "newton_tol": 1e-13, "newton_max_iter": 50, "farfield": FAR, "theta_wall": TW}
    d.update(kw)
    return d


def _oracle(orc, mesh, p, grid, par):
    finf = W.maxwellian(np.array(par["farfield"]), grid).numpy()
    return orc.Problem(mesh, p, grid, {**par, "f_inf": finf})


def _state(P, grid, seed, amp=0.2):
    prim = W.prim_random_modes(P.geo["xs"], seed=seed, U_amp=0.3)
    f = W.maxwellian(prim, grid).numpy()
    rng = np.random.default_rng(seed)
    return f * (1.0 + amp * rng.uniform(-1, 1, size=f.shape))


def _gpu(s, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=s.dtype).cuda()


def _small_cylinder():
    return W.cylinder_mesh(n_theta=8, n_r=3, n_z=2, r1=2.0)


GRID = W.grid_spec(7, 5.0)  # 343 velocities: two blocks, ragged


def _meshes():
    box = W.box_mesh((3, 3, 2), length=(1.0, 0.9, 0.7))
    reo, _ = W.reorient_elements(box, seed=3)
    return {"reoriented": reo, "quadratic_farfield": W.quadratic_map_mesh(2, eps=0.15, bc_all=1),
            "quadratic_wall": W.quadratic_map_mesh(2, eps=0.15, bc_all=2), "cylinder": _small_cylinder()}


@pytest.mark.parametrize("name,p", [("reoriented", 1), ("reoriented", 2), ("reoriented", 3),
                                    ("quadratic_farfield", 2), ("quadratic_wall", 3), ("cylinder", 2)])
def test_general_residual(F, orc, name, p):
    mesh = _meshes()[name]
    par = _params()
    P = _oracle(orc, mesh, p, GRID, par)
    f = _state(P, GRID, 4)
    s = F.FrDvm(mesh, p, GRID, par)
    R = torch.zeros(s.shape, dtype=s.dtype, device="cuda")
    s.residual(_gpu(s, f), R)
    got, ref = R.cpu().numpy(), P.residual(f)
    bad = ~np.isfinite(got)
    assert not bad.any(), (np.argwhere(bad)[:5], bad.sum())
    assert rel(got, ref) < 1e-12, np.unravel_index(np.abs(got - ref).argmax(), got.shape)


def test_general_moments_totals_dt_kn(F, orc):
    mesh = _small_cylinder()
    par = _params(model=0)
    P = _oracle(orc, mesh, 2, GRID, par)
    f = _state(P, GRID, 5)
    s = F.FrDvm(mesh, 2, GRID, par)
    fg = _gpu(s, f)
    Q = torch.zeros(s.ne * s.ns * 5, dtype=torch.float64, device="cuda")
    tot = s.moments(fg, Q, totals=True)
    assert rel(Q.cpu().numpy().reshape(s.ne, s.ns, 5), P.moments(f)) < 1e-13
    assert rel(tot, P.totals(f)) < 1e-13
    assert s.dt(0.2) == pytest.approx(P.dt(0.2), rel=1e-13)
    kn = torch.zeros(s.ne * s.ns, dtype=torch.float64, device="cuda")
    s.kn_gll(fg, kn)
    assert rel(kn.cpu().numpy().reshape(s.ne, s.ns), P.kn_gll(f)) < 1e-12


@pytest.mark.parametrize("model", [0, 1])
def test_general_moments_wide_xy_grid(F, orc, model):
    """The moment pass with more (x, y) velocity nodes than threads in a
    workgroup (40 x 30 = 1200 columns of 3): 1e-13 against the oracle."""
    mesh = _small_cylinder()
    grid = W.grid_spec((40, 30, 3), 6.0)
    par = _params(model=model, prandtl=2.0 / 3.0 if model == 1 else 1.0)
    P = _oracle(orc, mesh, 1, grid, par)
    f = _state(P, grid, 6)
    s = F.FrDvm(mesh, 1, grid, par)
    Q = torch.zeros(s.ne * s.ns * 5, dtype=torch.float64, device="cuda")
    s.moments(_gpu(s, f), Q)
    assert rel(Q.cpu().numpy().reshape(s.ne, s.ns, 5), P.moments(f)) < 1e-13



@pytest.mark.parametrize("model", [0, 1])
def test_general_moments_point_count_not_a_multiple_of_four(F, orc, model):
    """The moment pass takes four solution points per workgroup (one wave
    each); one quadratic-map element at p = 2 has 27, so the last workgroup
    has a single working wave: 1e-13 against the oracle on a ragged grid."""
    mesh = W.quadratic_map_mesh(1, eps=0.1, bc_all=1)
    grid = W.grid_spec((7, 6, 5), 5.0)
    par = _params(model=model, prandtl=2.0 / 3.0 if model == 1 else 1.0)
    P = _oracle(orc, mesh, 2, grid, par)
    f = _state(P, grid, 9)
    s = F.FrDvm(mesh, 2, grid, par)
    assert (s.ne * s.ns) % 4 == 3
    Q = torch.zeros(s.ne * s.ns * 5, dtype=torch.float64, device="cuda")
    s.moments(_gpu(s, f), Q)
    assert rel(Q.cpu().numpy().reshape(s.ne, s.ns, 5), P.moments(f)) < 1e-13

def test_general_collide_es(F, orc):
    mesh = _small_cylinder()
    par = _params(model=1, prandtl=2.0 / 3.0, mu_ref=0.02)
    P = _oracle(orc, mesh, 2, GRID, par)
    f = _state(P, GRID, 6, amp=0.1)
    s = F.FrDvm(mesh, 2, GRID, par)
    S = torch.zeros(s.shape, dtype=s.dtype, device="cuda")
    s.collide(_gpu(s, f), S)
    ref = P.collide(f)[0]
    assert rel(S.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("rk", [0, 1])
def test_general_rk_steps_es_fp64(F, orc, rk):
    mesh = _small_cylinder()
    par = _params(model=1, prandtl=2.0 / 3.0, mu_ref=0.02)
    P = _oracle(orc, mesh, 2, GRID, par)
    f0 = _state(P, GRID, 7, amp=0.1)
    dt = P.dt(0.2)
    ref = P.rk_step(f0, dt, scheme=rk, nsteps=2)
    s = F.FrDvm(mesh, 2, GRID, dict(par, rk=rk))
    f = _gpu(s, f0)
    s.rk_steps(f, dt, 2)
    assert rel(f.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("p,rk,nsteps", [(2, 1, 5), (1, 0, 5), (3, 1, 3)])
def test_general_rk_steps_mixed(F, orc, p, rk, nsteps):
    """FP32 f with FP64 moments and Newton, warm start: stated bounds after
    a few steps on the cylinder (p <= 2: stage values in registers; p = 3:
    in the LDS column)."""
    mesh = _small_cylinder()
    par = _params(model=1, prandtl=2.0 / 3.0, mu_ref=0.02)
    P = _oracle(orc, mesh, p, GRID, par)
    f0 = _state(P, GRID, 8, amp=0.1)
    dt = P.dt(0.2)
    ref = P.rk_step(f0, dt, scheme=rk, nsteps=nsteps)
    s = F.FrDvm(mesh, p, GRID, dict(par, rk=rk, precision=1, guess=1))
    f = _gpu(s, f0)
    s.rk_steps(f, dt, nsteps)
    got = f.double().cpu().numpy()
    assert rel(got, ref) < 1e-5
    Qg, Qr = P.moments(got), P.moments(ref)
    for a in range(5):
        assert rel(Qg[..., a], Qr[..., a]) < 1e-6, a


@pytest.mark.parametrize("p,prec", [(1, 0), (2, 0), (2, 1)])
def test_specular_wall(F, orc, p, prec):
    """Half box with specular walls at x = 0 and x = 1 (the oracle's mirror
    pin holds for it): residual against the oracle, FP64 to 1e-12, FP32 to
    1e-6."""
    from test_oracle_bc import _specular_half_and_mirror
    grid = W.grid_spec((7, 6, 8), 4.0)  # 336 velocities
    half, _ = _specular_half_and_mirror(p, grid)
    par = _params()
    P = _oracle(orc, half, p, grid, par)
    f = _state(P, grid, 9)
    s = F.FrDvm(half, p, grid, dict(par, precision=prec))
    R = torch.zeros(s.shape, dtype=s.dtype, device="cuda")
    s.residual(_gpu(s, f), R)
    ref = P.residual(f if prec == 0 else f.astype(np.float32).astype(np.float64))
    assert rel(R.double().cpu().numpy(), ref) < (1e-12 if prec == 0 else 1e-6)


def test_specular_box_rk_conserves_mass_and_energy(F):
    mesh = W.box_mesh((2, 2, 2), periodic=False, length=(1.0, 1.2, 0.8))
    mesh = dict(mesh, bc=np.where(mesh["nbr_elem"] < 0, 3, 0).astype(np.int8))
    grid = W.grid_spec(8, 6.0)
    s = F.FrDvm(mesh, 2, grid, _params(model=1, prandtl=2.0 / 3.0, mu_ref=0.02))
    prim = np.tile([1.0, 0.4, -0.2, 0.1, 1.1], (s.ne, s.ns, 1))
    prim[..., 0] += 0.1 * np.random.default_rng(3).uniform(-1, 1, size=(s.ne, s.ns))
    f = _gpu(s, W.maxwellian(prim, grid).numpy())
    t0 = s.moments(f, totals=True)
    s.rk_steps(f, s.dt(0.2), 3)
    t1 = s.moments(f, totals=True)
    assert abs(t1[0] - t0[0]) < 1e-13 * t0[0] and abs(t1[4] - t0[4]) < 1e-13 * t0[4]


def test_wall_box_conserves_mass_and_keeps_wall_maxwellian(F):
    mesh = W.quadratic_map_mesh(2, eps=0.1, bc_all=2)
    grid = W.grid_spec(8, 6.0)
    s = F.FrDvm(mesh, 2, grid, _params(theta_wall=1.3))
    Mw = W.maxwellian(np.array([0.8, 0.0, 0.0, 0.0, 1.3]), grid).numpy()
    f = _gpu(s, np.broadcast_to(Mw, s.shape))
    R = torch.zeros_like(f)
    s.residual(f, R)
    assert R.abs().max().item() < 1e-12 * Mw.max() * 100
    rng = np.random.default_rng(2)
    f = _gpu(s, np.broadcast_to(Mw, s.shape) * (1 + 0.3 * rng.uniform(-1, 1, size=s.shape)))
    s.residual(f, R)
    tot = s.moments(R, totals=True)
    scale = s.moments(R.abs(), totals=True)
    assert abs(tot[0]) < 1e-13 * scale[0]


def test_general_create_rejects_bad_meshes(F):
    box = W.box_mesh((2, 2, 2))
    reo, _ = W.reorient_elements(box, seed=1)
    bad = dict(reo, nbr_orient=reo["nbr_orient"].copy())
    e, f = np.argwhere(bad["nbr_orient"] != 0)[0]
    bad["nbr_orient"][e, f] ^= 1
    nb, nf = bad["nbr_elem"][e, f], bad["nbr_face"][e, f]
    with pytest.raises(F.FrDvmError):
        F.FrDvm(bad, 2, W.grid_spec(3, 2.0))
    open_box = W.box_mesh((2, 2, 2), periodic=False)
    untagged = dict(open_box, bc=np.zeros((8, 6), np.int8))
    with pytest.raises(F.FrDvmError):
        F.FrDvm(untagged, 1, W.grid_spec(3, 2.0))
    assert nb >= 0 and nf >= 0
    with pytest.raises(F.FrDvmError):  # specular faces must be coordinate planes
        F.FrDvm(W.quadratic_map_mesh(2, eps=0.15, bc_all=3), 2, W.grid_spec(4, 3.0))
    with pytest.raises(F.FrDvmError):  # ... on a grid symmetric in their axis
        sym = dict(open_box, bc=np.where(open_box["nbr_elem"] < 0, 3, 0).astype(np.int8))
        F.FrDvm(sym, 1, W.grid_spec(4, 3.0, umin=-2.0))


# ---------------------------------------------------------------------------
# The 48 x 24 x 2 O-grid at Mach 8 (p = 2, 24^3 velocities on [-14, 14]^3)
# ---------------------------------------------------------------------------

def _patch(mesh, e):
    """Element e, its face neighbours, and every other face of those as
    farfield: all that the residual of element e depends on."""
    ids = [e] + sorted({int(x) for x in mesh["nbr_elem"][e] if x >= 0} - {e})
    loc = {g: i for i, g in enumerate(ids)}
    ng = mesh["elem_nodes"].shape[1]
    en = mesh["elem_nodes"][ids]
    uniq, inv = np.unique(en.reshape(-1), return_inverse=True)
    n = len(ids)
    nbr = np.full((n, 6), -1, np.int32)
    nbf = np.zeros((n, 6), np.int8)
    nor = np.zeros((n, 6), np.int8)
    bc = np.ones((n, 6), np.int8)
    for i, g in enumerate(ids):
        for f in range(6):
            gb = mesh["nbr_elem"][g, f]
            if gb < 0:
                bc[i, f] = mesh["bc"][g, f]
            elif gb in loc and (i == 0 or gb == e):
                nbr[i, f] = loc[gb]
                nbf[i, f] = mesh["nbr_face"][g, f]
                nor[i, f] = mesh["nbr_orient"][g, f]
                bc[i, f] = 0
    return {"n_elem": n, "n_nodes": len(uniq), "geom_order": mesh["geom_order"], "nodes": mesh["nodes"][uniq],
            "elem_nodes": inv.reshape(n, ng).astype(np.int32), "nbr_elem": nbr, "nbr_face": nbf,
            "nbr_orient": nor, "bc": bc}, ids


@pytest.fixture(scope="module")
def cyl(F, orc):
    mesh = W.cylinder_mesh()
    grid = W.grid_spec(24, 14.0)
    uinf = 8.0 * math.sqrt(5.0 / 3.0)
    par = _params(model=1, prandtl=2.0 / 3.0, mu_ref=W.mu_ref_from_knudsen(0.01),
                  farfield=[1.0, uinf, 0.0, 0.0, 1.0], theta_wall=2.0)
    s = F.FrDvm(mesh, 2, grid, par)
    xs = orc.geometry(mesh, 2)["xs"]
    rng = np.random.default_rng(31)
    prim = np.zeros((s.ne, s.ns, 5))
    prim[..., 0] = 1.0 + 0.01 * rng.uniform(-1, 1, size=(s.ne, s.ns))
    prim[..., 1] = uinf * np.clip((np.hypot(xs[..., 0], xs[..., 1]) - 0.5) / 0.5, 0.0, 1.0)
    prim[..., 4] = 1.0
    f = W.maxwellian(prim, grid, device="cuda").reshape(s.shape)
    torch.cuda.synchronize()
    return mesh, grid, par, s, f


def test_cylinder_fullsize_residual_sampled_elements(cyl, orc):
    mesh, grid, par, s, f = cyl
    R = torch.empty_like(f)
    s.residual(f, R)
    torch.cuda.synchronize()
    n_r, n_t = 24, 48
    for e in [0, n_r - 1, 5 + n_r * 17, n_r * n_t + 11]:  # wall, farfield, interior, second layer
        pm, ids = _patch(mesh, e)
        Pp = _oracle(orc, pm, 2, grid, par)
        Rr = Pp.residual(f[ids].cpu().numpy())[0]
        assert rel(R[e].cpu().numpy(), Rr) < 1e-12, e


def test_cylinder_fullsize_mixed_step(cyl, F):
    """The Mach-8 O-grid workload as configured: FP32 f, low-storage RK, warm
    Newton start, positivity limiter, from the workload's own impulsive start
    (the seeded farfield state everywhere, a diffuse wall at theta_w = 2).
    Four steps: f stays finite and nonnegative, and every conservative-
    equilibrium solve converges (no fallback to g(Q), no ES guard, no
    non-realizable point), as the paper's conservation requires at every
    point."""
    mesh, grid, par, s, _ = cyl
    w = W.workload("cyl48x24x2_p2_v24_es")
    wpar = dict(W.physics_params(w), precision=1, rk=1, guess=1)
    assert wpar["positivity"] == 1
    m = F.FrDvm(mesh, 2, grid, wpar)
    g = W.maxwellian(W.initial_prim(mesh, 2, w), grid, dtype=torch.float32, device="cuda").reshape(m.shape)
    m.newton_stats(reset=True)
    m.rk_steps(g, m.dt(0.2), 4)
    st = m.newton_stats(reset=True)
    assert torch.isfinite(g).all().item()
    assert g.min().item() >= -1e-12 * g.max().item()
    m.collide(g, torch.empty_like(g))
    status = m.newton_points()[0]
    assert (status == 0).all().item(), torch.bincount(status.reshape(-1).long(), minlength=4).tolist()
    assert st["n_fallback"] == 0 and st["n_guard"] == 0, st
    m.destroy()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_general_single_element_all_farfield_one_velocity(F, orc, p):
    """Edge case: one curved element whose six faces are all farfield, a
    velocity grid of one node (one lane of one wave active)."""
    mesh = W.quadratic_map_mesh(1, eps=0.1, bc_all=1)
    grid = {"n": (1, 1, 1), "umin": (0.7, -0.4, 0.3), "umax": (0.7, -0.4, 0.3)}
    par = _params(farfield=[1.2, 0.1, 0.0, 0.0, 1.0])
    P = _oracle(orc, mesh, p, grid, par)
    f = np.random.default_rng(p).uniform(0.5, 1.5, size=P.shape)
    s = F.FrDvm(mesh, p, grid, par)
    R = torch.zeros(s.shape, dtype=s.dtype, device="cuda")
    s.residual(_gpu(s, f), R)
    assert rel(R.cpu().numpy(), P.residual(f)) < 1e-12


def test_general_wide_velocity_grid_ragged(F, orc):
    """A velocity count far from a multiple of 64 (17 x 19 x 13 = 4199) on
    the small O-grid with walls: residual and two FP64 ES steps."""
    mesh = _small_cylinder()
    grid = W.grid_spec((17, 19, 13), 6.0)
    par = _params(model=1, prandtl=2.0 / 3.0, mu_ref=0.02)
    P = _oracle(orc, mesh, 1, grid, par)
    f0 = _state(P, grid, 12, amp=0.1)
    s = F.FrDvm(mesh, 1, grid, par)
    f = _gpu(s, f0)
    R = torch.zeros_like(f)
    s.residual(f, R)
    assert rel(R.cpu().numpy(), P.residual(f0)) < 1e-12
    dt = P.dt(0.2)
    ref = P.rk_step(f0, dt, scheme=0, nsteps=1)
    s.rk_steps(f, dt, 1)
    assert rel(f.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("model", [0, 1])
def test_half_cylinder_paper_units(F, orc, model):
    """The paper's boundary set and units on curved elements: half O-grid
    with a specular symmetry plane on the cut, diffuse wall at the
    freestream temperature, farfield Maxwellian, Sutherland viscosity with
    mu_ref = 1/Re and P = 1/(gamma M^2) (Mach 2, Re 500): residual and one
    FP64 step against the oracle."""
    mesh = W.cylinder_mesh(n_theta=6, n_r=3, n_z=1, r1=2.0, half=True)
    grid = W.grid_spec((11, 12, 9), 2.5)
    par = dict(_params(model=model, prandtl=2.0 / 3.0 if model else 1.0), **W.paper_freestream(2.0, 500.0, 10.0))
    P = _oracle(orc, mesh, 2, grid, par)
    th = par["theta_ref"]
    prim = np.zeros(P.shape[:2] + (5,))
    prim[..., 0] = 1.0 + 0.05 * np.random.default_rng(6).uniform(-1, 1, size=P.shape[:2])
    prim[..., 1:4] = par["farfield"][1:4]
    prim[..., 4] = th
    f0 = W.maxwellian(prim, grid).numpy()
    s = F.FrDvm(mesh, 2, grid, par)
    f = _gpu(s, f0)
    R = torch.zeros_like(f)
    s.residual(f, R)
    assert rel(R.cpu().numpy(), P.residual(f0)) < 1e-12
    dt = P.dt(0.2)
    ref = P.rk_step(f0, dt, scheme=0, nsteps=1)
    s.rk_steps(f, dt, 1)
    assert rel(f.cpu().numpy(), ref) < 1e-12


@pytest.mark.parametrize("prec,rk", [(0, 0), (1, 1)])
def test_general_bitwise_reproducible(F, orc, prec, rk):
    """Runs from the same state give the same bits: twice on one handle
    (parameters set again in between, so the stage seeds of the stochastic
    rounding start over) and once on a second handle; positivity limiter on,
    ES-BGK, cold Newton start."""
    mesh = _small_cylinder()
    par = _params(model=1, prandtl=2.0 / 3.0, mu_ref=0.02, rk=rk, precision=prec, guess=0, positivity=1)
    P = _oracle(orc, mesh, 2, GRID, _params(model=1, prandtl=2.0 / 3.0, mu_ref=0.02))
    f0 = _state(P, GRID, 9, amp=0.1)
    dt = P.dt(0.2)
    s, t = F.FrDvm(mesh, 2, GRID, par), F.FrDvm(mesh, 2, GRID, par)
    runs = []
    for h in (s, s, t):
        h.set_params(**par)
        f = _gpu(h, f0)
        h.rk_steps(f, dt, 3)
        runs.append(f)
    assert torch.equal(runs[0], runs[1]) and torch.equal(runs[0], runs[2])
    assert not torch.equal(runs[0], _gpu(s, f0))  # it moved
