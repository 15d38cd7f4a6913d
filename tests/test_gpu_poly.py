"""GPU parity of the reduced distribution pair (F, G) for a gas with delta
internal degrees of freedom (fr_dvm_create_gas) against the oracle on the
same seeded inputs: FP64 to 1e-12 unless stated."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DELTA = 2.0
FAR = [1.0, 1.2, 0.0, 0.0, 1.0]


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
         "newton_tol": 1e-13, "newton_max_iter": 50, "farfield": FAR, "theta_wall": 1.5}
    d.update(kw)
    return d


def _pair_of(P, grid, seed, amp=0.2, th_i=0.7):
    prim = W.prim_random_modes(P.geo["xs"], seed=seed, U_amp=0.3)
    Fm = W.maxwellian(prim, grid).numpy()
    f = np.concatenate([Fm, 0.5 * DELTA * th_i * Fm], -1)
    return f * (1.0 + amp * np.random.default_rng(seed).uniform(-1, 1, size=f.shape))


def _make(orc, F, mesh, p, grid, par):
    fF = W.maxwellian(np.array(par["farfield"]), grid).numpy()
    finf = np.concatenate([fF, 0.5 * DELTA * par["farfield"][4] * fF])
    P = orc.Problem(mesh, p, grid, {**par, "f_inf": finf, "delta": DELTA})
    s = F.FrDvm(mesh, p, grid, par, delta=DELTA)
    assert s.shape == P.shape
    return P, s


def _gpu(s, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=s.dtype).cuda()


GRID = W.grid_spec((7, 6, 5), 5.0)  # 210 velocities, 420 state values per point


def _mesh(name):
    if name == "box":
        return W.box_mesh((3, 2, 2), length=(1.0, 0.8, 0.6))
    if name == "cylinder":
        return W.cylinder_mesh(n_theta=8, n_r=3, n_z=2, r1=2.0)
    return W.cylinder_mesh(n_theta=6, n_r=2, n_z=1, r1=2.0, half=True)


# periodic boxes run on the fused box path, the O-grids on the general path
@pytest.mark.parametrize("name,p", [("box", 1), ("box", 2), ("box", 3), ("cylinder", 2), ("half", 2)])
def test_pair_residual(F, orc, name, p):
    grid = GRID if name != "half" else W.grid_spec((7, 6, 5), 5.0)
    P, s = _make(orc, F, _mesh(name), p, grid, _params())
    f = _pair_of(P, grid, 3)
    R = torch.zeros(s.shape, dtype=s.dtype, device="cuda")
    s.residual(_gpu(s, f), R)
    assert rel(R.cpu().numpy(), P.residual(f)) < 1e-12


@pytest.mark.parametrize("model", [0, 1])
def test_pair_collide_moments_kn(F, orc, model):
    mesh = _mesh("box")
    grid = W.grid_spec(8, 6.0)
    par = _params(model=model, prandtl=0.71 if model else 1.0)
    P, s = _make(orc, F, mesh, 2, grid, par)
    f = _pair_of(P, grid, 4, amp=0.1)
    fg = _gpu(s, f)
    S = torch.zeros_like(fg)
    Qp = torch.zeros(s.ne * s.ns * 5, dtype=torch.float64, device="cuda")
    s.collide(fg, S, Qp)
    Sr, prim, z, st, it = P.collide(f)
    assert np.all(st == 0)
    scale = np.abs(Sr).max() + np.abs(f).max() / 0.05
    assert np.abs(S.cpu().numpy() - Sr).max() < 1e-12 * scale
    assert rel(Qp.cpu().numpy().reshape(prim.shape), prim) < 1e-12
    Q = torch.zeros(s.ne * s.ns * 5, dtype=torch.float64, device="cuda")
    tot = s.moments(fg, Q, totals=True)
    assert rel(Q.cpu().numpy().reshape(s.ne, s.ns, 5), P.moments(f)) < 1e-13
    assert rel(tot, P.totals(f)) < 1e-13
    kn = torch.zeros(s.ne * s.ns, dtype=torch.float64, device="cuda")
    s.kn_gll(fg, kn)
    assert rel(kn.cpu().numpy().reshape(s.ne, s.ns), P.kn_gll(f)) < 1e-12


# (5, 5, 6) nodes: 150 velocities, an odd number of 64-wide chunks per component
@pytest.mark.parametrize("name,rk,p,nv", [("box", 0, 2, 8), ("box", 1, 2, 8), ("box", 1, 3, (5, 5, 6)),
                                          ("box", 0, 1, (5, 5, 6)), ("cylinder", 0, 2, 8)])
def test_pair_rk_steps_es(F, orc, name, rk, p, nv):
    mesh = _mesh(name)
    grid = W.grid_spec(nv, 6.0)
    par = _params(model=1, prandtl=0.71, mu_ref=0.02, rk=rk)
    P, s = _make(orc, F, mesh, p, grid, par)
    f0 = _pair_of(P, grid, 5, amp=0.1)
    dt = P.dt(0.2)
    ref = P.rk_step(f0, dt, scheme=rk, nsteps=2)
    f = _gpu(s, f0)
    s.rk_steps(f, dt, 2)
    assert rel(f.cpu().numpy(), ref) < 1e-12


def test_pair_mixed_precision_bounds(F, orc):
    mesh = _mesh("box")
    grid = W.grid_spec(8, 6.0)
    par = _params(model=1, prandtl=0.71, mu_ref=0.02, rk=1, precision=1, guess=1)
    P, s = _make(orc, F, mesh, 2, grid, par)
    f0 = _pair_of(P, grid, 6, amp=0.1)
    dt = P.dt(0.2)
    ref = P.rk_step(f0, dt, scheme=1, nsteps=5)
    f = _gpu(s, f0)
    s.rk_steps(f, dt, 5)
    got = f.double().cpu().numpy()
    assert rel(got, ref) < 1e-5
    Qg, Qr = P.moments(got), P.moments(ref)
    for a in range(5):
        assert rel(Qg[..., a], Qr[..., a]) < 1e-6, a


@pytest.mark.parametrize("precision", [0, 1])
def test_pair_overlapped_newton_is_identical(F, orc, precision):
    # the Newton solve of the next stage on the second stream, half of the
    # elements at a time, gives the same bits as the one-stream order
    mesh = W.box_mesh((4, 2, 2), length=(1.0, 0.5, 0.5))
    grid = W.grid_spec((5, 5, 6), 6.0)
    out = []
    for ov in (0, 1):
        par = _params(model=1, prandtl=0.71, mu_ref=0.02, rk=1, precision=precision, guess=0, overlap=ov)
        P, s = _make(orc, F, mesh, 2, grid, par)
        f0 = _pair_of(P, grid, 9, amp=0.1)
        f = _gpu(s, f0)
        dt = P.dt(0.2)
        s.rk_steps(f, dt, 3)
        out.append(f.cpu().numpy())
    assert np.array_equal(out[0], out[1])
    if precision == 0:
        assert rel(out[1], P.rk_step(f0, dt, scheme=1, nsteps=3)) < 1e-12


def test_pair_periodic_step_conserves_total_energy(F):
    mesh = _mesh("box")
    grid = W.grid_spec(8, 6.0)
    s = F.FrDvm(mesh, 2, grid, _params(model=1, prandtl=0.71, mu_ref=0.02), delta=DELTA)
    prim = np.tile([1.0, 0.3, -0.1, 0.2, 1.2], (s.ne, s.ns, 1))
    prim[..., 0] += 0.1 * np.random.default_rng(8).uniform(-1, 1, size=(s.ne, s.ns))
    Fm = W.maxwellian(prim, grid).numpy()
    f = _gpu(s, np.concatenate([Fm, 0.5 * DELTA * 0.5 * Fm], -1))  # internal mode colder
    t0 = s.moments(f, totals=True)
    s.rk_steps(f, s.dt(0.2), 3)
    t1 = s.moments(f, totals=True)
    assert np.abs(t1 - t0).max() < 1e-12 * np.abs(t0).max()


def test_create_gas_rejects_negative_delta(F):
    with pytest.raises(F.FrDvmError):
        F.FrDvm(W.box_mesh(2), 1, W.grid_spec(3, 2.0), delta=-1.0)
