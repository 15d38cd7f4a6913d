"""GPU edge cases against the FP64 oracle: the largest velocity grid the
library accepts (64 nodes per axis), a velocity axis with a single node,
points whose moments admit no equilibrium, and a call with no steps."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_06567_amd import frdvm
    frdvm.lib()
    return frdvm


def _params(model=0, pr=1.0, mu=0.05, **kw):
    d = {"model": model, "prandtl": pr, "mu_ref": mu, "theta_ref": 1.0, "omega": 0.81,
         "newton_tol": 1e-13, "newton_max_iter": 50}
    d.update(kw)
    return d


def _noisy_maxwellian(mesh, p, grid, seed, amp=0.2):
    xs = W.box_solution_points(mesh, p)
    prim = W.prim_random_modes(xs, seed=seed, U_amp=0.3)
    f = W.maxwellian(prim, grid).numpy()
    rng = np.random.default_rng(seed)
    return f * (1.0 + amp * rng.uniform(-1, 1, size=f.shape))


def _gpu(s, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=s.dtype).cuda()


def test_largest_velocity_grid(F, orc):
    """64^3 velocities, the largest grid the library accepts (4096 chunks of
    64 per element; the ES Newton's factor tables no longer fit its LDS and
    it takes the direct sums): transport residual and ES collision against
    the oracle."""
    mesh = W.box_mesh((2, 2, 2))
    grid = W.grid_spec(64, 8.0)
    f = _noisy_maxwellian(mesh, 1, grid, 11, amp=0.1)
    par = _params(model=2)
    s = F.FrDvm(mesh, 1, grid, par)
    R = torch.zeros(s.shape, dtype=s.dtype, device="cuda")
    s.residual(_gpu(s, f), R)
    assert rel(R.cpu().numpy(), orc.Problem(mesh, 1, grid, par).residual(f)) < 1e-12
    s.destroy()
    par = _params(model=1, pr=0.71)
    s = F.FrDvm(mesh, 1, grid, par)
    S = torch.zeros(s.shape, dtype=s.dtype, device="cuda")
    s.collide(_gpu(s, f), S)
    Sr, prim, z, st, it = orc.Problem(mesh, 1, grid, par).collide(f)
    assert np.all(st == 0)
    tau_scale = np.abs(Sr).max() + np.abs(f).max() / 0.05
    assert np.abs(S.cpu().numpy() - Sr).max() < 1e-12 * tau_scale
    s.destroy()


def test_single_node_velocity_axis(F, orc):
    """A velocity axis with one node (weight 1): transport residual and
    moments against the oracle."""
    mesh = W.box_mesh((2, 3, 2))
    grid = W.grid_spec((9, 7, 1), 5.0)
    par = _params(model=2)
    f = _noisy_maxwellian(mesh, 2, grid, 12)
    s = F.FrDvm(mesh, 2, grid, par)
    P = orc.Problem(mesh, 2, grid, par)
    R = torch.zeros(s.shape, dtype=s.dtype, device="cuda")
    s.residual(_gpu(s, f), R)
    assert rel(R.cpu().numpy(), P.residual(f)) < 1e-12
    Q = torch.zeros(s.ne * s.ns * 5, dtype=torch.float64, device="cuda")
    s.moments(_gpu(s, f), Q)
    assert rel(Q.cpu().numpy().reshape(s.ne, s.ns, 5), P.moments(f)) < 1e-13


@pytest.mark.parametrize("model", [0, 1])
def test_points_without_equilibrium(F, orc, model):
    """Points whose moments admit no equilibrium (zero density, negative
    density) get no collision source, as in the oracle; every other point
    matches the oracle."""
    mesh = W.box_mesh((2, 2, 2))
    p = 1
    grid = W.grid_spec(8, 6.0)
    par = _params(model=model, pr=0.71 if model == 1 else 1.0)
    f = _noisy_maxwellian(mesh, p, grid, 13)
    fp = f.reshape(-1, f.shape[-1])
    fp[3] = 0.0
    fp[10] = -fp[10]
    s = F.FrDvm(mesh, p, grid, par)
    S = torch.zeros(s.shape, dtype=s.dtype, device="cuda")
    s.collide(_gpu(s, f), S)
    Sr, prim, z, st, it = orc.Problem(mesh, p, grid, par).collide(f)
    stp = st.reshape(-1)
    assert stp[3] != 0 and stp[10] != 0 and np.all(np.delete(stp, [3, 10]) == 0)
    Sg = S.cpu().numpy().reshape(fp.shape)
    assert np.all(Sg[3] == 0) and np.all(Sg[10] == 0)
    tau_scale = np.abs(Sr).max() + np.abs(f).max() / 0.05
    assert np.abs(Sg - Sr.reshape(fp.shape)).max() < 1e-12 * tau_scale


def test_zero_steps_leave_f_unchanged(F):
    mesh = W.box_mesh(2)
    grid = W.grid_spec(6, 5.0)
    s = F.FrDvm(mesh, 1, grid, _params())
    f0 = _noisy_maxwellian(mesh, 1, grid, 14)
    f = _gpu(s, f0)
    g = f.clone()
    s.rk_steps(f, 1e-3, 0)
    torch.cuda.synchronize()
    assert torch.equal(f, g)
