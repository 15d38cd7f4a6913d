"""GPU parity of the mixed-mesh path (hexahedra, prisms, tetrahedra; Section
"Implementation & problem setup": the paper's element types with
alpha-optimised points on simplices and Gauss-Lobatto points on
tensor-product elements; Section "Numerical method": FR with the
DG-recovering correction and the upwind flux) against the mixed-mesh FP64
oracle, on the periodic 3^3-cell box whose centre cell is six tetrahedra and
whose rows through it are prisms (20 hexahedra, 12 prisms, 6 tetrahedra).

* Residual, FP64, p = 1..3, on a grid of 7 x 6 x 5 velocities (210 nodes:
  four chunks of 64, the last one partial): 1e-12 relative; FP32 2e-6.
* RK steps, FP64, BGK and ES-BGK (Pr 2/3), both schemes: 1e-12 after two
  steps; every Newton solve converges; mass, momentum and energy conserved
  to 1e-13.  FP32 (low-storage RK, stochastic rounding): f 1e-5 and the
  moments 1e-6.
* An all-hexahedron mesh through the mixed path equals the hexahedral path
  with Gauss-Lobatto points (1e-12).
* Options the path does not take are refused.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

RAGGED = W.grid_spec((7, 6, 5), 4.0)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_06567_amd import frdvm
    frdvm.lib()
    return frdvm


@pytest.fixture(scope="module")
def mixed():
    from oracle import mixed as M
    return M


def _params(model=0):
    par = {"model": model, "mu_ref": 0.02, "theta_ref": 1.0, "omega": 0.81, "newton_tol": 1e-13,
           "newton_max_iter": 50}
    par["prandtl"] = 2.0 / 3.0 if model == 1 else 1.0
    return par


def _state(mesh, p, grid, seed=3, noise=0.02):
    xs = W.mixed_solution_points(mesh, p)
    two_pi = 2.0 * np.pi
    prim = np.stack([1.0 + 0.1 * np.sin(two_pi * xs[:, 0]) * np.cos(two_pi * xs[:, 2]),
                     0.2 * np.cos(two_pi * xs[:, 1]), 0.15 * np.sin(two_pi * (xs[:, 0] + xs[:, 2])),
                     -0.1 * np.sin(two_pi * xs[:, 1]), 1.0 + 0.05 * np.cos(two_pi * xs[:, 0])], 1)
    f0 = W.maxwellian(prim, grid).numpy()
    rng = np.random.default_rng(seed)
    return f0 * (1.0 + noise * rng.uniform(-1.0, 1.0, f0.shape))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_mixed_residual(F, mixed, p):
    mesh = W.mixed_box_mesh(3)
    f0 = _state(mesh, p, RAGGED)
    P = mixed.MixedProblem(mesh, p, RAGGED, _params())
    ref = P.residual(f0)
    s = F.FrDvm(mesh, p, RAGGED, dict(_params(), precision=0))
    assert s.ne == P.mm.npts and s.ns == 1
    f = torch.as_tensor(f0).cuda().contiguous()
    R = torch.empty_like(f)
    s.residual(f, R)
    assert rel(R.cpu().numpy(), ref) < 1e-12
    s32 = F.FrDvm(mesh, p, RAGGED, dict(_params(), precision=1))
    f32 = torch.as_tensor(f0, dtype=torch.float32).cuda().contiguous()
    R32 = torch.empty_like(f32)
    s32.residual(f32, R32)
    assert rel(R32.double().cpu().numpy(), ref) < 2e-6


@pytest.mark.parametrize("model,rk", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_mixed_rk_steps_fp64(F, mixed, model, rk):
    mesh = W.mixed_box_mesh(3)
    grid = W.grid_spec(8, 5.0)
    p = 2
    f0 = _state(mesh, p, grid)
    P = mixed.MixedProblem(mesh, p, grid, _params(model))
    dt = P.dt(0.2)
    ref = P.rk_step(f0, dt, scheme=rk, nsteps=2)
    s = F.FrDvm(mesh, p, grid, dict(_params(model), precision=0, rk=rk, guess=1))
    assert s.dt(0.2) == pytest.approx(dt, rel=1e-14)
    f = torch.as_tensor(f0).cuda().contiguous()
    tot0 = s.moments(f, totals=True)
    s.newton_stats(reset=True)
    s.rk_steps(f, dt, 2)
    st = s.newton_stats(reset=True)
    assert st["n_fallback"] == 0 and st["n_guard"] == 0, st
    got = f.cpu().numpy()
    assert rel(got, ref) < 1e-12
    tot = s.moments(f, totals=True)
    assert np.abs(np.asarray(tot) - np.asarray(tot0)).max() < 1e-13 * np.abs(np.asarray(tot0)).max()
    assert np.allclose(np.asarray(tot0), P.totals(f0), rtol=1e-13, atol=1e-15)


def test_mixed_rk_steps_fp32(F, mixed):
    mesh = W.mixed_box_mesh(3)
    grid = W.grid_spec(8, 5.0)
    p = 3
    f0 = _state(mesh, p, grid).astype(np.float32).astype(np.float64)
    P = mixed.MixedProblem(mesh, p, grid, _params(1))
    dt = P.dt(0.2)
    ref = P.rk_step(f0, dt, scheme=1, nsteps=2)
    s = F.FrDvm(mesh, p, grid, dict(_params(1), precision=1, rk=1, guess=1))
    f = torch.as_tensor(f0, dtype=torch.float32).cuda().contiguous()
    s.rk_steps(f, dt, 2)
    got = f.double().cpu().numpy()
    Qg, Qr = P.moments(got), P.moments(ref)
    ef = rel(got, ref)
    eq = max(rel(Qg[:, 0], Qr[:, 0]), rel(Qg[:, 1:4], Qr[:, 1:4]), rel(Qg[:, 4], Qr[:, 4]))
    print(f"mixed FP32: f {ef:.2e}, moments {eq:.2e}")
    assert ef < 1e-5 and eq < 1e-6


@pytest.mark.parametrize("p", [1, 2, 3])
def test_all_hexahedra_match_the_hexahedral_path(F, p):
    box = W.box_mesh(3)
    hexmesh = dict(box, elem_type=np.zeros(box["n_elem"], np.int8), period=(1.0, 1.0, 1.0))
    grid = W.grid_spec(6, 4.0)
    f0 = _state(hexmesh, p, grid)
    a = F.FrDvm(hexmesh, p, grid, dict(_params(), precision=0))
    b = F.FrDvm(box, p, grid, dict(_params(), precision=0), nodes=1)
    f = torch.as_tensor(f0).cuda().contiguous()
    Ra, Rb = torch.empty_like(f), torch.empty_like(f)
    a.residual(f, Ra)
    b.residual(f.reshape(b.shape), Rb.reshape(b.shape))
    assert rel(Ra.cpu().numpy(), Rb.cpu().numpy()) < 1e-12


def test_mixed_refuses_unsupported_options(F):
    mesh = W.mixed_box_mesh(3)
    grid = W.grid_spec(6, 4.0)
    with pytest.raises(F.FrDvmError):
        F.FrDvm(mesh, 2, grid, dict(_params(), positivity=1))
    with pytest.raises(F.FrDvmError):
        F.FrDvm(mesh, 2, grid, dict(_params(), precision=F.FP32_DEV, rk=1))
    s = F.FrDvm(mesh, 2, grid, dict(_params(), precision=0))
    f = torch.ones(s.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(F.FrDvmError):
        s.kn_gll(f, torch.empty(s.ne * s.ns, dtype=torch.float64, device="cuda"))
    bad = dict(mesh, nodes=mesh["nodes"].copy())
    bad["nodes"][5] += 0.01  # a moved vertex: elements no longer straight or faces unmatched
    with pytest.raises(F.FrDvmError):
        F.FrDvm(bad, 2, grid)


@pytest.mark.parametrize("prec,rk", [(0, 0), (1, 1)])
def test_mixed_bitwise_reproducible(F, prec, rk):
    """Runs from the same state give the same bits: twice on one handle
    (parameters set again in between: the stage seeds of the stochastic
    rounding start over) and once on a second handle."""
    mesh = W.mixed_box_mesh(3)
    grid = W.grid_spec(8, 5.0)
    p = 3
    par = dict(_params(1), precision=prec, rk=rk, guess=0)
    f0 = _state(mesh, p, grid)
    s, t = F.FrDvm(mesh, p, grid, par), F.FrDvm(mesh, p, grid, par)
    dt = s.dt(0.2)
    dtype = torch.float64 if prec == 0 else torch.float32
    runs = []
    for h in (s, s, t):
        h.set_params(**par)
        f = torch.as_tensor(f0, dtype=dtype).cuda().contiguous()
        h.rk_steps(f, dt, 3)
        runs.append(f)
    assert torch.equal(runs[0], runs[1]) and torch.equal(runs[0], runs[2])
    assert not torch.equal(runs[0], torch.as_tensor(f0, dtype=dtype).cuda())
