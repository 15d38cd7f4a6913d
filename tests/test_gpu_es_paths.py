"""The factorised ES-BGK Newton sums (3n + 3n^2 exponentials per evaluation)
against the direct per-node sums and the oracle, on grids where the two-axis
cross factors are large (shifted, anisotropic distributions)."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_06567_amd import frdvm
    frdvm.lib()
    return frdvm


def _aniso(u, U, C, rho=1.0):
    d = u - np.asarray(U)
    Ci = np.linalg.inv(C)
    return rho / np.sqrt(np.linalg.det(2 * np.pi * C)) * np.exp(-0.5 * np.einsum("ki,ij,kj->k", d, Ci, d))


@pytest.mark.parametrize("n,umax,U,pr", [(20, 8.0, (0.5, -0.3, 0.2), 0.71), (24, 14.0, (8.0, 1.0, -0.5), 2.0 / 3.0)])
def test_factorised_equals_direct_and_oracle(F, orc, n, umax, U, pr):
    grid = W.grid_spec(n, umax)
    par = {"model": 1, "prandtl": pr, "mu_ref": 0.01, "omega": 0.81}
    mesh = W.box_mesh(1)
    P = orc.Problem.points_only(grid, par)
    C = np.array([[1.6, 0.5, -0.3], [0.5, 1.0, 0.2], [-0.3, 0.2, 1.3]])
    f = np.stack([_aniso(P.u, U, C * s, 1.0 + 0.1 * s) for s in (0.6, 1.0, 1.7)])
    f = np.concatenate([f, np.zeros((5, P.nu))])[:8]  # the one p=1 element has 8 points
    f[3:] = f[:1] * (1 + 0.05 * np.sin(np.arange(P.nu)))[None]
    outs = {}
    for direct in (0, 1):
        os.environ["FRDVM_ES_DIRECT"] = str(direct)
        s = F.FrDvm(mesh, 1, grid, par)
        fg = torch.as_tensor(f.reshape(s.shape)).cuda().contiguous()
        S = torch.empty_like(fg)
        Qp = torch.empty(s.ne * s.ns * 5, dtype=torch.float64, device="cuda")
        s.collide(fg, S, Qp)
        outs[direct] = (S.cpu().numpy().reshape(8, -1), Qp.cpu().numpy().reshape(8, 5), s.newton_stats())
    os.environ.pop("FRDVM_ES_DIRECT", None)
    Sr, prim, z, st, it = P.collide(f)
    scale = np.abs(f).max() / 0.01 * 10
    for direct in (0, 1):
        S, Qp, stats = outs[direct]
        assert stats["n_fallback"] == 0
        assert np.abs(S - Sr).max() < 1e-11 * scale, direct
        assert np.allclose(Qp, prim, rtol=1e-11, atol=1e-12)
    assert np.abs(outs[0][0] - outs[1][0]).max() < 1e-11 * scale
