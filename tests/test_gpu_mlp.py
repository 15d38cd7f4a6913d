"""GPU tests of the learned Newton initial guess: the forward pass and the
gradient of the hand-written FP32/MFMA kernels against the FP64 oracle, one
Adam step, the conservative-equilibrium solve on caller moments, and the
gain of a trained network over the cold start (Newton alone decides convergence)."""
import numpy as np
import pytest

import workloads as W
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_06567_amd import frdvm
    frdvm.lib()
    return frdvm


def _rand_net(H, seed):
    rng = np.random.default_rng(seed)
    w = omlp.init(H, seed=seed) + 0.05 * rng.standard_normal(omlp.n_params(H))
    w[-10:-5] = rng.uniform(0.5, 2.0, 5)   # output scale
    w[-5:] = rng.uniform(-1, 1, 5)         # output offset
    return w


@pytest.mark.parametrize("H,B", [(64, 300), (16, 37), (64, 4096)])
def test_forward_matches_oracle(F, H, B):
    rng = np.random.default_rng(1)
    w = _rand_net(H, 2)
    X = rng.standard_normal((B, omlp.N_IN))
    ref = omlp.predict(w, X, H)
    net = F.Mlp(H)
    got = net.forward(torch.as_tensor(w, dtype=torch.float32).cuda(),
                      torch.as_tensor(X, dtype=torch.float32).cuda()).cpu().numpy()
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-5


@pytest.mark.parametrize("H,B", [(64, 512), (24, 99)])
def test_gradient_matches_oracle(F, H, B):
    """FP32 GPU backpropagation against FP64 backpropagation (itself pinned
    to central finite differences): relative L2 <= 1e-3 per layer."""
    rng = np.random.default_rng(3)
    w = _rand_net(H, 4)
    X = rng.standard_normal((B, omlp.N_IN))
    T = rng.standard_normal((B, 5))
    loss_ref, g_ref = omlp.loss_and_grad(w, X, T, H)
    net = F.Mlp(H)
    g, loss = net.grad(torch.as_tensor(w, dtype=torch.float32).cuda(), torch.as_tensor(X, dtype=torch.float32).cuda(),
                       torch.as_tensor(T, dtype=torch.float32).cuda())
    g = g.cpu().numpy()
    assert abs(loss.item() - loss_ref) < 1e-5 * loss_ref
    o = 0
    for (m, k) in omlp.layer_shapes(H):
        for n_ in (m * k, m):
            seg = slice(o, o + n_)
            assert np.linalg.norm(g[seg] - g_ref[seg]) <= 1e-3 * np.linalg.norm(g_ref[seg]), (m, k, n_)
            o += n_
    assert np.all(g[o:] == 0)


def test_adam_step_matches_oracle(F):
    H = 16
    rng = np.random.default_rng(5)
    w = _rand_net(H, 6)
    g = rng.standard_normal(w.size) * 1e-2
    m = rng.standard_normal(w.size) * 1e-3
    v = rng.uniform(0, 1e-4, w.size)
    nw = w.size - 10
    w_ref, m_ref, v_ref = omlp.adam_update(w[:nw], g[:nw], m[:nw], v[:nw], 7, 1e-3)
    t = lambda a: torch.as_tensor(a, dtype=torch.float32).cuda().contiguous()
    wd, md, vd = t(w), t(m), t(v)
    F.Mlp(H).adam(wd, t(g), md, vd, 7, 1e-3)
    assert np.allclose(wd.cpu().numpy()[:nw], w_ref, rtol=1e-5, atol=1e-7)
    assert np.allclose(vd.cpu().numpy()[:nw], v_ref, rtol=1e-5, atol=1e-12)
    assert np.array_equal(wd.cpu().numpy()[nw:], w[nw:].astype(np.float32))


def test_equilibrium_on_caller_moments_matches_oracle(F, orc):
    """Newton on given moments (the training-target path) against the oracle
    collision of a distribution with those moments."""
    grid = W.grid_spec(12, 6.0)
    h = F.FrDvm(W.box_mesh(1), 1, grid, {"model": 0, "mu_ref": 1.0})
    rng = np.random.default_rng(8)
    P = orc.Problem.points_only(grid, {"model": 0, "mu_ref": 1.0})
    f = np.exp(-0.5 * ((P.u - [0.4, -0.3, 0.2]) ** 2).sum(1) / 0.8)[None] * rng.uniform(0.6, 1.4, (5, P.nu))
    Q = orc.moments(f, P.u, P.w)
    z, it, ev, st, res = h.equilibrium(torch.as_tensor(Q).cuda().contiguous())
    zr = P.collide(f)[2]
    assert np.all(st.cpu().numpy() == 0)
    assert np.abs(z.cpu().numpy() - zr).max() < 1e-10


def test_trained_guess_saves_newton_iterations(F):
    """Train on solver-solved states of the 32^3 grids with u_max in
    {6, 10, 14}; on held-out states the MLP-seeded Newton converges to the
    same root and tolerance with fewer linear solves, and no more grid
    passes (the extra pass that compares the two starts included), than the
    cold start."""
    from paper_2312_06567_amd import learned
    w, info = learned.fit_guess(n_states=30000, steps=4000, seed=4)
    assert info["n_converged"] > 0.95 * info["n_states"]
    test = W.sample_states(4000, seed=99)
    a = learned.solve_targets(test, guess=F.GUESS_COLD)
    b = learned.solve_targets(test, guess=F.GUESS_MLP, weights=w)
    ok0, ok1 = a["status"] == 0, b["status"] == 0
    assert ok1.mean() >= ok0.mean()
    both = ok0 & ok1
    hard = both & (a["iters"] >= 5)
    print(f"cold {a['iters'][both].mean():.3f} solves / {a['evals'][both].mean():.3f} passes, "
          f"MLP {b['iters'][both].mean():.3f} / {b['evals'][both].mean():.3f}; hard states ({hard.sum()}): "
          f"cold {a['iters'][hard].mean():.2f}, MLP {b['iters'][hard].mean():.2f}; "
          f"fallback cold {1 - ok0.mean():.4f} MLP {1 - ok1.mean():.4f}; reject {info['reject_rate']:.3f}")
    assert b["iters"][both].mean() < a["iters"][both].mean()
    assert b["iters"][hard].mean() < a["iters"][hard].mean() - 0.5
    assert np.abs(b["z"][both] - a["z"][both]).max() < 1e-9
    assert b["resid"][both].max() <= 1e-11
