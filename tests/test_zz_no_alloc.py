"""The no-allocation MLP forward (fr_mlp_forward_noalloc) against the
workspace forward (fr_mlp_forward), both through the C ABI: calls in a row on
the same GPU, each later one with a smaller batch, for two hidden widths; the
largest batch the fixed scratch holds; and a batch one larger, which is
refused before any launch."""
import ctypes as C

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_06567_amd import frdvm
    frdvm.lib()
    return frdvm


def _p(t):
    return C.c_void_p(t.data_ptr())


def test_noalloc_forward_equals_workspace_forward(F):
    g = torch.Generator().manual_seed(7)
    for H in (64, 24):
        m = F.Mlp(H)
        w = ((torch.rand(m.n, generator=g) - 0.5) * 0.5).cuda()
        for B in (5000, 1237):
            X = torch.randn(B, F.MLP_INPUTS, generator=g).cuda()
            ref = m.forward(w, X)
            out = torch.full((B, 5), float("nan"), device="cuda")
            m.forward_noalloc(w, X, out)
            torch.cuda.synchronize()
            print(f"H {H} B {B}: max |diff| {(out - ref).abs().max().item():.3e}", flush=True)
            assert torch.equal(out, ref), (H, B)


def test_noalloc_forward_capacity(F):
    H = 64
    m = F.Mlp(H)
    g = torch.Generator().manual_seed(8)
    w = ((torch.rand(m.n, generator=g) - 0.5) * 0.5).cuda()
    bmax = F.MLP_NOALLOC_FLOATS // (2 * H + 5)
    X = torch.randn(bmax + 1, F.MLP_INPUTS, generator=g).cuda()
    out = torch.full((bmax + 1, 5), float("nan"), device="cuda")
    rc = F.lib().fr_mlp_forward_noalloc(H, _p(w), _p(X), bmax + 1, _p(out), None)
    assert rc == F.E_SCRATCH
    torch.cuda.synchronize()
    assert torch.isnan(out).all().item()  # nothing was launched
    Xm = X[:bmax].contiguous()
    ref = m.forward(w, Xm)
    got = out[:bmax].contiguous()
    m.forward_noalloc(w, Xm, got)
    torch.cuda.synchronize()
    assert torch.equal(got, ref)
