"""The allocation-free contrastive entry point against the one that takes a
workspace: same kernels, so every output must agree bitwise.  Two calls in a
row, the second smaller, so the second runs on scratch the first left
behind; a size past the static scratch is refused on the host."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    from paper_2505_00690_amd import vl
    vl.lib()
    return vl


def _pairs(n, dim, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    e = rng.standard_normal((n, dim))
    t = rng.standard_normal((n, dim))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    t[: n // 2] = 0.7 * t[: n // 2] + 0.3 * e[: n // 2]
    return (torch.from_numpy(e.astype(np.float32)).cuda(),
            torch.from_numpy(t.astype(np.float32)).cuda())


def test_noalloc_matches_workspace_entry_point(V):
    cases = [(2048, 768, "sigmoid", 10.0, -10.0), (300, 128, "softmax", 100.0, 0.0),
             (37, 512, "sigmoid", 10.0, -10.0)]
    for n, dim, head, scale, bias in cases:
        print(f"noalloc contrastive n={n} dim={dim} head={head}", flush=True)
        e, t = _pairs(n, dim, 700 + n)
        ref = V.vl_contrastive_loss(e, t, head, scale, bias)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        de = torch.empty_like(e)
        dt = torch.empty_like(t)
        dsb = torch.empty(2, dtype=torch.float32, device="cuda")
        V.vl_contrastive_loss_noalloc(e, t, head, scale, bias, loss, de, dt, dsb)
        torch.cuda.synchronize()
        for name, got, want in zip(("loss", "d_emb", "d_texts", "d_scale_bias"),
                                   (loss, de, dt, dsb), ref):
            assert torch.equal(got, want), (n, dim, head, name)
        assert np.isfinite(loss.item())


def test_noalloc_rejects_oversize_on_host(V):
    e = torch.zeros((2529, 768), dtype=torch.float32, device="cuda")
    out = [torch.empty(1, device="cuda"), torch.empty_like(e), torch.empty_like(e),
           torch.empty(2, device="cuda")]
    with pytest.raises(V.VlError) as ei:
        V.vl_contrastive_loss_noalloc(e, e, "softmax", 10.0, 0.0, *out)
    assert "scratch" in str(ei.value)
