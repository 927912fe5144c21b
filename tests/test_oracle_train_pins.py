"""Pins of the training (backward) oracle, oracle/train64.py, on the CPU.

The explicit chain rule is checked against things other than itself:
float64 autograd through an encoder written with PyTorch library operations
(conv2d patchify, bilinear interpolate of the position grid, layer_norm,
linear, softmax attention), central finite differences of the oracle's own
forward, and the closed-form invariants of LayerNorm, softmax attention and
GELU derivatives."""
import math

import numpy as np
import pytest

import synth
from oracle import train64 as TR
from oracle import vit64 as O

torch = pytest.importorskip("torch")


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _small(layers=2, std=0.2):
    c = synth.ModelConfig("tiny_train", 16, 64, layers, 4, 256, 32, 4)
    p = synth.make_params(c, 41, std=std)
    return c, p


def _torch_encode(c, tp, img):
    """The forward written with torch library operations on torch tensors
    (tp: name -> leaf tensor; block tensors under '<layer>.<name>')."""
    F = torch.nn.functional
    x = torch.from_numpy(np.asarray(img, np.float64))
    mean = torch.tensor(c.chan_mean, dtype=torch.float64)[:, None, None]
    std = torch.tensor(c.chan_std, dtype=torch.float64)[:, None, None]
    x = (x - mean) / std
    t = F.conv2d(x[None], tp["patch_w"], tp["patch_b"], stride=c.patch)[0]
    gh, gw = t.shape[1], t.shape[2]
    D = c.width
    grid = tp["pos"][1:].reshape(c.base_grid, c.base_grid, D).permute(2, 0, 1)[None]
    if (gh, gw) != (c.base_grid, c.base_grid):
        grid = F.interpolate(grid, size=(gh, gw), mode="bilinear", align_corners=False)
    pos = torch.cat([tp["pos"][:1], grid[0].permute(1, 2, 0).reshape(gh * gw, D)])
    t = torch.cat([tp["cls"][None], t.flatten(1).T]) + pos
    d = D // c.heads
    for l in range(c.layers):
        g = lambda n: tp[f"{l}.{n}"]  # noqa: E731
        y = F.layer_norm(t, (D,), g("ln1_g"), g("ln1_b"), c.ln_eps)
        qkv = F.linear(y, g("qkv_w"), g("qkv_b"))
        q, k, v = qkv.split(D, dim=1)
        heads = []
        for h in range(c.heads):
            sl = slice(h * d, (h + 1) * d)
            a = torch.softmax(q[:, sl] @ k[:, sl].T / math.sqrt(d), dim=-1)
            heads.append(a @ v[:, sl])
        t = t + F.linear(torch.cat(heads, dim=1), g("o_w"), g("o_b"))
        y = F.layer_norm(t, (D,), g("ln2_g"), g("ln2_b"), c.ln_eps)
        t = t + F.linear(F.gelu(F.linear(y, g("fc1_w"), g("fc1_b"))), g("fc2_w"), g("fc2_b"))
    if getattr(c, "pool", "cls") == "map":
        # attention pooling through torch's own multi-head attention, the
        # learned probe as the one query (in-projection [W_q; W_kv])
        xl = F.layer_norm(t, (D,), tp["lnf_g"], tp["lnf_b"], c.ln_eps)
        y, _ = F.multi_head_attention_forward(
            tp["map_probe"][None, None], xl[:, None], xl[:, None], D, c.heads,
            torch.cat([tp["map_q_w"], tp["map_kv_w"]]), torch.cat([tp["map_q_b"], tp["map_kv_b"]]),
            None, None, False, 0.0, tp["map_o_w"], tp["map_o_b"], training=False,
            need_weights=False)
        y = y[0, 0]
        zl = F.layer_norm(y, (D,), tp["map_ln_g"], tp["map_ln_b"], c.ln_eps)
        z = y + F.linear(F.gelu(F.linear(zl, tp["map_fc1_w"], tp["map_fc1_b"])),
                         tp["map_fc2_w"], tp["map_fc2_b"])
    else:
        z = F.layer_norm(t[0], (D,), tp["lnf_g"], tp["lnf_b"], c.ln_eps)
    return F.normalize(tp["proj_w"] @ z, dim=0)


@pytest.mark.parametrize("pool", ["cls", "map"])
@pytest.mark.parametrize("sizes", [[(64, 64), (64, 64)], [(48, 80), (96, 64)]])
def test_backward_matches_torch_autograd(sizes, pool):
    """Every parameter gradient of sum_i <d_emb_i, e_hat_i> against float64
    autograd, at the base resolution and at two resampled grids (adjoint of
    the bilinear position resampling), with class-token pooling and with the
    attention-pooling head (autograd through torch's multi-head attention)."""
    if pool == "cls":
        c, p = _small()
    else:
        c = synth.ModelConfig("tiny_train_map", 16, 64, 2, 4, 256, 32, 4, pool="map")
        p = synth.make_params(c, 48, std=0.2)
    imgs = synth.make_images(sizes, 43)
    d_emb = _rng(44).standard_normal((len(imgs), c.proj_dim))
    layout = synth.weight_layout(c)
    flat = synth.params_to_blob(c, p).astype(np.float64)
    tp, o = {}, 0
    for name, shape in layout:
        n = int(np.prod(shape))
        tp[name] = torch.tensor(flat[o:o + n].reshape(shape), requires_grad=True)
        o += n
    loss = sum((_torch_encode(c, tp, im) * torch.from_numpy(de)).sum()
               for im, de in zip(imgs, d_emb))
    loss.backward()
    ref = np.concatenate([tp[name].grad.numpy().reshape(-1) for name, _ in layout])
    got = TR.flatten_grads(TR.encode_backward(imgs, p, c, d_emb), c, layout)
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.max(np.abs(got - ref)) <= 1e-11 * scale
    # every tensor gets a gradient that is not identically zero
    o = 0
    for name, shape in layout:
        n = int(np.prod(shape))
        assert np.abs(ref[o:o + n]).max() > 0, name
        o += n


def test_backward_central_differences():
    """Selected entries of every tensor kind against (f(w+h) - f(w-h)) / 2h of
    the oracle's own forward, f = sum_i <d_emb_i, e_hat_i>."""
    c, p = _small(layers=1)
    imgs = synth.make_images([(64, 64), (48, 64)], 45)
    d_emb = _rng(46).standard_normal((2, c.proj_dim))
    g = TR.encode_backward(imgs, p, c, d_emb)
    rng = _rng(47)

    def f(pp):
        return float((O.encode(imgs, pp, c) * d_emb).sum())

    h = 1e-6
    picks = [("patch_w", None), ("patch_b", None), ("cls", None), ("pos", None),
             ("lnf_g", None), ("proj_w", None)] + \
            [(n, 0) for n in ("ln1_g", "ln1_b", "qkv_w", "qkv_b", "o_w", "o_b", "ln2_g",
                              "fc1_w", "fc1_b", "fc2_w", "fc2_b")]
    for name, layer in picks:
        src = p if layer is None else p["layers"][layer]
        gt = g[name] if layer is None else g["layers"][layer][name]
        for _ in range(2):
            idx = tuple(int(rng.integers(0, s)) for s in np.shape(src[name]))
            pp = {k: v for k, v in p.items() if k != "layers"}
            pp["layers"] = [dict(lp) for lp in p["layers"]]
            tgt = pp if layer is None else pp["layers"][layer]
            a = np.asarray(src[name], np.float64).copy()
            a[idx] += h
            tgt[name] = a
            fp = f(pp)
            a = a.copy()
            a[idx] -= 2 * h
            tgt[name] = a
            fm = f(pp)
            fd = (fp - fm) / (2 * h)
            assert abs(fd - gt[idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, gt[idx])


def test_map_backward_central_differences():
    """Entries of every attention-pooling head tensor (and the final
    LayerNorm over all tokens it reads) against central differences of the
    oracle's own MAP forward (vit64.map_head)."""
    c = synth.ModelConfig("tiny_train_map", 16, 64, 1, 4, 256, 32, 4, pool="map")
    p = synth.make_params(c, 49, std=0.2)
    imgs = synth.make_images([(64, 64), (48, 64)], 50)
    d_emb = _rng(51).standard_normal((2, c.proj_dim))
    g = TR.encode_backward(imgs, p, c, d_emb)
    rng = _rng(52)

    def f(pp):
        return float((O.encode(imgs, pp, c) * d_emb).sum())

    h = 1e-6
    for name in ("map_probe", "map_q_w", "map_q_b", "map_kv_w", "map_kv_b", "map_o_w",
                 "map_o_b", "map_ln_g", "map_ln_b", "map_fc1_w", "map_fc1_b", "map_fc2_w",
                 "map_fc2_b", "lnf_g", "lnf_b"):
        for _ in range(2):
            idx = tuple(int(rng.integers(0, s)) for s in np.shape(p[name]))
            pp = {k: v for k, v in p.items() if k != "layers"}
            pp["layers"] = p["layers"]
            a = np.array(p[name], np.float64)
            a[idx] += h
            pp[name] = a
            fp = f(pp)
            a = a.copy()
            a[idx] -= 2 * h
            pp[name] = a
            fm = f(pp)
            fd = (fp - fm) / (2 * h)
            assert abs(fd - g[name][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, idx, fd, g[name][idx])


def test_map_forward_is_the_inference_head():
    """The backward's MAP forward computes vit64.map_head (pinned against
    torch's multi-head attention) exactly."""
    c = synth.MODELS["tiny_map"]
    p = synth.make_params(c, 53)
    x = _rng(54).standard_normal((29, c.width))
    got = TR.map_forward(x, p, c.heads, c.ln_eps)["out"]
    assert np.max(np.abs(got - O.map_head(x, p, c.heads, c.ln_eps))) <= 1e-12


def test_layernorm_backward_invariants():
    """LN is invariant to adding a constant and to a positive rescale of its
    input (up to eps), so dx sums to zero over the row and is orthogonal to
    x - mean when eps = 0."""
    rng = _rng(48)
    x = rng.standard_normal((5, 33)) * 3 + 1
    g = rng.standard_normal(33)
    dy = rng.standard_normal((5, 33))
    dx, dg, db = TR.layernorm_backward(x, g, dy, 0.0)
    assert np.max(np.abs(dx.sum(axis=1))) <= 1e-13
    xc = x - x.mean(axis=1, keepdims=True)
    assert np.max(np.abs((dx * xc).sum(axis=1))) <= 1e-12
    np.testing.assert_allclose(db, dy.sum(axis=0), rtol=0, atol=1e-14)


def test_attention_backward_invariants():
    """Softmax ignores a per-row shift of the scores, so dS rows sum to zero:
    then sum_j dK_j = 0 for every head; identical keys give uniform
    attention, whose dQ vanishes."""
    rng = _rng(49)
    q, k, v = (rng.standard_normal((7, 8)) for _ in range(3))
    do = rng.standard_normal((7, 8))
    dq, dk, dv = TR.attention_head_backward(q, k, v, do)
    assert np.max(np.abs(dk.sum(axis=0))) <= 1e-12
    np.testing.assert_allclose(dv.sum(axis=0), do.sum(axis=0), rtol=0, atol=1e-12)
    k_same = np.repeat(k[:1], 7, axis=0)
    dq2, _, _ = TR.attention_head_backward(q, k_same, v, do)
    assert np.max(np.abs(dq2)) <= 1e-13


def test_gelu_grad_textbook_values_and_identity():
    """GELU'(z) = Phi(z) + z phi(z): GELU'(0) = 1/2; GELU'(1) = Phi(1) +
    phi(1) with the tabulated Phi(1) = 0.8413447460685429 and phi(1) =
    e^(-1/2) / sqrt(2 pi) = 0.24197072451914337; GELU(z) - GELU(-z) = z gives
    GELU'(z) + GELU'(-z) = 1."""
    assert TR.gelu_grad(np.array([0.0]))[0] == 0.5
    assert abs(TR.gelu_grad(np.array([1.0]))[0] - (0.8413447460685429 + 0.24197072451914337)) \
        <= 1e-15
    z = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(TR.gelu_grad(z) + TR.gelu_grad(-z), 1.0, rtol=0, atol=1e-15)


def test_training_step_composes_loss_gradients():
    """training_step = contrastive loss of the encoder's embeddings, with the
    embedding gradient pushed through the encoder backward."""
    c, p = _small(layers=1)
    imgs = synth.make_images([(64, 64)] * 3, 50)
    texts = synth.make_texts(3, c.proj_dim, 51)
    loss, g, dt, ds, db = TR.training_step(imgs, p, c, texts, "sigmoid", 10.0, -10.0)
    emb = O.encode(imgs, p, c)
    assert loss == O.contrastive_loss(emb, texts, "sigmoid", 10.0, -10.0)
    de, dt2, ds2, db2 = O.contrastive_grads(emb, texts, "sigmoid", 10.0, -10.0)
    np.testing.assert_array_equal(dt, dt2)
    ref = TR.encode_backward(imgs, p, c, de)
    np.testing.assert_array_equal(g["proj_w"], ref["proj_w"])
