"""Pins of the FP64 oracle against things other than itself: textbook values,
closed forms, invariants, library routines (PyTorch CPU float64 modules) and
brute force on tiny inputs.  CPU only."""
import math
import os

import numpy as np
import pytest
import torch

import synth
from oracle import vit64 as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(autouse=True, scope="module")
def _float64_default():
    """torch modules built in these pins default to float64; restored after,
    so other test modules keep torch's float32 default."""
    old = torch.get_default_dtype()
    torch.set_default_dtype(torch.float64)
    yield
    torch.set_default_dtype(old)


def _rng(seed=0):
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------- GELU
def test_gelu_textbook_table():
    rows = [l.split() for l in open(os.path.join(GOLD, "normal_cdf.txt"))
            if l.strip() and not l.startswith("#")]
    for xs, phis in rows:
        x, phi = float(xs), float(phis)
        assert abs(O.gelu(np.array([x]))[0] - x * phi) <= 1e-14
        # GELU(x) - GELU(-x) = x * (Phi(x) + Phi(-x) - 1 + 1) = x
        assert abs(O.gelu(np.array([x]))[0] - O.gelu(np.array([-x]))[0] - x) <= 1e-14
    assert O.gelu(np.array([0.0]))[0] == 0.0
    assert abs(O.gelu(np.array([-1.0]))[0] + 0.15865525393145707) <= 1e-15


def test_gelu_matches_torch_erf_form():
    x = _rng(1).standard_normal(10000) * 4
    ref = torch.nn.functional.gelu(torch.from_numpy(x), approximate="none").numpy()
    assert np.max(np.abs(O.gelu(x) - ref)) <= 1e-14
    # and differs from the tanh form by far more than the FP32 tolerance
    tanh = torch.nn.functional.gelu(torch.from_numpy(x), approximate="tanh").numpy()
    assert np.max(np.abs(O.gelu(x) - tanh)) > 1e-4


# ---------------------------------------------------------------- LayerNorm
def test_layernorm_moments_closed_form():
    rng = _rng(2)
    x = rng.standard_normal((64, 96)) * 3 + 1.5
    eps = 1e-5
    y = O.layernorm(x, np.ones(96), np.zeros(96), eps)
    var_in = x.var(axis=1)
    assert np.max(np.abs(y.mean(axis=1))) <= 1e-14 * 10
    # biased variance of the output is sigma^2 / (sigma^2 + eps) exactly
    np.testing.assert_allclose(y.var(axis=1), var_in / (var_in + eps), rtol=1e-13)


def test_layernorm_affine_invariance_and_torch():
    rng = _rng(3)
    x = rng.standard_normal((32, 128))
    g = rng.standard_normal(128)
    b = rng.standard_normal(128)
    a = O.layernorm(x, g, b, 0.0)
    assert np.max(np.abs(O.layernorm(7.0 * x + 3.0, g, b, 0.0) - a)) <= 1e-12
    ref = torch.nn.functional.layer_norm(torch.from_numpy(x), (128,), torch.from_numpy(g),
                                         torch.from_numpy(b), 1e-5).numpy()
    assert np.max(np.abs(O.layernorm(x, g, b, 1e-5) - ref)) <= 1e-13


# ------------------------------------------------------------------ softmax
def test_softmax_rows_and_shift():
    rng = _rng(4)
    x = rng.standard_normal((50, 300)) * 30
    p = O.softmax(x)
    assert np.max(np.abs(p.sum(axis=1) - 1)) <= 1e-14
    assert np.max(np.abs(O.softmax(x + 123.0) - p)) <= 1e-13  # x + 123 itself rounds
    ref = torch.softmax(torch.from_numpy(x), dim=1).numpy()
    assert np.max(np.abs(p - ref)) <= 1e-15
    # scale 100 logits would overflow exp() without the max subtraction
    big = np.array([[100.0, 99.0, -100.0]])
    assert np.isfinite(O.softmax(big * 10)).all()


# ---------------------------------------------------------------- attention
def test_attention_two_tokens_one_head_by_hand():
    rng = _rng(5)
    d = 8
    q, k, v = rng.standard_normal((3, 2, d))
    s11 = q[0] @ k[0] / math.sqrt(d)
    s12 = q[0] @ k[1] / math.sqrt(d)
    p11 = 1.0 / (1.0 + math.exp(-(s11 - s12)))
    o1 = p11 * v[0] + (1 - p11) * v[1]
    out = O.attention_head(q, k, v)
    assert np.max(np.abs(out[0] - o1)) <= 1e-15


def test_attention_identical_tokens_uniform():
    rng = _rng(6)
    n, dm, heads = 9, 32, 4
    tok = rng.standard_normal(dm)
    y = np.tile(tok, (n, 1))
    qkv_w = rng.standard_normal((3 * dm, dm))
    qkv_b = rng.standard_normal(3 * dm)
    o_w = rng.standard_normal((dm, dm))
    o_b = rng.standard_normal(dm)
    out = O.mhsa(y, qkv_w, qkv_b, o_w, o_b, heads)
    v = tok @ qkv_w[2 * dm:].T + qkv_b[2 * dm:]
    np.testing.assert_allclose(out, np.tile(v @ o_w.T + o_b, (n, 1)), rtol=1e-12, atol=1e-12)
    # W_q = W_k = 0, b_q = b_k = 0: uniform weights 1/N for distinct tokens
    y2 = rng.standard_normal((n, dm))
    w0 = qkv_w.copy()
    w0[:2 * dm] = 0
    b0 = qkv_b.copy()
    b0[:2 * dm] = 0
    out2 = O.mhsa(y2, w0, b0, o_w, o_b, heads)
    vv = y2 @ qkv_w[2 * dm:].T + qkv_b[2 * dm:]
    np.testing.assert_allclose(out2, np.tile(vv.mean(axis=0) @ o_w.T + o_b, (n, 1)),
                               rtol=1e-12, atol=1e-12)


def test_mhsa_matches_torch_multihead_attention():
    rng = _rng(7)
    n, dm, heads = 13, 48, 6
    y = rng.standard_normal((n, dm))
    qkv_w = rng.standard_normal((3 * dm, dm)) * 0.2
    qkv_b = rng.standard_normal(3 * dm) * 0.2
    o_w = rng.standard_normal((dm, dm)) * 0.2
    o_b = rng.standard_normal(dm) * 0.2
    m = torch.nn.MultiheadAttention(dm, heads, batch_first=True)
    with torch.no_grad():
        m.in_proj_weight.copy_(torch.from_numpy(qkv_w))
        m.in_proj_bias.copy_(torch.from_numpy(qkv_b))
        m.out_proj.weight.copy_(torch.from_numpy(o_w))
        m.out_proj.bias.copy_(torch.from_numpy(o_b))
        t = torch.from_numpy(y)[None]
        ref = m(t, t, t, need_weights=False)[0][0].numpy()
    assert np.max(np.abs(O.mhsa(y, qkv_w, qkv_b, o_w, o_b, heads) - ref)) <= 1e-12


def test_block_matches_torch_pre_ln_encoder_layer():
    c = synth.MODELS["tiny"]
    p = synth.make_params(c, 11, std=0.2)
    lp = p["layers"][0]
    x = _rng(8).standard_normal((17, c.width))
    layer = torch.nn.TransformerEncoderLayer(
        c.width, c.heads, c.mlp, dropout=0.0, activation="gelu",
        layer_norm_eps=c.ln_eps, batch_first=True, norm_first=True)
    layer.eval()
    f = lambda a: torch.from_numpy(np.asarray(a, np.float64))  # noqa: E731
    with torch.no_grad():
        layer.self_attn.in_proj_weight.copy_(f(lp["qkv_w"]))
        layer.self_attn.in_proj_bias.copy_(f(lp["qkv_b"]))
        layer.self_attn.out_proj.weight.copy_(f(lp["o_w"]))
        layer.self_attn.out_proj.bias.copy_(f(lp["o_b"]))
        layer.linear1.weight.copy_(f(lp["fc1_w"]))
        layer.linear1.bias.copy_(f(lp["fc1_b"]))
        layer.linear2.weight.copy_(f(lp["fc2_w"]))
        layer.linear2.bias.copy_(f(lp["fc2_b"]))
        layer.norm1.weight.copy_(f(lp["ln1_g"]))
        layer.norm1.bias.copy_(f(lp["ln1_b"]))
        layer.norm2.weight.copy_(f(lp["ln2_g"]))
        layer.norm2.bias.copy_(f(lp["ln2_b"]))
        ref = layer(torch.from_numpy(x)[None])[0].numpy()
    out = O.block(x, lp, c.heads, c.ln_eps)
    assert np.max(np.abs(out - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())


# ----------------------------------------------------------------- patchify
def test_patchify_conv_loops_equal_unfold_gemm_and_torch_conv():
    rng = _rng(9)
    P, D = 4, 5
    img = rng.standard_normal((3, 13, 10))          # ragged: 3x2 grid, extra pixels
    w = rng.standard_normal((D, 3, P, P))
    b = rng.standard_normal(D)
    gemm = O.patch_embed(img, w, b, P)
    loops = O.patch_embed_conv(img, w, b, P)
    assert gemm.shape == (6, D)
    assert np.max(np.abs(gemm - loops)) <= 1e-13 * np.abs(loops).max()
    ref = torch.nn.functional.conv2d(torch.from_numpy(img)[None], torch.from_numpy(w),
                                     torch.from_numpy(b), stride=P)[0]
    ref = ref.permute(1, 2, 0).reshape(-1, D).numpy()
    assert np.max(np.abs(gemm - ref)) <= 1e-13 * np.abs(ref).max()


def test_patch_vector_order_is_channel_major():
    P = 2
    img = np.arange(3 * 4 * 4, dtype=np.float64).reshape(3, 4, 4)
    u = O.patchify(img, P)
    # patch (r=0, q=1): channel 0 rows 0..1, cols 2..3, then channel 1, ...
    assert list(u[1][:4]) == [2.0, 3.0, 6.0, 7.0]
    assert u[1][4] == 16 + 2.0


def test_normalisation_fold_closed_form():
    """Folding (x - mu)/sigma into the patch weights is exact in real
    arithmetic: W' = W / sigma_c, b' = b - sum W * mu_c / sigma_c."""
    rng = _rng(10)
    P, D = 4, 6
    img = rng.random((3, 8, 8))
    w = rng.standard_normal((D, 3, P, P))
    b = rng.standard_normal(D)
    mu = np.array([0.5, 0.4, 0.3])
    sd = np.array([0.29, 0.25, 0.2])
    ref = O.patch_embed(O.normalise_pixels(img, mu, sd), w, b, P)
    w2 = w / sd[None, :, None, None]
    b2 = b - (w * (mu / sd)[None, :, None, None]).sum(axis=(1, 2, 3))
    assert np.max(np.abs(O.patch_embed(img, w2, b2, P) - ref)) <= 1e-13 * np.abs(ref).max()


# ------------------------------------------------------------ position interp
def test_pos_interp_identity_constant_and_torch_bilinear():
    rng = _rng(11)
    g0, D = 5, 7
    pos = rng.standard_normal((1 + g0 * g0, D))
    assert np.array_equal(O.interp_pos(pos, g0, g0, g0), pos)
    const = np.ones((1 + g0 * g0, D)) * 2.5
    np.testing.assert_allclose(O.interp_pos(const, g0, 9, 3), 2.5, rtol=0, atol=1e-15)
    for gh, gw in [(9, 9), (3, 7), (8, 5), (2, 2)]:
        out = O.interp_pos(pos, g0, gh, gw)
        grid = torch.from_numpy(pos[1:].reshape(g0, g0, D)).permute(2, 0, 1)[None]
        ref = torch.nn.functional.interpolate(grid, size=(gh, gw), mode="bilinear",
                                              align_corners=False, antialias=False)
        ref = ref[0].permute(1, 2, 0).reshape(gh * gw, D).numpy()
        assert np.max(np.abs(out[1:] - ref)) <= 1e-14
        assert np.array_equal(out[0], pos[0])


def test_pos_interp_reproduces_linear_ramp_in_interior():
    g0, g = 6, 11
    r = np.arange(g0, dtype=np.float64)
    ramp = (2.0 * r[:, None] - 3.0 * r[None, :]).reshape(-1, 1)
    pos = np.concatenate([[[0.0]], ramp])
    out = O.interp_pos(pos, g0, g, g)[1:].reshape(g, g)
    for o in range(g):
        s = (o + 0.5) * g0 / g - 0.5
        if 0 <= s <= g0 - 1:
            for q in range(g):
                t = (q + 0.5) * g0 / g - 0.5
                if 0 <= t <= g0 - 1:
                    assert abs(out[o, q] - (2 * s - 3 * t)) <= 1e-13


# ------------------------------------------------------------- whole encoder
def _tiny_setup(seed=12, model="tiny"):
    c = synth.MODELS[model]
    p = synth.make_params(c, seed)
    imgs = synth.make_images([(64, 64)] * 3, seed + 1, channels=c.channels)
    return c, p, imgs


def test_zero_block_model_closed_form():
    c, p, imgs = _tiny_setup()
    for lp in p["layers"]:
        for k in list(lp):
            lp[k] = np.zeros_like(lp[k])
    z = O.layernorm(np.asarray(p["cls"], np.float64) + p["pos"][0], p["lnf_g"], p["lnf_b"])
    e = p["proj_w"].astype(np.float64) @ z
    e /= np.linalg.norm(e)
    for im in imgs:
        assert np.max(np.abs(O.encode_image(im, p, c) - e)) <= 1e-14


def test_permutation_equivariance_with_zero_pos():
    c, p, imgs = _tiny_setup(13)
    p["pos"] = np.zeros_like(p["pos"])
    img = imgs[0]
    P = c.patch
    # swap two patches of the image: the class-token output must not change
    img2 = img.copy()
    img2[:, 0:P, 0:P], img2[:, 2 * P:3 * P, P:2 * P] = \
        img[:, 2 * P:3 * P, P:2 * P].copy(), img[:, 0:P, 0:P].copy()
    a = O.encode_image(img, p, c)
    b = O.encode_image(img2, p, c)
    assert np.max(np.abs(a - b)) <= 1e-12
    assert np.max(np.abs(a - O.encode_image(imgs[1], p, c))) > 1e-3


def test_embeddings_unit_norm_and_not_degenerate():
    c, p, imgs = _tiny_setup(14)
    e = O.encode(imgs, p, c)
    np.testing.assert_allclose(np.linalg.norm(e, axis=1), 1.0, rtol=0, atol=1e-15)
    cos = e @ e.T
    off = cos[~np.eye(len(e), dtype=bool)]
    assert off.max() < 0.99, "different images must not collapse to one embedding"


@pytest.mark.parametrize("model", ["tiny", "tiny_rgbd"])
def test_encoder_matches_torch_modules(model):
    """Whole forward against PyTorch library modules (conv patchify,
    pre-LN TransformerEncoderLayer, layer_norm, linear), all float64; RGB
    and 4-plane RGB-D inputs."""
    c, p, imgs = _tiny_setup(15, model)
    assert imgs[0].shape[0] == c.channels
    f = lambda a: torch.from_numpy(np.asarray(a, np.float64))  # noqa: E731
    layers = []
    for lp in p["layers"]:
        L = torch.nn.TransformerEncoderLayer(c.width, c.heads, c.mlp, dropout=0.0,
                                             activation="gelu", layer_norm_eps=c.ln_eps,
                                             batch_first=True, norm_first=True).eval()
        with torch.no_grad():
            L.self_attn.in_proj_weight.copy_(f(lp["qkv_w"]))
            L.self_attn.in_proj_bias.copy_(f(lp["qkv_b"]))
            L.self_attn.out_proj.weight.copy_(f(lp["o_w"]))
            L.self_attn.out_proj.bias.copy_(f(lp["o_b"]))
            L.linear1.weight.copy_(f(lp["fc1_w"]))
            L.linear1.bias.copy_(f(lp["fc1_b"]))
            L.linear2.weight.copy_(f(lp["fc2_w"]))
            L.linear2.bias.copy_(f(lp["fc2_b"]))
            L.norm1.weight.copy_(f(lp["ln1_g"]))
            L.norm1.bias.copy_(f(lp["ln1_b"]))
            L.norm2.weight.copy_(f(lp["ln2_g"]))
            L.norm2.bias.copy_(f(lp["ln2_b"]))
        layers.append(L)
    mean = torch.tensor(c.chan_mean)[:, None, None]
    std = torch.tensor(c.chan_std)[:, None, None]
    with torch.no_grad():
        for im in imgs:
            x = (f(im) - mean) / std
            t = torch.nn.functional.conv2d(x[None], f(p["patch_w"]), f(p["patch_b"]),
                                           stride=c.patch)[0]
            t = t.flatten(1).T
            t = torch.cat([f(p["cls"])[None], t]) + f(p["pos"])
            t = t[None]
            for L in layers:
                t = L(t)
            z = torch.nn.functional.layer_norm(t[0, 0], (c.width,), f(p["lnf_g"]),
                                               f(p["lnf_b"]), c.ln_eps)
            e = torch.nn.functional.normalize(z @ f(p["proj_w"]).T, dim=0).numpy()
            assert np.max(np.abs(O.encode_image(im, p, c) - e)) <= 1e-12


# ------------------------------------------------------------------- scoring
def test_score_heads_bounds_special_cases_and_ties():
    rng = _rng(16)
    e = rng.standard_normal((5, 32))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    t = rng.standard_normal((40, 32))
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    t[7] = e[2]                                   # a text equal to image 2
    p, top1 = O.score(e, t, "softmax", 100.0)
    assert np.max(np.abs(p.sum(axis=1) - 1)) <= 1e-14
    assert abs(O.logits(e, t, 100.0)[2, 7] - 100.0) <= 1e-12
    assert top1[2] == 7
    ps, top1s = O.score(e, t, "sigmoid", 10.0, -10.0)
    lo, hi = 1 / (1 + math.exp(20.0)), 0.5
    assert ps.min() >= lo - 1e-18 and ps.max() <= hi + 1e-15
    assert np.array_equal(top1, top1s)            # same ranking, monotone heads
    t2 = np.concatenate([t[:3], t[:3]])           # exact ties -> lowest index
    assert (O.score(e, t2, "softmax", 100.0)[1] < 3).all()


# ------------------------------------------------------------ number formats
def test_bf16_round_matches_torch():
    rng = _rng(17)
    x = np.concatenate([rng.standard_normal(200000).astype(np.float32) * 10,
                        np.array([0.0, -0.0, 1.0, 65504.0, 3.0e38, 1e-40, -1e-38],
                                 np.float32)])
    bits = rng.integers(0, 2 ** 32, size=200000, dtype=np.uint64).astype(np.uint32)
    y = bits.view(np.float32)
    y = y[np.isfinite(y)]
    for arr in (x, y):
        ref = torch.from_numpy(arr).to(torch.bfloat16).to(torch.float64).numpy()
        got = O.bf16_round(arr)
        finite = np.isfinite(ref)
        assert np.array_equal(got[finite], ref[finite])
    # exact tie cases: 1 + 2^-8 rounds to even (1.0), 1 + 3*2^-8 rounds up
    assert O.bf16_round(np.array([1 + 2 ** -8], np.float32))[0] == 1.0
    assert O.bf16_round(np.array([1 + 3 * 2 ** -8], np.float32))[0] == 1 + 2 ** -6


def test_e4m3_landmarks_and_grid_vs_torch():
    rows = [l.split() for l in open(os.path.join(GOLD, "e4m3fn_points.txt"))
            if l.strip() and not l.startswith("#")]
    codes = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64)
    for hx, val, _ in rows:
        v = float(val)
        assert codes[int(hx, 16)].item() == v
        assert O.e4m3_round(np.array([v]))[0] == v
    grid = codes.numpy()
    grid = np.unique(grid[np.isfinite(grid)])
    assert grid.max() == 448.0 and len(grid) == 253   # 126 pos, 126 neg, one zero
    # every representable value is a fixed point
    assert np.array_equal(O.e4m3_round(grid), grid)
    # random values: nearest grid point, ties to even code, vs torch's cast
    rng = _rng(18)
    y = np.concatenate([rng.standard_normal(100000) * 50, rng.standard_normal(20000) * 0.01,
                        (grid[:-1] + grid[1:]) / 2])
    y = y[np.abs(y) <= 448]
    ref = torch.from_numpy(y.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(O.e4m3_round(y.astype(np.float32)), ref)
    assert O.e4m3_round(np.array([1000.0, -500.0]))[0] == 448.0
    assert O.e4m3_round(np.array([-500.0]))[0] == -448.0


def test_fp8_row_quantiser_properties():
    rng = _rng(19)
    w = (rng.standard_normal((64, 200)) * 0.02).astype(np.float32)
    q, s = O.quantise_fp8_rows(w)
    amax_idx = np.abs(w).argmax(axis=1)
    assert np.all(np.abs(q[np.arange(64), amax_idx]) == 448.0)
    assert np.abs(q).max() <= 448.0
    deq = q * s[:, None]
    y = np.abs(w / s[:, None])
    normal = y >= 2.0 ** -6
    err = np.abs(deq - w)
    assert np.all(err[normal] <= 2.0 ** -4 * np.abs(w)[normal] * (1 + 1e-6))
    assert np.all(err[~normal] <= (s[:, None] * 2.0 ** -10 * (1 + 1e-6)).repeat(200, 1)[~normal])
    # round trip of values already on the grid is exact
    q2, s2 = O.quantise_fp8_rows((q * s[:, None]).astype(np.float32))
    assert np.allclose(q2 * s2[:, None], q * s[:, None], rtol=1e-6, atol=0)


def test_weights_for_only_touches_block_linears():
    c = synth.MODELS["tiny"]
    p = synth.make_params(c, 20)
    for prec in ("bf16", "fp8w"):
        w = O.weights_for(p, prec)
        assert np.array_equal(w["patch_w"], p["patch_w"])
        assert np.array_equal(w["layers"][0]["qkv_b"], p["layers"][0]["qkv_b"])
        assert not np.array_equal(w["layers"][0]["qkv_w"], p["layers"][0]["qkv_w"])
        rel = np.abs(w["layers"][1]["fc1_w"] - p["layers"][1]["fc1_w"]) / \
            np.abs(p["layers"][1]["fc1_w"]).max()
        assert rel.max() < (2 ** -8 if prec == "bf16" else 2 ** -4)


def test_weights_for_map_head_rounds_only_kv_projection():
    """With an attention-pooling head, every reduced precision rounds the
    head's K/V projection (and only it) to BF16 -- checked against torch's
    own BF16 cast, not the oracle's rounding -- while FP32 leaves it as is."""
    c = synth.MODELS["tiny_map"]
    p = synth.make_params(c, 21)
    want = torch.from_numpy(np.asarray(p["map_kv_w"], np.float32)).to(torch.bfloat16)
    want = want.to(torch.float64).numpy()
    head = [k for k in p if k.startswith("map_")]
    assert "map_kv_w" in head and len(head) == 13
    for prec in ("bf16", "fp8w", "mxfp8"):
        w = O.weights_for(p, prec)
        assert np.array_equal(w["map_kv_w"], want), prec
        assert not np.array_equal(w["map_kv_w"], p["map_kv_w"])
        for k in head:
            if k != "map_kv_w":
                assert np.array_equal(w[k], p[k]), (prec, k)
    w = O.weights_for(p, "fp32")
    for k in head:
        assert np.array_equal(w[k], p[k]), k


# ------------------------------------------ MXFP8 (OCP Microscaling Formats)
def test_mx_hand_worked_block():
    # amax 1.0: floor(log2) = 0, X = 0 - 8; elements are v * 2^8 rounded on
    # the e4m3 grid: 1.0 -> 256 exactly; 0.9 -> 230.4 in [128, 256), step 16
    # -> 224; -0.3 -> -76.8 in [64, 128), step 8 -> -80; 1e-4 -> 0.0256 in
    # [2^-6, 2^-5), step 2^-9 -> 13 * 2^-9.
    x = np.zeros(32)
    x[:4] = [1.0, 0.9, -0.3, 1e-4]
    q, X = O.mx_quantise(x)
    assert X.tolist() == [-8]
    assert q[0, :4].tolist() == [256.0, 224.0, -80.0, 13 * 2.0 ** -9]
    assert not q[0, 4:].any()
    assert O.mx_round(x)[:3].tolist() == [1.0, 0.875, -0.3125]
    # amax 1.9: still X = -8, and 1.9 * 256 = 486.4 saturates to 448 (1.75)
    x[0] = 1.9
    assert O.mx_round(x)[0] == 1.75
    # all-zero blocks take the least scale and stay zero
    q, X = O.mx_quantise(np.zeros((2, 64)))
    assert X.tolist() == [[-127, -127], [-127, -127]] and not q.any()
    with pytest.raises(ValueError):
        O.mx_quantise(np.zeros(48))


def test_mx_exponent_bruteforce_and_elements_vs_torch_cast():
    rng = _rng(30)
    x = rng.standard_normal((64, 256)) * np.exp(rng.uniform(-8, 8, (64, 1)))
    x[3, 32:64] = 0.0                       # zero block
    x[5, :32] *= 1e-37                      # shared exponent below -127: clamped
    x[6, 64:96] = 0.0
    x[6, 70] = -3.0                         # one non-zero element
    x = x.astype(np.float32).astype(np.float64)
    q, X = O.mx_quantise(x)
    xb = x.reshape(64, 8, 32)
    for r in range(64):
        for b in range(8):
            amax = np.abs(xb[r, b]).max()
            if amax == 0:
                assert X[r, b] == -127
                continue
            e = -200                        # 2^e <= amax < 2^(e+1), by search
            while math.ldexp(1.0, e + 1) <= amax:
                e += 1
            assert X[r, b] == max(e - 8, -127), (r, b)
    assert X[5, 0] == -127 and X[6, 2] == 1 - 8
    y = np.clip(xb / np.ldexp(1.0, X)[..., None], -448, 448).astype(np.float32)
    ref = torch.from_numpy(y).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(q, ref)


def test_mx_grid_fixed_points_equivariance_idempotence_and_error_bound():
    rng = _rng(31)
    codes = np.arange(256)
    grid = O.e4m3_value(codes[(codes & 0x7F) != 0x7F])
    for k in (-20, 0, 7):
        blk = np.concatenate([rng.choice(grid, size=(16, 31)), np.full((16, 1), 448.0)], axis=1)
        blk = np.ldexp(blk, k)
        assert np.array_equal(O.mx_round(blk), blk)       # X = k: every value on the grid
    x = rng.standard_normal((32, 512)) * 3.0
    r = O.mx_round(x)
    for k in (-7, 1, 30):
        assert np.array_equal(O.mx_round(np.ldexp(x, k)), np.ldexp(r, k))
    assert np.array_equal(O.mx_round(r), r)
    q, X = O.mx_quantise(x)
    s = np.ldexp(1.0, X)[..., None]
    xb = x.reshape(q.shape)
    sat = np.abs(xb) > 448 * s
    err = np.abs(q * s - xb)
    bound = np.maximum(2.0 ** -4 * np.abs(xb), s * 2.0 ** -10)
    assert np.all(err[~sat] <= bound[~sat])
    assert np.all(np.abs(q[sat]) == 448.0)
    assert sat.any()                                      # saturation does occur


def test_e4m3_codes_round_trip_and_match_torch():
    codes = np.arange(256)
    codes = codes[(codes & 0x7F) != 0x7F]
    v = O.e4m3_value(codes)
    ref = torch.from_numpy(codes.astype(np.uint8)).view(torch.float8_e4m3fn).to(torch.float64)
    assert np.array_equal(v, ref.numpy())
    assert np.array_equal(O.e4m3_code(v), codes.astype(np.uint8))
    assert O.e4m3_code(np.array([-0.0]))[0] == 0x80
    rows = [l.split() for l in open(os.path.join(GOLD, "e4m3fn_points.txt"))
            if l.strip() and not l.startswith("#")]
    for hx, val, _ in rows:
        assert O.e4m3_value(np.array([int(hx, 16)]))[0] == float(val)
    with pytest.raises(ValueError):
        O.e4m3_value(np.array([0x7F]))


def test_activation_hook_sits_on_every_linear_input():
    # With a map that zeroes every linear input, attention sees Q = K = V =
    # bias rows and both projections reduce to their biases, so a block is
    # x + o_b + fc2_b; a missed or misplaced hook would leave a data term.
    rng = _rng(32)
    d, f, t = 64, 128, 5
    lp = {"ln1_g": rng.standard_normal(d), "ln1_b": rng.standard_normal(d),
          "qkv_w": rng.standard_normal((3 * d, d)), "qkv_b": rng.standard_normal(3 * d),
          "o_w": rng.standard_normal((d, d)), "o_b": rng.standard_normal(d),
          "ln2_g": rng.standard_normal(d), "ln2_b": rng.standard_normal(d),
          "fc1_w": rng.standard_normal((f, d)), "fc1_b": rng.standard_normal(f),
          "fc2_w": rng.standard_normal((d, f)), "fc2_b": rng.standard_normal(d)}
    x = rng.standard_normal((t, d))
    got = O.block(x, lp, 2, 1e-5, aq=lambda a: 0.0 * a)
    assert np.allclose(got, x + lp["o_b"] + lp["fc2_b"], rtol=0, atol=1e-12)
    assert np.array_equal(O.block(x, lp, 2, 1e-5), O.block(x, lp, 2, 1e-5, aq=lambda a: a))


def test_mxfp8_variant_close_to_exact_but_not_equal():
    c = synth.MODELS["tiny"]
    p = synth.make_params(c, 33)
    imgs = synth.make_images([(c.patch * 4, c.patch * 3)] * 2, 34)
    exact = O.encode(imgs, p, c)
    mxw = O.weights_for(p, "mxfp8")
    got = O.encode(imgs, mxw, c, act="mx")
    cos = np.sum(got * exact, axis=1)
    assert np.all(cos > 0.99) and np.all(cos < 1 - 1e-9)
    w = mxw["layers"][0]["fc1_w"]
    assert np.array_equal(O.mx_round(w), w)              # weights on the MX grid


def test_mx_decode_inverts_quantise():
    rng = _rng(35)
    x = rng.standard_normal((8, 128)) * 5.0
    q, X = O.mx_quantise(x)
    assert np.array_equal(O.mx_decode(O.e4m3_code(q).reshape(8, 128), X), O.mx_round(x))
    # one block, by hand: code 0x38 is 1.0, 0xC0 is -2.0; X = 3 scales by 8
    c = np.zeros((1, 32), np.uint8)
    c[0, 0], c[0, 31] = 0x38, 0xC0
    v = O.mx_decode(c, np.array([[3]]))
    assert v[0, 0] == 8.0 and v[0, 31] == -16.0 and not v[0, 1:31].any()


# ----------------------------------------------------------------- text tower
def _text_setup(seed):
    c = synth.TEXT_MODELS["tiny_text"]
    p = synth.text_blob_to_params(c, synth.make_text_blob(c, seed))
    return c, p


def test_causal_attention_bruteforce_rows():
    # row i by hand: softmax over the prefix 0..i only
    rng = _rng(40)
    n, d = 7, 8
    q, k, v = (rng.standard_normal((n, d)) for _ in range(3))
    got = O.causal_attention_head(q, k, v)
    for i in range(n):
        s = np.array([q[i] @ k[j] / math.sqrt(d) for j in range(i + 1)])
        w = np.exp(s - s.max())
        w /= w.sum()
        assert np.allclose(got[i], sum(w[j] * v[j] for j in range(i + 1)), rtol=0, atol=1e-14)
    assert np.array_equal(got[0], v[0])          # token 0 sees only itself


def test_text_tower_matches_torch_causal_layers():
    """Text tower against PyTorch modules: embedding lookup, pre-LN
    TransformerEncoderLayer with the square subsequent (causal) mask,
    layer_norm of the last token, linear projection; float64."""
    c, p = _text_setup(41)
    f = lambda a: torch.from_numpy(np.asarray(a, np.float64))  # noqa: E731
    layers = []
    for lp in p["layers"]:
        L = torch.nn.TransformerEncoderLayer(c.width, c.heads, c.mlp, dropout=0.0,
                                             activation="gelu", layer_norm_eps=c.ln_eps,
                                             batch_first=True, norm_first=True).eval()
        with torch.no_grad():
            L.self_attn.in_proj_weight.copy_(f(lp["qkv_w"]))
            L.self_attn.in_proj_bias.copy_(f(lp["qkv_b"]))
            L.self_attn.out_proj.weight.copy_(f(lp["o_w"]))
            L.self_attn.out_proj.bias.copy_(f(lp["o_b"]))
            L.linear1.weight.copy_(f(lp["fc1_w"]))
            L.linear1.bias.copy_(f(lp["fc1_b"]))
            L.linear2.weight.copy_(f(lp["fc2_w"]))
            L.linear2.bias.copy_(f(lp["fc2_b"]))
            L.norm1.weight.copy_(f(lp["ln1_g"]))
            L.norm1.bias.copy_(f(lp["ln1_b"]))
            L.norm2.weight.copy_(f(lp["ln2_g"]))
            L.norm2.bias.copy_(f(lp["ln2_b"]))
        layers.append(L)
    emb = torch.nn.Embedding(c.vocab, c.width)
    with torch.no_grad():
        emb.weight.copy_(f(p["tok_emb"]))
    for ids in synth.make_token_ids([1, 6, 19, c.ctx], c.vocab, 42):
        n = len(ids)
        mask = torch.nn.Transformer.generate_square_subsequent_mask(n, dtype=torch.float64)
        with torch.no_grad():
            t = (emb(torch.from_numpy(ids.astype(np.int64))) + f(p["pos"])[:n])[None]
            for L in layers:
                t = L(t, src_mask=mask, is_causal=True)
            z = torch.nn.functional.layer_norm(t[0, -1], (c.width,), f(p["lnf_g"]),
                                               f(p["lnf_b"]), c.ln_eps)
            e = torch.nn.functional.linear(z, f(p["proj_w"]))
            e = (e / e.norm()).numpy()
        assert np.max(np.abs(O.encode_text(ids, p, c) - e)) <= 1e-12


def test_text_prefix_invariance_and_last_token_pooling():
    # causal: a prefix's hidden states do not depend on later tokens, so the
    # embedding of a prefix equals pooling the full sequence at its end
    c, p = _text_setup(43)
    ids = synth.make_token_ids([30], c.vocab, 44)[0]
    full = O.text_hidden(ids, p, c)
    for k in (1, 2, 11, 29):
        assert np.allclose(O.text_hidden(ids[:k], p, c), full[:k], rtol=0, atol=1e-13)
        z = O.layernorm(full[k - 1], p["lnf_g"], p["lnf_b"], c.ln_eps)
        e = np.asarray(p["proj_w"], np.float64) @ z
        assert np.allclose(O.encode_text(ids[:k], p, c), e / np.linalg.norm(e), atol=1e-13)
    # and the later tokens do change the last position (not vacuous)
    other = ids.copy()
    other[5] = (other[5] + 1) % (c.vocab - 2)
    assert not np.allclose(O.text_hidden(other, p, c)[-1], full[-1], atol=1e-6)
    assert np.allclose(O.text_hidden(other, p, c)[:5], full[:5], rtol=0, atol=1e-13)


# ------------------------------------------------------ attention pooling (MAP)
def test_map_head_matches_torch_multihead_attention():
    c = synth.MODELS["tiny_map"]
    p = synth.make_params(c, 50)
    x = _rng(51).standard_normal((37, c.width))
    f = lambda a: torch.from_numpy(np.asarray(a, np.float64))  # noqa: E731
    mha = torch.nn.MultiheadAttention(c.width, c.heads, batch_first=True)
    with torch.no_grad():
        mha.in_proj_weight.copy_(torch.cat([f(p["map_q_w"]), f(p["map_kv_w"])]))
        mha.in_proj_bias.copy_(torch.cat([f(p["map_q_b"]), f(p["map_kv_b"])]))
        mha.out_proj.weight.copy_(f(p["map_o_w"]))
        mha.out_proj.bias.copy_(f(p["map_o_b"]))
        y, _ = mha(f(p["map_probe"])[None, None], f(x)[None], f(x)[None], need_weights=False)
        y = y[0, 0]
        z = torch.nn.functional.layer_norm(y, (c.width,), f(p["map_ln_g"]), f(p["map_ln_b"]),
                                           c.ln_eps)
        hdn = torch.nn.functional.gelu(torch.nn.functional.linear(z, f(p["map_fc1_w"]),
                                                                  f(p["map_fc1_b"])))
        ref = (y + torch.nn.functional.linear(hdn, f(p["map_fc2_w"]), f(p["map_fc2_b"]))).numpy()
    assert np.max(np.abs(O.map_head(x, p, c.heads, c.ln_eps) - ref)) <= 1e-12


def test_map_head_identical_tokens_independent_of_count():
    # uniform attention over copies of one token: the pooled vector is that
    # token's V whatever the number of copies
    c = synth.MODELS["tiny_map"]
    p = synth.make_params(c, 52)
    t = _rng(53).standard_normal(c.width)
    outs = [O.map_head(np.tile(t, (n, 1)), p, c.heads, c.ln_eps) for n in (1, 2, 17, 65)]
    for o in outs[1:]:
        assert np.allclose(o, outs[0], rtol=0, atol=1e-12)
    # the head adds exactly its own tensors to the blob
    import dataclasses
    D, F = c.width, c.mlp
    extra = D + (D * D + D) + (2 * D * D + 2 * D) + (D * D + D) + 2 * D + (F * D + F) + (D * F + D)
    assert synth.weight_count(c) - synth.weight_count(dataclasses.replace(c, pool="cls")) == extra


# -------------------------------------------------------- contrastive losses
@pytest.mark.parametrize("head", ["softmax", "sigmoid"])
def test_contrastive_grads_vs_torch_autograd_and_finite_differences(head):
    rng = _rng(60)
    n, d = 9, 16
    e = rng.standard_normal((n, d)) * 0.3
    t = rng.standard_normal((n, d)) * 0.3
    scale, bias = 7.0, -2.0
    E = torch.tensor(e, requires_grad=True)
    T = torch.tensor(t, requires_grad=True)
    s = torch.tensor(scale, requires_grad=True)
    b = torch.tensor(bias, requires_grad=True)
    l = s * E @ T.T + b
    if head == "softmax":
        tgt = torch.arange(n)
        loss = (torch.nn.functional.cross_entropy(l, tgt) +
                torch.nn.functional.cross_entropy(l.T, tgt)) / 2
    else:
        z = 2 * torch.eye(n, dtype=torch.float64) - 1
        loss = -torch.nn.functional.logsigmoid(z * l).sum() / n
    loss.backward()
    assert abs(O.contrastive_loss(e, t, head, scale, bias) - loss.item()) <= 1e-13
    de, dt, dsc, db = O.contrastive_grads(e, t, head, scale, bias)
    assert np.allclose(de, E.grad.numpy(), rtol=0, atol=1e-13)
    assert np.allclose(dt, T.grad.numpy(), rtol=0, atol=1e-13)
    assert abs(dsc - s.grad.item()) <= 1e-12 and abs(db - b.grad.item()) <= 1e-12
    # central differences on a few coordinates, independent of both
    h = 1e-6
    for (i, k) in [(0, 0), (4, 7), (8, 15)]:
        ep, em = e.copy(), e.copy()
        ep[i, k] += h
        em[i, k] -= h
        fd = (O.contrastive_loss(ep, t, head, scale, bias) -
              O.contrastive_loss(em, t, head, scale, bias)) / (2 * h)
        assert abs(fd - de[i, k]) <= 1e-7


def test_contrastive_special_cases():
    rng = _rng(61)
    e = rng.standard_normal((1, 16))
    t = rng.standard_normal((1, 16))
    # one pair: the softmax over a single logit is 1, so loss and gradient vanish
    assert O.contrastive_loss(e, t, "softmax", 10.0) == 0.0
    de, dt, dsc, _ = O.contrastive_grads(e, t, "softmax", 10.0)
    assert not de.any() and not dt.any() and dsc == 0.0
    # sigmoid with one pair: softplus(-(scale <e,t> + b))
    l = 3.0 * float(e[0] @ t[0]) + 0.5
    assert abs(O.contrastive_loss(e, t, "sigmoid", 3.0, 0.5) - math.log1p(math.exp(-l))) <= 1e-14
    # softmax ignores the bias; sigmoid does not
    e2, t2 = rng.standard_normal((5, 16)), rng.standard_normal((5, 16))
    assert abs(O.contrastive_loss(e2, t2, "softmax", 4.0, 3.0) -
               O.contrastive_loss(e2, t2, "softmax", 4.0, 0.0)) <= 1e-13
    assert O.contrastive_grads(e2, t2, "softmax", 4.0, 3.0)[3] == pytest.approx(0.0, abs=1e-15)
