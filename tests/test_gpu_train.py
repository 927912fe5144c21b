"""GPU parity of contrastive training through the image tower: the training
forward against the inference forward (bitwise), and every weight gradient of
the backward pass against the FP64 oracle's chain rule (oracle/train64.py) on
the same seeded inputs, with dL/d(embedding) from the library's contrastive
loss fed to both.

Bars: FP32 -- per tensor, max |g - g_ref| <= 1e-4 max |g_ref|; BF16 -- per
tensor cosine >= 0.999 against the oracle on the exact BF16 weights."""
import sys

import numpy as np
import pytest

import synth
from oracle import train64 as TR
from oracle import vit64 as O

from helpers import pack

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_00690_amd import vl
    vl.lib()
    return vl


# 65 tokens per image (8 x 8 patches + class token): two 64-token attention
# blocks, the second a one-token tail.
SMALL = synth.ModelConfig("train_small", patch=8, width=128, layers=2, heads=4, mlp=512,
                          proj_dim=64, base_grid=8)
SMALL_HD64 = synth.ModelConfig("train_small64", patch=8, width=128, layers=1, heads=2, mlp=256,
                               proj_dim=64, base_grid=8)
# the attention-pooling (MAP) head over every token instead of the class token
SMALL_MAP = synth.ModelConfig("train_small_map", patch=8, width=128, layers=2, heads=4, mlp=512,
                              proj_dim=64, base_grid=8, pool="map")
# one ViT-B/16-shaped block with the pooling head at 224 px: 197 tokens
B16_MAP_1 = synth.ModelConfig("b16_map_1block", patch=16, width=768, layers=1, heads=12,
                              mlp=3072, proj_dim=768, base_grid=14, pool="map")
# three blocks at widths that are multiples of 256 (the K-major weight-
# gradient path, whose LayerNorm backward also writes dX's BF16 copy)
MID3 = synth.ModelConfig("train_mid3", patch=8, width=256, layers=3, heads=4, mlp=1024,
                         proj_dim=64, base_grid=8)
# one ViT-L/14-shaped block at 336 px: 577 tokens, width 1024, 16 heads
L14_1 = synth.ModelConfig("l14_1block", patch=14, width=1024, layers=1, heads=16, mlp=4096,
                          proj_dim=768, base_grid=24)


def _run(V, cfg, seed, sizes, precision, std):
    p = synth.make_params(cfg, seed, std=std)
    blob = torch.from_numpy(synth.params_to_blob(cfg, p)).cuda()
    tr = V.Trainer(cfg, blob, precision)
    imgs = synth.make_images(sizes, seed + 1)
    pix = torch.from_numpy(pack(imgs)).cuda()
    _say(f"train {cfg.name} {precision} n={len(sizes)} size={sizes[0]}")
    emb = tr.forward(pix, sizes).clone()
    texts = torch.from_numpy(synth.make_texts(len(sizes), cfg.proj_dim, seed + 2)).cuda()
    _, de, _, _ = V.vl_contrastive_loss(emb, texts, "sigmoid", 10.0, -10.0)
    grads = tr.backward(pix, sizes, de)
    torch.cuda.synchronize()
    de64 = de.cpu().numpy().astype(np.float64)
    pw = O.weights_for(p, precision)
    ref = TR.flatten_grads(TR.encode_backward(imgs, pw, cfg, de64), cfg, synth.weight_layout(cfg))
    got = grads.cpu().numpy().astype(np.float64)
    emb_ref = O.encode(imgs, pw, cfg)
    tr.close()
    return got, ref, emb.cpu().numpy(), emb_ref


def _per_tensor(cfg, got, ref):
    o = 0
    for name, shape in synth.weight_layout(cfg):
        n = int(np.prod(shape))
        yield name, got[o:o + n], ref[o:o + n]
        o += n


def _check_fp32(cfg, got, ref):
    worst = 0.0
    for name, g, r in _per_tensor(cfg, got, ref):
        scale = np.abs(r).max()
        assert scale > 0, name
        err = np.abs(g - r).max() / scale
        worst = max(worst, err)
        assert err <= 1e-4, (name, err)
    _say(f"  fp32 worst per-tensor relative error {worst:.2e}")


def _check_bf16(cfg, got, ref):
    worst = 1.0
    for name, g, r in _per_tensor(cfg, got, ref):
        cos = float(g @ r / (np.linalg.norm(g) * np.linalg.norm(r)))
        worst = min(worst, cos)
        assert cos >= 0.999, (name, cos)
    _say(f"  bf16 worst per-tensor cosine {worst:.6f}")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_train_forward_with_pooling_head_equals_inference_bitwise(V, precision):
    """With the attention-pooling head the training forward keeps the head's
    values too and still gives vl_encode_images' embeddings bit for bit."""
    p = synth.make_params(SMALL_MAP, 66, std=0.1)
    blob = torch.from_numpy(synth.params_to_blob(SMALL_MAP, p)).cuda()
    sizes = [(64, 64)] * 5
    pix = torch.from_numpy(pack(synth.make_images(sizes, 67))).cuda()
    tr = V.Trainer(SMALL_MAP, blob, precision)
    a = tr.forward(pix, sizes).clone()
    b = tr.encode(pix, sizes).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    tr.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_backward_with_pooling_head(V, precision):
    """Every weight gradient of a tower with the attention-pooling head
    (learned query over every final-LayerNormed token): the head's tensors,
    the final LayerNorm over all tokens, and the blocks below it."""
    got, ref, emb, emb_ref = _run(V, SMALL_MAP, 68, [(64, 64)] * 5, precision, 0.1)
    if precision == "fp32":
        assert np.abs(emb - emb_ref).max() <= 1e-4
        _check_fp32(SMALL_MAP, got, ref)
    else:
        _check_bf16(SMALL_MAP, got, ref)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_backward_with_pooling_head_b16_block(V, precision):
    """The pooling head at ViT-B/16 width (768, 12 heads of 64, MLP 3072),
    three 224-px images, N(0, 0.02^2) weights."""
    got, ref, _, _ = _run(V, B16_MAP_1, 73, [(224, 224)] * 3, precision, 0.02)
    if precision == "fp32":
        _check_fp32(B16_MAP_1, got, ref)
    else:
        _check_bf16(B16_MAP_1, got, ref)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_train_forward_equals_inference_bitwise(V, precision):
    """The training forward keeps activations (including the normalised
    LayerNorm rows the weight gradients need, so its LayerNorms are not
    folded into the GEMMs) and otherwise runs the inference kernels with the
    same arithmetic: embeddings equal vl_encode_images bit for bit with the
    LayerNorm folding off (the default), and within rounding with it on."""
    p = synth.make_params(SMALL, 60, std=0.1)
    blob = torch.from_numpy(synth.params_to_blob(SMALL, p)).cuda()
    sizes = [(64, 64)] * 5
    pix = torch.from_numpy(pack(synth.make_images(sizes, 61))).cuda()
    tr = V.Trainer(SMALL, blob, precision)
    a = tr.forward(pix, sizes).clone()
    b = tr.encode(pix, sizes).clone()
    V.vl_model_set_option(tr.handle, V.VL_OPT_FUSED_LN, 1)
    folded = tr.encode(pix, sizes).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    cos = (a * folded).sum(dim=1) / (a.norm(dim=1) * folded.norm(dim=1))
    assert float(cos.min()) >= 0.9999
    tr.close()


@pytest.mark.parametrize("cfg,std", [(SMALL, 0.1), (SMALL_HD64, 0.2)])
def test_backward_fp32_small(V, cfg, std):
    """Every weight gradient, FP32, head width 32 and 64, 65-token images
    (a ragged attention tile), 5 images (ragged token count)."""
    got, ref, emb, emb_ref = _run(V, cfg, 62, [(64, 64)] * 5, "fp32", std)
    assert np.abs(emb - emb_ref).max() <= 1e-4
    _check_fp32(cfg, got, ref)


@pytest.mark.parametrize("cfg,std", [(SMALL, 0.1), (SMALL_HD64, 0.2)])
def test_backward_bf16_small(V, cfg, std):
    got, ref, _, _ = _run(V, cfg, 63, [(64, 64)] * 5, "bf16", std)
    _check_bf16(cfg, got, ref)


def test_backward_bf16_three_blocks_kmajor(V):
    """Three blocks of width 256 / MLP 1024 (the K-major weight-gradient path,
    its GEMMs on the side stream beside the next block's input-gradient
    chain), five 65-token images: every gradient against the oracle."""
    got, ref, _, _ = _run(V, MID3, 76, [(64, 64)] * 5, "bf16", 0.1)
    _check_bf16(MID3, got, ref)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_backward_l14_one_block(V, precision):
    """One ViT-L/14-shaped block at 336 px (577 tokens, ten 64-token
    attention blocks per image), two images, N(0, 0.02^2) weights."""
    got, ref, _, _ = _run(V, L14_1, 64, [(336, 336)] * 2, precision, 0.02)
    if precision == "fp32":
        _check_fp32(L14_1, got, ref)
    else:
        _check_bf16(L14_1, got, ref)


def test_backward_needs_matching_train_call(V):
    p = synth.make_params(SMALL, 65, std=0.1)
    blob = torch.from_numpy(synth.params_to_blob(SMALL, p)).cuda()
    tr = V.Trainer(SMALL, blob, "fp32")
    sizes = [(64, 64)] * 2
    pix = torch.from_numpy(pack(synth.make_images(sizes, 66))).cuda()
    de = torch.zeros((2, SMALL.proj_dim), dtype=torch.float32, device="cuda")
    with pytest.raises(V.VlError):
        tr.backward(pix, sizes, de)                      # no training forward yet
    tr.forward(pix, sizes)
    with pytest.raises(V.VlError):
        tr.backward(pix, [(64, 64)] * 1, de[:1])         # other shapes
    pix2 = torch.zeros(3 * (80 * 64 + 64 * 64), dtype=torch.float32, device="cuda")
    with pytest.raises(V.VlError):
        tr.forward(pix2, [(80, 64), (64, 64)])           # not the base grid
    tr.close()
    mx = V.Trainer(SMALL, blob, "fp8w")
    with pytest.raises(V.VlError) as ei:
        mx.forward(pix, sizes)
    mx.close()


def test_backward_kmajor_weight_gradients_match_transposed(V):
    """The weight gradients formed from the token-major operands equal those
    of the transposed-copy path (same BF16 operands, same K splits) up to
    FP32 summation order inside the matrix instructions; every other
    gradient is bitwise equal.  One ViT-L/14-shaped block (widths 1024,
    3072, 4096: the K-major path's multiples of 256), two 336-px images:
    1154 token rows, a ragged last 64-row K tile in the last split; and
    three blocks of width 256, whose weight gradients on the side stream
    overlap the next block's input-gradient chain."""
    for cfg, seed, sizes in ((L14_1, 67, [(336, 336)] * 2), (MID3, 77, [(64, 64)] * 5)):
        p = synth.make_params(cfg, seed, std=0.02 if cfg is L14_1 else 0.1)
        blob = torch.from_numpy(synth.params_to_blob(cfg, p)).cuda()
        pix = torch.from_numpy(pack(synth.make_images(sizes, seed + 1))).cuda()
        de = torch.from_numpy(synth.make_texts(len(sizes), cfg.proj_dim, seed + 2)).cuda() * 0.1
        tr = V.Trainer(cfg, blob, "bf16")
        got = {}
        for km in (1, 0):
            _say(f"train {cfg.name} bf16 kmajor={km}")
            V.vl_model_set_option(tr.handle, V.VL_OPT_KMAJOR_WGRAD, km)
            tr.forward(pix, sizes)
            got[km] = tr.backward(pix, sizes, de).clone().cpu().numpy()
        tr.close()
        block_w = {"qkv_w", "o_w", "fc1_w", "fc2_w"}
        for name, a, b in _per_tensor_pair(cfg, got[1], got[0]):
            if name.split(".")[-1] in block_w:
                scale = np.abs(b).max()
                assert scale > 0, name
                err = np.abs(a - b).max() / scale
                assert err <= 1e-5, (name, err)
            else:
                assert np.array_equal(a, b), name


def test_backward_repeats_bitwise_with_kept_transposed_weights(V):
    """A BF16 model forms its blocks' transposed weights on the first
    backward call and reuses them: the second and third calls on one model
    (the third on another stream) and a first call on a fresh model give
    the same gradients bit for bit."""
    p = synth.make_params(SMALL, 73, std=0.1)
    blob = torch.from_numpy(synth.params_to_blob(SMALL, p)).cuda()
    sizes = [(64, 64)] * 3
    pix = torch.from_numpy(pack(synth.make_images(sizes, 74))).cuda()
    de = torch.from_numpy(synth.make_texts(3, SMALL.proj_dim, 75)).cuda()
    tr = V.Trainer(SMALL, blob, "bf16")
    runs = []
    for k in range(2):
        _say(f"train {SMALL.name} bf16 repeat {k}")
        tr.forward(pix, sizes)
        runs.append(tr.backward(pix, sizes, de).clone())
    _say(f"train {SMALL.name} bf16 repeat 2, another stream")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        tr.forward(pix, sizes)
        runs.append(tr.backward(pix, sizes, de).clone())
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    tr.close()
    fresh = V.Trainer(SMALL, blob, "bf16")
    fresh.forward(pix, sizes)
    runs.append(fresh.backward(pix, sizes, de).clone())
    torch.cuda.synchronize()
    fresh.close()
    for r in runs[1:]:
        assert torch.equal(r, runs[0])


def test_training_forward_in_two_halves_is_bitwise_one_pass(V):
    """VL_OPT_SPLIT: the training forward runs the batch as two halves of
    consecutive images on two streams.  Eight 336-px images of a ViT-L/14
    block (4616 tokens, enough to split): embeddings and every gradient of
    the following backward equal the one-pass run bit for bit."""
    p = synth.make_params(L14_1, 70, std=0.02)
    blob = torch.from_numpy(synth.params_to_blob(L14_1, p)).cuda()
    sizes = [(336, 336)] * 8
    pix = torch.from_numpy(pack(synth.make_images(sizes, 71))).cuda()
    de = torch.from_numpy(synth.make_texts(8, L14_1.proj_dim, 72)).cuda() * 0.1
    out = {}
    for split in (False, True):
        _say(f"train l14_1block bf16 n=8 split={split}")
        tr = V.Trainer(L14_1, blob, "bf16", split=split)
        emb = tr.forward(pix, sizes).clone()
        grads = tr.backward(pix, sizes, de).clone()
        torch.cuda.synchronize()
        out[split] = (emb.cpu(), grads.cpu())
        tr.close()
    assert torch.equal(out[True][0], out[False][0])
    assert torch.equal(out[True][1], out[False][1])


def _per_tensor_pair(cfg, a, b):
    o = 0
    for name, shape in synth.weight_layout(cfg):
        n = int(np.prod(shape))
        yield name, a[o:o + n], b[o:o + n]
        o += n
