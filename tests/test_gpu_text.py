"""GPU parity of the text tower (causal transformer over token ids, last-token
pooling) through the C ABI against the FP64 oracle, same bars as the image
tower: FP32 relative embedding error <= 1e-4; BF16 / FP8-weight cosine >=
0.999 on the exact weights; MXFP8 by the bar relative to its own rounding."""
import sys

import numpy as np
import pytest

import synth
from oracle import vit64 as O

from helpers import cosine, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FP32_TOL = 1e-4
COS_TOL = 0.999


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


_BLOBS = {}


def blob(model, seed):
    if (model, seed) not in _BLOBS:
        _BLOBS[(model, seed)] = synth.make_text_blob(synth.TEXT_MODELS[model], seed)
    return _BLOBS[(model, seed)]


def run(enc, seqs):
    ids = torch.from_numpy(np.concatenate(seqs).astype(np.int32)).cuda()
    out = enc.encode(ids, [len(s) for s in seqs])
    torch.cuda.synchronize()
    return out.cpu().numpy()


def oracle(model, seed, precision, seqs):
    c = synth.TEXT_MODELS[model]
    p = O.weights_for(synth.text_blob_to_params(c, blob(model, seed)), precision)
    return O.encode_texts(seqs, p, c, act="mx" if precision == "mxfp8" else "none")


RAGGED = [1, 2, 5, 17, 77, 64, 33, 8]


def test_text_tiny_fp32_ragged(V):
    c = synth.TEXT_MODELS["tiny_text"]
    seqs = synth.make_token_ids(RAGGED, c.vocab, 6000)
    enc = V.TextEncoder(c, torch.from_numpy(blob("tiny_text", 7000)).cuda(), "fp32")
    got = run(enc, seqs)
    err = rel_err(got, oracle("tiny_text", 7000, "fp32", seqs))
    _say(f"  tiny text fp32 max rel err {err.max():.3e}")
    assert err.max() <= FP32_TOL
    enc.close()


@pytest.mark.parametrize("precision", ["bf16", "fp8w", "mxfp8"])
def test_text_tiny_reduced_precision(V, precision):
    c = synth.TEXT_MODELS["tiny_text"]
    seqs = synth.make_token_ids(RAGGED, c.vocab, 6001)
    enc = V.TextEncoder(c, torch.from_numpy(blob("tiny_text", 7000)).cuda(), precision)
    got = run(enc, seqs)
    ref = oracle("tiny_text", 7000, precision, seqs)
    if precision == "mxfp8":
        exact = O.encode_texts(seqs, O.weights_for(
            synth.text_blob_to_params(c, blob("tiny_text", 7000)), "mxfp8"), c)
        e_gpu, e_ref = 1 - cosine(got, exact), 1 - cosine(ref, exact)
        _say(f"  tiny text mxfp8 1-cos vs exact activations: gpu mean {e_gpu.mean():.2e}, "
             f"oracle MX mean {e_ref.mean():.2e}")
        assert e_ref.mean() > 1e-6
        assert e_gpu.mean() <= 2.0 * e_ref.mean() + 1e-4
        assert e_gpu.max() <= 4.0 * e_ref.mean() + 1e-4
    else:
        cos = cosine(got, ref)
        _say(f"  tiny text {precision} min cos {cos.min():.6f}")
        assert cos.min() >= COS_TOL
    enc.close()


def test_text_l14_bf16_sampled(V):
    """The CLIP ViT-L/14 text tower's shape (width 768, 12 blocks, context
    77), 512 prompt-length texts in one call; oracle on three of them,
    including a full-context one."""
    c = synth.TEXT_MODELS["l14_text"]
    lens = synth.draw_text_lengths(512, c.ctx, 6002)
    lens[7] = c.ctx
    seqs = synth.make_token_ids(lens, c.vocab, 6003)
    enc = V.TextEncoder(c, torch.from_numpy(blob("l14_text", 7001)).cuda(), "bf16")
    got = run(enc, seqs)
    sample = [0, 7, 511]
    cos = cosine(got[sample], oracle("l14_text", 7001, "bf16", [seqs[i] for i in sample]))
    _say(f"  l14 text bf16 min cos {cos.min():.6f}")
    assert cos.min() >= COS_TOL
    assert np.allclose(np.linalg.norm(got, axis=1), 1.0, atol=1e-5)
    enc.close()


def test_text_batch_invariance_graphs_and_split_bitwise(V):
    """A text's embedding is the same alone, inside a batch, replayed from a
    captured graph, and in a batch run as two parts on two streams."""
    c = synth.TEXT_MODELS["tiny_text"]
    lens = synth.draw_text_lengths(400, c.ctx, 6004)
    seqs = synth.make_token_ids(lens, c.vocab, 6005)
    assert sum(lens) >= 4096
    w = torch.from_numpy(blob("tiny_text", 7000)).cuda()
    enc = V.TextEncoder(c, w, "bf16")
    full = run(enc, seqs)
    for i in (0, 123, 399):
        assert np.array_equal(run(enc, [seqs[i]])[0], full[i])
    genc = V.TextEncoder(c, w, "bf16", graphs=True)
    for _ in range(3):
        assert np.array_equal(run(genc, seqs), full)
    V.vl_model_set_option(enc.handle, V.VL_OPT_SPLIT, 1)
    assert np.array_equal(run(enc, seqs), full)
    enc.close()
    genc.close()


def test_text_rejects_bad_lengths(V):
    c = synth.TEXT_MODELS["tiny_text"]
    enc = V.TextEncoder(c, torch.from_numpy(blob("tiny_text", 7000)).cuda(), "fp32")
    assert V.vl_text_workspace_bytes(enc.handle, [5, 0]) == 0
    assert V.vl_text_workspace_bytes(enc.handle, [c.ctx + 1]) == 0
    ids = torch.zeros(10, dtype=torch.int32, device="cuda")
    with pytest.raises(V.VlError):
        V.vl_encode_texts(enc.handle, ids, [5, 5], torch.empty((2, c.proj_dim), device="cuda",
                                                             dtype=torch.float32),
                          torch.empty(16, dtype=torch.uint8, device="cuda"))
    enc.close()
