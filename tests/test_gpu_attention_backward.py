"""GPU parity of the attention backward on its own (vl_attention_backward),
element by element against the FP64 oracle (oracle/train64.py
attention_head_backward: the derivative of Vaswani et al. 2017, Sec. 3.2.1
Eq. 1, per sequence and head).

Inputs are BF16-representable, so both kernels and the oracle see the same
Q, K, V; the forward output O handed to the backward is the oracle's, rounded
to the kernel's element type (the test does not depend on the forward
kernel); dO is FP32.

Bars (derived from the arithmetic).  BF16 kernels: scores are exact products
of the BF16 inputs accumulated in FP32, P is formed in FP32 from the
log-sum-exp; dO is rounded to BF16 (relative 2^-9) as an operand of
dP = dO V^T and dV = P^T dO, O is BF16 in D = rowsum(dO O), P and dS are
rounded to BF16 as operands, and every output once more.  So, with
A = |dO| |V|^T, B = rowsum(|dO| |O|) and E = P (A + B) + |dS| (per query and
key), |dS - dS_ref| <= 2^-9 E, hence
  |dQ - dQ_ref| <= 2^-9 (E |K| / sqrt(d) + |dQ_ref|),
  |dK - dK_ref| <= 2^-9 (E^T |Q| / sqrt(d) + |dK_ref|),
  |dV - dV_ref| <= 2^-9 (2 P^T |dO| + |dV_ref|)
up to FP32 accumulation terms; the test allows twice that.  FP32 kernels:
1e-4 of the same magnitudes.  These worst-case bars grow with the number of
keys where the terms of a sum cancel, so each (sequence, head, gradient)
block of more than one token must also meet |err|_F <= b |ref|_F, with
b = 2^-6 for BF16 (the rounding errors above are independent: about 2^-8 of
a gradient in RMS), 2^-5 where the scores are peaked (dS = P (dP - D) then
cancels: D is formed from the FP32 dO, dP from its BF16 rounding), 1e-4 for
FP32.  A dropped key, a dropped query, a transposed operand or a wrong D
moves a block by more.  (A one-token sequence has dQ = dK = 0 exactly; the
kernels leave the rounding of dO in dP - D there, which the element bar
covers.)
"""
import math
import sys

import numpy as np
import pytest

from oracle import train64 as TR
from oracle import vit64 as O

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


def _bf16_round(x):
    return O.bf16_round(np.asarray(x, np.float32)).astype(np.float64)


def oracle_backward(qkv, dout, lengths, heads, d):
    """Per sequence and head: the oracle's forward O and (dQ, dK, dV), and the
    magnitudes the bars scale with."""
    D = heads * d
    T = qkv.shape[0]
    out = np.zeros((T, D))
    dqkv = np.zeros((T, 3 * D))
    mag = np.zeros((T, 3 * D))
    c = 1.0 / math.sqrt(d)
    t0 = 0
    for n in lengths:
        blk = qkv[t0:t0 + n]
        for h in range(heads):
            sl = slice(h * d, (h + 1) * d)
            q, k, v = blk[:, sl], blk[:, D:][:, sl], blk[:, 2 * D:][:, sl]
            do = dout[t0:t0 + n, sl]
            o = O.attention_head(q, k, v)
            dq, dk, dv = TR.attention_head_backward(q, k, v, do)
            out[t0:t0 + n, sl] = o
            dqkv[t0:t0 + n, sl] = dq
            dqkv[t0:t0 + n, D + h * d:D + (h + 1) * d] = dk
            dqkv[t0:t0 + n, 2 * D + h * d:2 * D + (h + 1) * d] = dv
            p = O.softmax((q @ k.T) * c, axis=-1)
            dp = do @ v.T
            ds = p * (dp - (do * o).sum(axis=1, keepdims=True))
            e = p * (np.abs(do) @ np.abs(v).T + (np.abs(do) * np.abs(o)).sum(axis=1, keepdims=True))
            e += np.abs(ds)
            mag[t0:t0 + n, sl] = (e @ np.abs(k)) * c
            mag[t0:t0 + n, D + h * d:D + (h + 1) * d] = (e.T @ np.abs(q)) * c
            mag[t0:t0 + n, 2 * D + h * d:2 * D + (h + 1) * d] = 2.0 * (p.T @ np.abs(do))
        t0 += n
    return out, dqkv, mag


def _check(V, qkv, dout, lengths, heads, d, blk_bf16=2.0 ** -6):
    qkv = _bf16_round(qkv)
    dout = dout.astype(np.float32).astype(np.float64)
    out, ref, mag = oracle_backward(qkv, dout, lengths, heads, d)
    for dtype in ("bf16", "fp32"):
        tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
        x = torch.from_numpy(qkv.astype(np.float32)).to(tdt).cuda()
        o = torch.from_numpy(out.astype(np.float32)).to(tdt).cuda()
        g = torch.from_numpy(dout.astype(np.float32)).cuda()
        dx = torch.full_like(x, float("nan"))
        _say(f"  {dtype} lengths {lengths} heads {heads} d {d}")
        V.vl_attention_backward(x, o, g, lengths, heads, d, dx)
        torch.cuda.synchronize()
        got = dx.float().cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(got)), dtype
        unit = 2.0 ** -8 if dtype == "bf16" else 1e-4
        blk_unit = blk_bf16 if dtype == "bf16" else 1e-4
        tol = unit * (mag + np.abs(ref)) + 1e-30
        err = np.abs(got - ref)
        _say(f"    max |err| / element bar = {float(np.max(err / tol)):.3f}")
        worst_blk = 0.0
        for j, name in enumerate(("dQ", "dK", "dV")):
            for h in range(heads):
                cols = slice(j * heads * d + h * d, j * heads * d + (h + 1) * d)
                bad = err[:, cols] > tol[:, cols]
                assert not bad.any(), (dtype, name, h, int(bad.sum()))
                t0 = 0
                for n in lengths:
                    if n > 1:
                        e = float(np.linalg.norm(err[t0:t0 + n, cols]))
                        r = float(np.linalg.norm(ref[t0:t0 + n, cols]))
                        assert e <= blk_unit * r, (dtype, name, h, t0, e / r)
                        worst_blk = max(worst_blk, e / r)
                    t0 += n
        _say(f"    max over (sequence, head, gradient) of |err|_F / |ref|_F = {worst_blk:.2e}")


@pytest.mark.parametrize("d", [64, 32])
def test_attention_backward_ragged(V, d):
    """Ragged lengths: one full key tile plus one key, a single token, the
    ViT-L/14@336 image (five 128-query blocks, the last with one query), two
    partial 128-blocks, and the longest image sequence."""
    rng = np.random.Generator(np.random.PCG64(5100 + d))
    lengths = [65, 1, 577, 130, 1025]
    heads = 4
    T = sum(lengths)
    qkv = rng.standard_normal((T, 3 * heads * d))
    dout = rng.standard_normal((T, heads * d))
    _check(V, qkv, dout, lengths, heads, d)


def test_attention_backward_peaked_scores(V):
    """Scores of standard deviation 10 (Q, K entries of std sqrt(10)): most
    rows of P are dominated by a few keys, so P and dS span many binades."""
    rng = np.random.Generator(np.random.PCG64(5200))
    lengths = [577, 64, 129]
    heads, d = 4, 64
    T = sum(lengths)
    qkv = rng.standard_normal((T, 3 * heads * d))
    qkv[:, :2 * heads * d] *= math.sqrt(10.0)
    dout = rng.standard_normal((T, heads * d))
    _check(V, qkv, dout, lengths, heads, d, blk_bf16=2.0 ** -5)


def test_attention_backward_l14_heads(V):
    """ViT-L/14@336 shape: 16 heads of 64 over two 577-token images, with
    N(0, 0.02^2)-weight-like activations (small scores, nearly uniform P)."""
    rng = np.random.Generator(np.random.PCG64(5300))
    lengths = [577, 577]
    heads, d = 16, 64
    T = sum(lengths)
    qkv = rng.standard_normal((T, 3 * heads * d)) * 0.5
    dout = rng.standard_normal((T, heads * d)) * 1e-3
    _check(V, qkv, dout, lengths, heads, d)


def test_attention_backward_rejects_bad_arguments(V):
    x = torch.zeros((10, 3 * 64), dtype=torch.bfloat16, device="cuda")
    o = torch.zeros((10, 64), dtype=torch.bfloat16, device="cuda")
    g = torch.zeros((10, 64), dtype=torch.float32, device="cuda")
    dx = torch.zeros_like(x)
    assert V.vl_attention_backward_workspace_bytes([10], 1, 48) == 0
    assert V.vl_attention_backward_workspace_bytes([0], 1, 64) == 0
    with pytest.raises(ValueError):
        V.vl_attention_backward(x, o, g, [9], 1, 64, dx)           # shapes do not add up
    with pytest.raises(ValueError):
        V.vl_attention_backward(x, o.float(), g, [10], 1, 64, dx)  # O of another dtype
    x48 = torch.zeros((10, 3 * 48), dtype=torch.bfloat16, device="cuda")
    with pytest.raises(V.VlError):                                  # head_dim 48
        V.vl_attention_backward(x48, o[:, :48].contiguous(), g[:, :48].contiguous(), [10], 1, 48,
                                torch.zeros_like(x48))
