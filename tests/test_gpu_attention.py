"""GPU parity of the attention kernels on their own (vl_attention), element by
element against the FP64 oracle, on inputs built to reach the BF16 kernel's
online-softmax rescale.

The BF16 kernel keeps a reference maximum per query and raises it only when
a 64-key tile's maximum exceeds it by more than 2^8 (in log2 units of the
scaled scores); the rescale then multiplies the running sum and the output
accumulators.  Random N(0, 0.02^2) weights never drive a later tile that far
above the first one, so these inputs are built for it:
  * adversarial logits: Q and K entries with standard deviation sqrt(10), so
    the scores q.k / sqrt(d) have standard deviation 10;
  * a dominant key in the last key tile (or in a middle one): every query
    shares a direction u, and that one key is kappa * u;
  * the causal mask with a dominant late key.
Each case asserts, from the oracle's FP64 scores, that some query meets a
tile whose maximum exceeds the maximum of all earlier tiles by more than 8
log2 units (the reference maximum of the kernel can only be lower, so the
rescale runs there), then compares every output element.

Bars (derived from the arithmetic).  BF16 kernel: scores are exact products
of the BF16 inputs accumulated in FP32; the probabilities are rounded to BF16
(relative 2^-9) before the product with V while their sum stays FP32; the
output is rounded to BF16 once.  So |o - o_ref| <= 2^-9 sum_j p_j |v_j| +
2^-9 |o_ref| plus FP32 accumulation terms; the test allows twice that.  FP32
kernel: 1e-4 of sum_j p_j |v_j| (FP32 score accumulation over the head
dimension at scores of magnitude 30 moves a probability by about 1e-5
relative).  A rescale that forgets the sum or the accumulators, or applies
the wrong factor, is wrong by O(1) of the same scale.
"""
import math
import sys

import numpy as np
import pytest

from oracle import vit64 as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TAU = 8.0   # the kernel's rescale threshold, log2 units
LOG2E = 1.0 / math.log(2.0)


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
    return O.bf16_round(np.asarray(x, np.float32))


def oracle_attention(qkv, lengths, heads, d, causal):
    """FP64 multi-head attention of packed sequences (oracle functions per
    sequence and head), the per-element magnitude sum_j p_j |v_j|, and the
    largest rescale excursion: per query, the maximum over key tiles t >= 1
    of (max score of tile t - max score of tiles < t), in log2 units."""
    qkv = np.asarray(qkv, np.float64)
    D = heads * d
    out = np.zeros((qkv.shape[0], D))
    mag = np.zeros_like(out)
    exc = -np.inf
    exc_last = -np.inf          # excursions at the sequence's last key tile
    t0 = 0
    for n in lengths:
        blk = qkv[t0:t0 + n]
        for h in range(heads):
            sl = slice(h * d, (h + 1) * d)
            q, k, v = blk[:, sl], blk[:, D:][:, sl], blk[:, 2 * D:][:, sl]
            head = O.causal_attention_head if causal else O.attention_head
            out[t0:t0 + n, sl] = head(q, k, v)
            s = (q @ k.T) / math.sqrt(d)
            if causal:
                s = np.where(np.tril(np.ones((n, n), dtype=bool)), s, -np.inf)
            mag[t0:t0 + n, sl] = O.softmax(s, axis=-1) @ np.abs(v)
            s2 = s * LOG2E
            nt = (n + 63) // 64
            run = np.max(s2[:, :64], axis=1)
            for t in range(1, nt):
                tm = np.max(s2[:, 64 * t:64 * (t + 1)], axis=1)
                ok = np.isfinite(tm) & np.isfinite(run)
                if ok.any():
                    e = float(np.max(tm[ok] - run[ok]))
                    exc = max(exc, e)
                    if t == nt - 1:
                        exc_last = max(exc_last, e)
                run = np.maximum(run, tm)
        t0 += n
    return out, mag, exc, exc_last


def _run(V, qkv64, lengths, heads, d, causal, dtype):
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
    x = torch.from_numpy(qkv64.astype(np.float32)).to(tdt).cuda()
    out = torch.empty((x.shape[0], heads * d), dtype=tdt, device="cuda")
    V.vl_attention(x, lengths, heads, d, causal, out)
    torch.cuda.synchronize()
    return out.float().cpu().numpy().astype(np.float64)


def _compare(V, qkv, lengths, heads, d, causal, want_exc, want_last=False):
    """Both kernels against the oracle on the same (BF16-representable)
    inputs; asserts the rescale excursion from the oracle's scores first."""
    qkv = _bf16_round(qkv)                  # the inputs both kernels see exactly
    ref, mag, exc, exc_last = oracle_attention(qkv, lengths, heads, d, causal)
    _say(f"  lengths {lengths} heads {heads} d {d} causal {causal}: max excursion "
         f"{exc:.1f} log2 (last tile {exc_last:.1f})")
    assert exc > want_exc, exc
    if want_last:
        assert exc_last > want_exc, exc_last
    for dtype in ("bf16", "fp32"):
        got = _run(V, qkv, lengths, heads, d, causal, dtype)
        err = np.abs(got - ref)
        if dtype == "bf16":
            tol = 2.0 ** -8 * (mag + np.abs(ref)) + 1e-30
        else:
            tol = 1e-4 * mag + 1e-30
        worst = float(np.max(err / tol))
        _say(f"    {dtype}: max |err| / bar = {worst:.3f}")
        assert np.all(err <= tol), (dtype, worst)


def _qkv(lengths, heads, d, rng, qk_std=1.0):
    T = sum(lengths)
    D = heads * d
    x = rng.standard_normal((T, 3 * D))
    x[:, :2 * D] *= qk_std
    return x


@pytest.mark.parametrize("d", [64, 32])
def test_adversarial_logits(V, d):
    """Scores of standard deviation 10 (Q, K entries of std sqrt(10)),
    ragged lengths: one token, one full key tile plus one key, five query
    blocks, the longest image sequence."""
    rng = np.random.Generator(np.random.PCG64(4100 + d))
    lengths = [65, 1, 577, 130, 1025]
    heads = 4
    # q.k / sqrt(d) with iid N(0, a^2) entries has standard deviation a^2
    x = _qkv(lengths, heads, d, rng, qk_std=math.sqrt(10.0))
    _compare(V, x, lengths, heads, d, False, want_exc=TAU + 2)


def _plant(x, lengths, heads, d, key_pos, kappa, a, heads_planted, rng):
    """Every query of the planted heads gets the component a*u; the key at
    key_pos (index within each sequence) becomes kappa*u, so its score is
    about a*kappa/sqrt(d) above the others."""
    D = heads * d
    t0 = 0
    for n in lengths:
        for h in heads_planted:
            u = rng.standard_normal(d)
            u /= np.linalg.norm(u)
            x[t0:t0 + n, h * d:(h + 1) * d] += a * u
            if key_pos(n) is not None:
                x[t0 + key_pos(n), D + h * d:D + (h + 1) * d] = kappa * u
        t0 += n
    return x


@pytest.mark.parametrize("n", [65, 577, 1025])
@pytest.mark.parametrize("d", [64, 32])
def test_dominant_key_in_last_tile(V, n, d):
    """The last key of each sequence (alone in its 64-key tile for these
    lengths) dominates every query of heads 0 and 2; heads 1 and 3 stay
    plain, so a wave's rescale vote and the heads' independence are both
    exercised.  Two strengths: about 20 and about 90 log2 units past the
    other keys."""
    heads = 4
    for kappa, a in ((12.0, 10.0), (40.0, 10.0)):
        rng = np.random.Generator(np.random.PCG64(4200 + n + d + int(kappa)))
        lengths = [n, n]
        x = _qkv(lengths, heads, d, rng)
        x = _plant(x, lengths, heads, d, lambda m: m - 1, kappa * math.sqrt(d) / 8.0, a,
                   (0, 2), rng)
        _compare(V, x, lengths, heads, d, False, want_exc=TAU + 1, want_last=True)


def test_dominant_key_mid_sequence(V):
    """A dominant key in a middle tile (key 300 of 577): the reference
    maximum is raised there and the later tiles run against it."""
    heads, d = 4, 64
    rng = np.random.Generator(np.random.PCG64(4300))
    lengths = [577, 200, 577]
    x = _qkv(lengths, heads, d, rng)
    x = _plant(x, lengths, heads, d, lambda m: 300 if m > 300 else None, 12.0, 10.0,
               (0, 1, 2, 3), rng)
    _compare(V, x, lengths, heads, d, False, want_exc=TAU + 1)


@pytest.mark.parametrize("pos", [70, 250, 299])
def test_causal_dominant_late_key(V, pos):
    """Causal attention over text-length sequences with a dominant key at
    position pos: queries before it never see it (masked), the ones after it
    must rescale inside the tile that holds it; 300 tokens span three query
    blocks and five key tiles."""
    heads, d = 4, 64
    rng = np.random.Generator(np.random.PCG64(4400 + pos))
    lengths = [77, 300, 20]
    x = _qkv(lengths, heads, d, rng)
    x = _plant(x, lengths, heads, d, lambda m: pos if m > pos else None, 12.0, 10.0,
               (0, 3), rng)
    _compare(V, x, lengths, heads, d, True, want_exc=TAU + 1)


def test_causal_adversarial(V):
    heads, d = 2, 32
    rng = np.random.Generator(np.random.PCG64(4500))
    lengths = [300, 1, 64, 65, 129]
    x = _qkv(lengths, heads, d, rng, qk_std=math.sqrt(10.0))
    _compare(V, x, lengths, heads, d, True, want_exc=TAU + 1)


def test_plain_inputs_match(V):
    """Unit-variance inputs (no excursion needed): the common path."""
    heads, d = 16, 64
    rng = np.random.Generator(np.random.PCG64(4600))
    lengths = [577, 197, 2]
    x = _qkv(lengths, heads, d, rng)
    qkv = _bf16_round(x)
    ref, mag, _, _ = oracle_attention(qkv, lengths, heads, d, False)
    for dtype, f in (("bf16", 2.0 ** -8), ("fp32", 1e-4)):
        got = _run(V, qkv, lengths, heads, d, False, dtype)
        tol = f * (mag + (np.abs(ref) if dtype == "bf16" else 0.0)) + 1e-30
        assert np.all(np.abs(got - ref) <= tol), dtype
