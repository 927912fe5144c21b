"""FP64 CPU oracle of the contrastive image-encoder hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module; only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the HIP path: the only thing both sides read
is the seeded input generator in `synth/`, which holds none of the arithmetic
below.

What is computed.  The URBAN-SIM paper itself does not define an image
encoder: its only image tensor is the per-environment RGB-D observation at
128x128 fed to the navigation policy (Appendix, "Navigation Benchmark",
observation spaces), and it names vision-language models only as an
application in its datasheet and future work.  The encoder here is therefore
written from the standard definitions, each function citing the one it
follows:
  * ViT: Dosovitskiy et al., "An Image is Worth 16x16 Words", ICLR 2021,
    Sec. 3.1, Eq. 1-4 (patch embedding, class token, position embedding,
    pre-LN blocks, final LN on the class token).
  * Scaled dot-product and multi-head attention: Vaswani et al., "Attention
    Is All You Need", 2017, Sec. 3.2.1 Eq. 1 and Sec. 3.2.2.
  * LayerNorm: Ba et al., 2016, Sec. 3 (mean and biased variance over the
    hidden units).
  * GELU: Hendrycks & Gimpel, 2016, Sec. 2 (x * Phi(x)).
  * CLIP scoring: Radford et al., 2021, Sec. 2.3 and 3.1.2 (L2-normalised
    embeddings, scaled cosine logits, softmax over the class texts).
  * SigLIP scoring: Zhai et al., "Sigmoid Loss for Language Image
    Pre-Training", 2023, Sec. 3.2 Eq. 1 (logit t*x.y + b, sigmoid per pair).
  * Bilinear position-embedding resampling for other resolutions: ViT
    Sec. 3.2 ("2D interpolation of the pre-trained position embeddings"),
    with half-pixel centres and clamped edges.
  * BF16: round-to-nearest-even of FP32 to 8 significand bits.
  * FP8 e4m3fn: OCP 8-bit Floating Point Specification (OFP8) rev 1.0,
    Sec. 5.1 (E4M3: bias 7, max normal 448, no infinities) with one scale
    per output row.
  * MXFP8: OCP Microscaling Formats (MX) Specification v1.0 -- blocks of 32
    E4M3 elements sharing one E8M0 power-of-two scale, and its conversion
    of a vector of scalars to MX (shared exponent = floor(log2 of the
    block's largest magnitude) minus the element format's largest exponent,
    elements rounded after division by the scale, saturating).

Readings of unspecified points: pixels are
normalised with mean 1/2 and std 1/sqrt(12) per channel; patch vectors are
channel-major (c, a, b) like a conv weight [D, 3, P, P]; tokens are row-major
over the patch grid with the class token first; the grid is floor(H/P) x
floor(W/P) (extra pixels dropped); LayerNorm eps 1e-5 with biased variance;
exact erf GELU; no LayerNorm before the first block; MX shared exponents
are clamped below at -127 (the least E8M0 value; an all-zero block takes it); final LayerNorm on the
class token, then a bias-free projection and L2 normalisation (norm clamped
at 1e-12); attention never crosses images; softmax over texts per image;
top-1 is the lowest index attaining the maximum logit.

Every function computes in float64 with plain loops over images and heads and
no blocking, fusion or online softmax.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence, Tuple

import numpy as np
from scipy.special import erf as _erf

F64 = np.float64


# ---------------------------------------------------------------------------
# Elementwise / row operations
# ---------------------------------------------------------------------------
def layernorm(x: np.ndarray, gamma: np.ndarray, beta: np.ndarray,
              eps: float = 1e-5) -> np.ndarray:
    """LayerNorm over the last axis (Ba et al. 2016, Sec. 3): mean and biased
    variance over the hidden units, then the per-unit gain and bias."""
    x = np.asarray(x, F64)
    mu = x.mean(axis=-1, keepdims=True)
    var = ((x - mu) ** 2).mean(axis=-1, keepdims=True)
    return (x - mu) / np.sqrt(var + eps) * np.asarray(gamma, F64) + np.asarray(beta, F64)


def gelu(x: np.ndarray) -> np.ndarray:
    """GELU(x) = x * Phi(x) with Phi the standard normal CDF
    (Hendrycks & Gimpel 2016, Sec. 2), Phi(x) = (1 + erf(x / sqrt 2)) / 2."""
    x = np.asarray(x, F64)
    return 0.5 * x * (1.0 + _erf(x / math.sqrt(2.0)))


def softmax(x: np.ndarray, axis: int = -1) -> np.ndarray:
    """exp(x - max) / sum exp(x - max) along `axis` (the max is subtracted
    only to avoid overflow; the value is the plain softmax)."""
    x = np.asarray(x, F64)
    e = np.exp(x - x.max(axis=axis, keepdims=True))
    return e / e.sum(axis=axis, keepdims=True)


def sigmoid(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, F64)
    return 1.0 / (1.0 + np.exp(-x))


# ---------------------------------------------------------------------------
# Patch embedding and position embedding (ViT Sec. 3.1 Eq. 1, Sec. 3.2)
# ---------------------------------------------------------------------------
def normalise_pixels(img: np.ndarray, mean: Sequence[float],
                     std: Sequence[float]) -> np.ndarray:
    """x_hat[c] = (x[c] - mean_c) / std_c for a [C, H, W] image."""
    img = np.asarray(img, F64)
    m = np.asarray(mean, F64)[:, None, None]
    s = np.asarray(std, F64)[:, None, None]
    return (img - m) / s


def patch_grid(h: int, w: int, patch: int) -> Tuple[int, int]:
    """Grid of whole patches; pixels past the last whole patch are dropped."""
    return h // patch, w // patch


def patchify(img: np.ndarray, patch: int) -> np.ndarray:
    """Flatten every P x P patch of a [C, H, W] image into a vector ordered
    (c, a, b); patches row-major over the grid.  Returns [gh*gw, C*P*P]."""
    c, h, w = img.shape
    gh, gw = patch_grid(h, w, patch)
    x = np.asarray(img, F64)[:, :gh * patch, :gw * patch]
    x = x.reshape(c, gh, patch, gw, patch).transpose(1, 3, 0, 2, 4)
    return x.reshape(gh * gw, c * patch * patch)


def patch_embed(img_norm: np.ndarray, w: np.ndarray, b: np.ndarray,
                patch: int) -> np.ndarray:
    """Linear projection of flattened patches, E x_p + b (ViT Eq. 1), with
    E stored as a conv weight [D, C, P, P].  Returns [gh*gw, D]."""
    u = patchify(img_norm, patch)
    wm = np.asarray(w, F64).reshape(w.shape[0], -1)
    return u @ wm.T + np.asarray(b, F64)


def patch_embed_conv(img_norm: np.ndarray, w: np.ndarray, b: np.ndarray,
                     patch: int) -> np.ndarray:
    """The same map written as a stride-P convolution with direct loops over
    output pixels, channels and kernel taps (used only as a cross-check)."""
    x = np.asarray(img_norm, F64)
    wt = np.asarray(w, F64)
    d, c, p, _ = wt.shape
    gh, gw = patch_grid(x.shape[1], x.shape[2], patch)
    out = np.zeros((gh, gw, d))
    for r in range(gh):
        for q in range(gw):
            acc = np.array(b, F64, copy=True)
            for ch in range(c):
                for a in range(p):
                    for bb in range(p):
                        acc = acc + wt[:, ch, a, bb] * x[ch, r * p + a, q * p + bb]
            out[r, q] = acc
    return out.reshape(gh * gw, d)


def _interp_matrix(g0: int, g: int) -> np.ndarray:
    """[g, g0] weights of 1-D linear resampling with half-pixel centres:
    source coordinate s = (o + 1/2) * g0 / g - 1/2, clamped to [0, g0 - 1];
    neighbours floor(s) and min(floor(s) + 1, g0 - 1)."""
    m = np.zeros((g, g0))
    for o in range(g):
        s = (o + 0.5) * g0 / g - 0.5
        s = min(max(s, 0.0), g0 - 1.0)
        i0 = int(math.floor(s))
        i1 = min(i0 + 1, g0 - 1)
        t = s - i0
        m[o, i0] += 1.0 - t
        m[o, i1] += t
    return m


def interp_pos(pos: np.ndarray, g0: int, gh: int, gw: int) -> np.ndarray:
    """Position table [1 + g0*g0, D] resampled to a gh x gw grid by separable
    bilinear interpolation (ViT Sec. 3.2).  The class-token row is kept."""
    pos = np.asarray(pos, F64)
    d = pos.shape[1]
    grid = pos[1:].reshape(g0, g0, d)
    mh = _interp_matrix(g0, gh)
    mw = _interp_matrix(g0, gw)
    out = np.einsum("ri,ijd,qj->rqd", mh, grid, mw)
    return np.concatenate([pos[:1], out.reshape(gh * gw, d)], axis=0)


# ---------------------------------------------------------------------------
# Transformer block (ViT Eq. 2-3; attention per Vaswani et al. Sec. 3.2)
# ---------------------------------------------------------------------------
def attention_head(q: np.ndarray, k: np.ndarray, v: np.ndarray) -> np.ndarray:
    """softmax(q k^T / sqrt(d)) v for one head of one image (Eq. 1)."""
    d = q.shape[1]
    s = (q @ k.T) / math.sqrt(d)
    return softmax(s, axis=-1) @ v


def _identity(a: np.ndarray) -> np.ndarray:
    return a


def causal_attention_head(q: np.ndarray, k: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Masked self-attention for one head of one text sequence (the CLIP
    text encoder's masked self-attention, CLIP Sec. 2.4): token i takes the
    softmax over keys 0..i of q_i.k_j / sqrt(d); later keys get weight 0."""
    n, d = q.shape
    s = (q @ k.T) / math.sqrt(d)
    s = np.where(np.tril(np.ones((n, n), dtype=bool)), s, -np.inf)
    return softmax(s, axis=-1) @ v


def mhsa(y: np.ndarray, qkv_w, qkv_b, o_w, o_b, heads: int,
         aq=_identity, causal: bool = False) -> np.ndarray:
    """Multi-head self-attention over the tokens of one image.  The fused
    projection's outputs are [Q | K | V]; head k uses columns k*d .. k*d+d-1
    of each.  Heads are concatenated, then the output projection.  `aq` is
    applied to the left operand of both projections (the identity, or an
    activation encoding such as mx_round).  causal selects the masked form
    (text tower)."""
    y = np.asarray(y, F64)
    dm = y.shape[1]
    d = dm // heads
    qkv = aq(y) @ np.asarray(qkv_w, F64).T + np.asarray(qkv_b, F64)
    q, k, v = qkv[:, :dm], qkv[:, dm:2 * dm], qkv[:, 2 * dm:]
    o = np.zeros_like(q)
    for h in range(heads):
        sl = slice(h * d, (h + 1) * d)
        head = causal_attention_head if causal else attention_head
        o[:, sl] = head(q[:, sl], k[:, sl], v[:, sl])
    return aq(o) @ np.asarray(o_w, F64).T + np.asarray(o_b, F64)


def mlp(y: np.ndarray, fc1_w, fc1_b, fc2_w, fc2_b, aq=_identity) -> np.ndarray:
    """Two linear layers with GELU between them (ViT Sec. 3.1); `aq` as in
    mhsa, applied to the input of each layer."""
    h = gelu(aq(np.asarray(y, F64)) @ np.asarray(fc1_w, F64).T + np.asarray(fc1_b, F64))
    return aq(h) @ np.asarray(fc2_w, F64).T + np.asarray(fc2_b, F64)


def block(x: np.ndarray, lp: Dict[str, np.ndarray], heads: int,
          eps: float, aq=_identity, causal: bool = False) -> np.ndarray:
    """One pre-LN block: x' = x + MSA(LN(x)); x'' = x' + MLP(LN(x'))
    (ViT Eq. 2 and 3)."""
    x = np.asarray(x, F64)
    h = x + mhsa(layernorm(x, lp["ln1_g"], lp["ln1_b"], eps),
                 lp["qkv_w"], lp["qkv_b"], lp["o_w"], lp["o_b"], heads, aq, causal)
    return h + mlp(layernorm(h, lp["ln2_g"], lp["ln2_b"], eps),
                   lp["fc1_w"], lp["fc1_b"], lp["fc2_w"], lp["fc2_b"], aq)


# ---------------------------------------------------------------------------
# Whole encoder
# ---------------------------------------------------------------------------
def embed_tokens(img: np.ndarray, params: Dict, cfg) -> np.ndarray:
    """z_0 = [x_class; x_p^1 E; ...; x_p^N E] + E_pos (ViT Eq. 1), with E_pos
    resampled to the image's grid."""
    x = normalise_pixels(img, cfg.chan_mean, cfg.chan_std)
    gh, gw = patch_grid(x.shape[1], x.shape[2], cfg.patch)
    e = patch_embed(x, params["patch_w"], params["patch_b"], cfg.patch)
    tok = np.concatenate([np.asarray(params["cls"], F64)[None, :], e], axis=0)
    return tok + interp_pos(params["pos"], cfg.base_grid, gh, gw)


def act_encoding(act: str):
    """The map applied to the four block-linear inputs: "none" (identity)
    or "mx" (MXFP8 rounding of each token row, mx_round)."""
    if act == "none":
        return _identity
    if act == "mx":
        return mx_round
    raise ValueError(act)


def map_head(x: np.ndarray, params: Dict, heads: int, eps: float) -> np.ndarray:
    """Multi-head attention pooling with a learned query (pooling by
    multihead attention, Lee et al. 2019, Sec. 3.2, as the SigLIP image
    tower's head uses it): q = probe W_q^T + b_q; K, V from the tokens by
    W_kv; per head softmax(q k^T / sqrt(d)) v; output projection; then
    x + MLP(LN(x)) with GELU.  x: [N, D] final-LayerNormed tokens."""
    x = np.asarray(x, F64)
    dm = x.shape[1]
    d = dm // heads
    q = np.asarray(params["map_probe"], F64) @ np.asarray(params["map_q_w"], F64).T + \
        np.asarray(params["map_q_b"], F64)
    kv = x @ np.asarray(params["map_kv_w"], F64).T + np.asarray(params["map_kv_b"], F64)
    k, v = kv[:, :dm], kv[:, dm:]
    o = np.zeros(dm)
    for h in range(heads):
        sl = slice(h * d, (h + 1) * d)
        o[sl] = attention_head(q[None, sl], k[:, sl], v[:, sl])[0]
    y = o @ np.asarray(params["map_o_w"], F64).T + np.asarray(params["map_o_b"], F64)
    z = layernorm(y, params["map_ln_g"], params["map_ln_b"], eps)
    return y + mlp(z[None], params["map_fc1_w"], params["map_fc1_b"], params["map_fc2_w"],
                   params["map_fc2_b"])[0]


def encode_image(img: np.ndarray, params: Dict, cfg,
                 return_unnormalised: bool = False, act: str = "none"):
    """Image -> unit embedding: blocks, then either the final LN on the class
    token (ViT Eq. 4) or, for pool == "map", the final LN on every token and
    the attention-pooling head; bias-free projection, division by the L2
    norm (CLIP Sec. 2.3)."""
    aq = act_encoding(act)
    x = embed_tokens(img, params, cfg)
    for lp in params["layers"]:
        x = block(x, lp, cfg.heads, cfg.ln_eps, aq)
    if getattr(cfg, "pool", "cls") == "map":
        z = map_head(layernorm(x, params["lnf_g"], params["lnf_b"], cfg.ln_eps), params,
                     cfg.heads, cfg.ln_eps)
    else:
        z = layernorm(x[0], params["lnf_g"], params["lnf_b"], cfg.ln_eps)
    e = np.asarray(params["proj_w"], F64) @ z
    eh = e / max(np.linalg.norm(e), 1e-12)
    return (eh, e) if return_unnormalised else eh


def encode(images: Sequence[np.ndarray], params: Dict, cfg,
           act: str = "none") -> np.ndarray:
    """Unit embeddings [n, P_dim] of every image, one image at a time."""
    return np.stack([encode_image(im, params, cfg, act=act) for im in images])


# ---------------------------------------------------------------------------
# Text tower (CLIP Sec. 2.4)
# ---------------------------------------------------------------------------
def text_hidden(ids: np.ndarray, params: Dict, cfg, act: str = "none") -> np.ndarray:
    """Token embeddings plus learned absolute positions, then the pre-LN
    blocks with masked (causal) self-attention.  Returns [len, D]."""
    ids = np.asarray(ids, np.int64)
    aq = act_encoding(act)
    x = np.asarray(params["tok_emb"], F64)[ids] + np.asarray(params["pos"], F64)[:len(ids)]
    for lp in params["layers"]:
        x = block(x, lp, cfg.heads, cfg.ln_eps, aq, causal=True)
    return x


def encode_text(ids: np.ndarray, params: Dict, cfg, act: str = "none") -> np.ndarray:
    """Unit text embedding: the last token's (the end-of-text token's) final
    activations, LayerNorm, bias-free projection, L2 normalisation."""
    x = text_hidden(ids, params, cfg, act)
    z = layernorm(x[-1], params["lnf_g"], params["lnf_b"], cfg.ln_eps)
    e = np.asarray(params["proj_w"], F64) @ z
    return e / max(np.linalg.norm(e), 1e-12)


def encode_texts(seqs: Sequence[np.ndarray], params: Dict, cfg,
                 act: str = "none") -> np.ndarray:
    """Unit embeddings [n, P_dim] of every token sequence, one at a time."""
    return np.stack([encode_text(s, params, cfg, act) for s in seqs])


# ---------------------------------------------------------------------------
# Scoring heads
# ---------------------------------------------------------------------------
def logits(emb: np.ndarray, texts: np.ndarray, scale: float,
           bias: float = 0.0) -> np.ndarray:
    """l_ij = scale * <e_i, t_j> + bias."""
    return scale * (np.asarray(emb, F64) @ np.asarray(texts, F64).T) + bias


def score(emb: np.ndarray, texts: np.ndarray, head: str, scale: float,
          bias: float = 0.0) -> Tuple[np.ndarray, np.ndarray]:
    """CLIP head: softmax of the logits over texts for each image (CLIP
    Sec. 3.1.2).  SigLIP head: sigmoid of each logit (SigLIP Eq. 1).
    top1_i = lowest j attaining max_j l_ij."""
    l = logits(emb, texts, scale, bias)
    if head == "softmax":
        p = softmax(l, axis=1)
    elif head == "sigmoid":
        p = sigmoid(l)
    else:
        raise ValueError(head)
    return p, np.argmax(l, axis=1).astype(np.int32)


def contrastive_loss(emb: np.ndarray, texts: np.ndarray, head: str, scale: float,
                     bias: float = 0.0) -> float:
    """Loss of n matched pairs with logits l_ij = scale <e_i, t_j> + bias.
    softmax (CLIP Sec. 2.3): the mean of the row-wise (image -> text) and
    column-wise (text -> image) cross-entropies with target j = i.
    sigmoid (SigLIP Eq. 1): -(1/n) sum_ij log sigmoid(z_ij l_ij), z_ij = 1 if
    i == j else -1."""
    l = logits(emb, texts, scale, bias)
    n = l.shape[0]
    if head == "softmax":
        lr = np.log(softmax(l, axis=1))
        lc = np.log(softmax(l, axis=0))
        return float(-(np.trace(lr) + np.trace(lc)) / (2 * n))
    if head == "sigmoid":
        z = 2.0 * np.eye(n) - 1.0
        return float(np.sum(np.logaddexp(0.0, -z * l)) / n)   # -log sigmoid(x) = softplus(-x)
    raise ValueError(head)


def contrastive_grads(emb: np.ndarray, texts: np.ndarray, head: str, scale: float,
                      bias: float = 0.0):
    """Analytic gradient of contrastive_loss.  G = dL/dl:
    softmax: (P_row - I) / 2n + (P_col - I) / 2n with P_row / P_col the
    row- / column-wise softmax of l; sigmoid: -z sigmoid(-z l) / n.  Then
    dL/de = scale G t, dL/dt = scale G^T e, dL/dscale = sum G <e_i, t_j>,
    dL/dbias = sum G.  Returns (de, dt, dscale, dbias)."""
    e = np.asarray(emb, F64)
    t = np.asarray(texts, F64)
    l = logits(e, t, scale, bias)
    n = l.shape[0]
    if head == "softmax":
        g = (softmax(l, axis=1) - np.eye(n)) / (2 * n) + (softmax(l, axis=0) - np.eye(n)) / (2 * n)
    elif head == "sigmoid":
        z = 2.0 * np.eye(n) - 1.0
        g = -z * sigmoid(-z * l) / n
    else:
        raise ValueError(head)
    return scale * g @ t, scale * g.T @ e, float(np.sum(g * (e @ t.T))), float(np.sum(g))


# ---------------------------------------------------------------------------
# Number formats of the reduced-precision variants
# ---------------------------------------------------------------------------
def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest BF16 value (ties to even), returned
    as float64.  Done on the FP32 bit pattern: add 0x7FFF plus the lowest kept
    bit, then clear the 16 dropped bits.  NaN inputs are not expected."""
    b = np.ascontiguousarray(np.asarray(x, np.float32)).view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = ((b + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32).astype(F64)


E4M3_MAX = 448.0


def e4m3_round(y: np.ndarray) -> np.ndarray:
    """Nearest e4m3fn value (ties to even significand), saturating at +-448
    (OFP8 Sec. 5.1 with the saturating conversion).  Normal values have
    quantum 2^(e-3) for |y| in [2^e, 2^(e+1)), e >= -6; below 2^-6 the
    quantum is the subnormal step 2^-9."""
    y = np.asarray(y, F64)
    a = np.minimum(np.abs(y), E4M3_MAX)
    _, ex = np.frexp(a)                       # a = m * 2^ex, m in [0.5, 1)
    e = np.maximum(ex - 1, -6)                # binade exponent, clamped to subnormal
    quantum = np.ldexp(1.0, e - 3)
    q = np.round(a / quantum) * quantum       # np.round: half to even
    q = np.minimum(q, E4M3_MAX)
    return np.copysign(q, y)


def quantise_fp8_rows(w: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Per-output-row e4m3 weights: s_o = max_k |W_ok| / 448 and
    q = e4m3(W / s_o).  The scale and the division are taken in FP32, the
    precision in which the quantised code is decided.  Returns (q as float64
    values on the e4m3 grid, s as float64 [rows])."""
    w32 = np.asarray(w, np.float32)
    amax = np.abs(w32).max(axis=1)
    s = (amax / np.float32(E4M3_MAX)).astype(np.float32)
    s = np.where(s > 0, s, np.float32(1.0)).astype(np.float32)
    y = (w32 / s[:, None]).astype(np.float32)
    return e4m3_round(y), s.astype(F64)


E4M3_EMAX = 8      # exponent of the largest e4m3 normal, 448 = 1.75 * 2^8
MX_BLOCK = 32
E8M0_MIN = -127    # least exponent an E8M0 scale encodes


def mx_quantise(x: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """MXFP8 encoding of the last axis (length a multiple of 32) in blocks
    of 32 consecutive values.  Per block: amax = max |v|; shared exponent
    X = floor(log2 amax) - 8, at least -127 (and -127 for amax = 0); each
    element becomes e4m3_round(v / 2^X), saturating at 448.  Returns (the
    element values on the e4m3 grid, before scaling; X per block, int64).
    Division by 2^X is exact, so the rounding decision is that of the
    input value itself."""
    x = np.asarray(x, F64)
    n = x.shape[-1]
    if n % MX_BLOCK:
        raise ValueError("last axis must be a multiple of 32")
    xb = x.reshape(x.shape[:-1] + (n // MX_BLOCK, MX_BLOCK))
    amax = np.abs(xb).max(axis=-1)
    _, ex = np.frexp(amax)                   # amax = m * 2^ex, m in [0.5, 1)
    X = np.where(amax > 0, ex - 1 - E4M3_EMAX, E8M0_MIN)
    X = np.maximum(X, E8M0_MIN).astype(np.int64)
    q = e4m3_round(np.ldexp(xb, -X[..., None]))
    return q, X


def mx_round(x: np.ndarray) -> np.ndarray:
    """The values an MXFP8 encoding of x represents: element times 2^X."""
    x = np.asarray(x, F64)
    q, X = mx_quantise(x)
    return np.ldexp(q, X[..., None]).reshape(x.shape)


def e4m3_code(v: np.ndarray) -> np.ndarray:
    """Byte of each e4m3 value v (on the grid, |v| <= 448; OFP8 Sec. 5.1):
    sign bit 7; for |v| >= 2^-6 biased exponent e + 7 in bits 6..3 and
    (|v| / 2^e - 1) * 8 in bits 2..0, e = floor(log2 |v|); below 2^-6 the
    subnormal mantissa |v| * 2^9.  -0 keeps its sign bit."""
    v = np.asarray(v, F64)
    a = np.abs(v)
    _, ex = np.frexp(np.where(a > 0, a, 1.0))
    e = ex - 1
    normal = a >= 2.0 ** -6
    mant = np.where(normal, (np.ldexp(a, -e) - 1.0) * 8.0, a * 512.0)
    code = np.where(normal, ((e + 7) << 3) + mant, mant)
    code = code.astype(np.int64) | np.where(np.signbit(v), 0x80, 0)
    return code.astype(np.uint8)


def e4m3_value(code: np.ndarray) -> np.ndarray:
    """Value of e4m3fn bytes (OFP8 Sec. 5.1): exponent field E, mantissa M;
    E > 0: (1 + M/8) * 2^(E-7); E = 0: M/8 * 2^-6.  0x7F / 0xFF (NaN) are
    rejected."""
    c = np.asarray(code, np.int64)
    if np.any((c & 0x7F) == 0x7F):
        raise ValueError("NaN code")
    E = (c >> 3) & 15
    M = c & 7
    mag = np.where(E > 0, np.ldexp(1.0 + M / 8.0, E - 7), np.ldexp(M / 8.0, -6))
    return np.where(c & 0x80, -mag, mag)


def mx_decode(codes: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Values of an MXFP8 array: codes [..., n] (e4m3 bytes), X [..., n/32]
    shared exponents; element k is e4m3_value(code) * 2^X[k // 32]."""
    v = e4m3_value(codes)
    return np.ldexp(v, np.repeat(np.asarray(X, np.int64), MX_BLOCK, axis=-1))


BLOCK_LINEARS = ("qkv_w", "o_w", "fc1_w", "fc2_w")


def weights_for(params: Dict, precision: str) -> Dict:
    """The exact weights a precision variant computes with, as float64.
    fp32: unchanged.  bf16: the four per-block linear weights rounded to BF16.
    fp8w: those four as q * s_o (per-row e4m3 codes times FP32 scales).
    mxfp8: those four MXFP8-rounded along their input dimension (mx_round;
    the activations are rounded too, by encode(..., act="mx")).
    Biases, LayerNorm parameters, class token, position table, patch
    embedding and final projection stay FP32 in every variant; an
    attention-pooling head's K/V projection is rounded to BF16 in every
    variant but fp32 (its other weights stay FP32)."""
    out = {k: v for k, v in params.items() if k != "layers"}
    layers = []
    for lp in params["layers"]:
        nl = dict(lp)
        for n in BLOCK_LINEARS:
            if precision == "fp32":
                pass
            elif precision == "bf16":
                nl[n] = bf16_round(lp[n])
            elif precision == "fp8w":
                q, s = quantise_fp8_rows(lp[n])
                nl[n] = q * s[:, None]
            elif precision == "mxfp8":
                nl[n] = mx_round(np.asarray(lp[n], np.float32))
            else:
                raise ValueError(precision)
        layers.append(nl)
    out["layers"] = layers
    if "map_kv_w" in params and precision != "fp32":
        out["map_kv_w"] = bf16_round(params["map_kv_w"])
    return out
