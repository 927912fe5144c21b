"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds no arithmetic of the encoder or the scoring head: it only
draws random weights, images, text embeddings, resolutions and request
arrivals, and lays the weights out in the flat FP32 blob the C ABI consumes.
Both `oracle/` and the product package read what it produces; neither calls
into the other.

Generator: NumPy ``Generator(PCG64(seed))``.  Seed convention for workload k
(k = 0..4, in the order of ``WORKLOADS``): weights 1000+k, images 2000+k,
texts 3000+k, resolution draws 4000+k, request arrivals 5000+k.

Context: the paper's only image workload is a per-environment RGB-D frame at
128x128 (Appendix, navigation benchmark, observation spaces); the encoder
sizes below are the standard CLIP/SigLIP vision towers (ViT-B/16, ViT-L/14)
plus a tiny model for fast checks.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

__all__ = [
    "ModelConfig", "Workload", "MODELS", "WORKLOADS",
    "weight_layout", "weight_count", "make_blob", "make_params", "params_to_blob",
    "blob_to_params", "make_images", "make_texts", "draw_resolutions",
    "draw_requests", "seeds_for", "TextConfig", "TEXT_MODELS", "text_weight_layout",
    "text_weight_count", "make_text_blob", "text_blob_to_params", "make_token_ids",
    "draw_text_lengths",
]


@dataclass(frozen=True)
class ModelConfig:
    """Dimensions of a ViT image tower (patch P, width D, L blocks, h heads,
    MLP width F, projection width P_dim, base position grid g0 x g0, input
    planes C)."""
    name: str
    patch: int
    width: int
    layers: int
    heads: int
    mlp: int
    proj_dim: int
    base_grid: int
    ln_eps: float = 1e-5
    # Per-channel pixel statistics.  Pixels are U[0,1]; its exact mean is 1/2
    # and its exact standard deviation is 1/sqrt(12).
    chan_mean: Tuple[float, ...] = (0.5, 0.5, 0.5)
    chan_std: Tuple[float, ...] = (
        0.28867513459481287, 0.28867513459481287, 0.28867513459481287)
    channels: int = 3
    pool: str = "cls"          # "cls" (class token) or "map" (attention pooling head)

    @property
    def head_dim(self) -> int:
        return self.width // self.heads

    @property
    def base_res(self) -> int:
        return self.patch * self.base_grid


MODELS: Dict[str, ModelConfig] = {
    "tiny": ModelConfig("tiny", patch=16, width=128, layers=4, heads=4,
                        mlp=512, proj_dim=128, base_grid=4),
    "b16": ModelConfig("b16", patch=16, width=768, layers=12, heads=12,
                       mlp=3072, proj_dim=512, base_grid=14),
    "l14": ModelConfig("l14", patch=14, width=1024, layers=24, heads=16,
                       mlp=4096, proj_dim=768, base_grid=24),
    # RGB-D (4 planes) observation encoders for the navigation benchmark's
    # 128x128 frames: a ViT-S/16-shaped tower (the policy network is not
    # specified, so its size is a choice) and a tiny one for checks.
    "rgbd_s16": ModelConfig("rgbd_s16", patch=16, width=384, layers=12, heads=6, mlp=1536,
                            proj_dim=256, base_grid=8, chan_mean=(0.5,) * 4,
                            chan_std=(0.28867513459481287,) * 4, channels=4),
    # attention-pooling (MAP) heads, as in SigLIP image towers
    "tiny_map": ModelConfig("tiny_map", patch=16, width=128, layers=2, heads=4, mlp=512,
                            proj_dim=128, base_grid=4, pool="map"),
    "b16_map": ModelConfig("b16_map", patch=16, width=768, layers=12, heads=12, mlp=3072,
                           proj_dim=768, base_grid=14, pool="map"),
    "tiny_rgbd": ModelConfig("tiny_rgbd", patch=16, width=128, layers=2, heads=4, mlp=512,
                             proj_dim=128, base_grid=4, chan_mean=(0.5,) * 4,
                             chan_std=(0.28867513459481287,) * 4, channels=4),
}


@dataclass(frozen=True)
class Workload:
    """One benchmark/parity workload: model, batch, resolutions, scoring."""
    name: str
    index: int                 # k in the seed convention
    model: str
    n_images: int
    resolutions: Tuple[int, ...]   # one entry: fixed; several: drawn per image
    n_texts: int
    head: str                  # "softmax" | "sigmoid"
    scale: float
    bias: float
    precision: str             # "fp32" | "bf16" | "fp8w"
    requests: bool = False     # serving workload (Poisson arrivals)


WORKLOADS: Dict[str, Workload] = {
    w.name: w for w in [
        Workload("tiny_fp32", 0, "tiny", 8, (64,), 16, "softmax", 100.0, 0.0, "fp32"),
        Workload("b16_224", 1, "b16", 64, (224,), 1000, "softmax", 100.0, 0.0, "bf16"),
        Workload("l14_336", 2, "l14", 32, (336,), 4096, "sigmoid", 10.0, -10.0, "bf16"),
        Workload("b16_mixed", 3, "b16", 96, (224, 336, 448), 1000, "softmax", 100.0, 0.0, "bf16"),
        Workload("l14_serve", 4, "l14", 0, (224, 336, 384, 448), 8192, "sigmoid", 10.0, -10.0,
                 "fp8w", requests=True),
    ]
}


def seeds_for(workload: Workload) -> Dict[str, int]:
    k = workload.index
    return {"weights": 1000 + k, "images": 2000 + k, "texts": 3000 + k,
            "resolutions": 4000 + k, "arrivals": 5000 + k}


# ---------------------------------------------------------------------------
# Weight blob layout.  One FP32 array, tensors back to back, each C-contiguous,
# in exactly this order (documented identically in include/vl.h):
#   patch_w [D,C,P,P], patch_b [D], cls [D], pos [1+g0*g0, D],
#   per block: ln1_g [D], ln1_b [D], qkv_w [3D,D], qkv_b [3D], o_w [D,D],
#              o_b [D], ln2_g [D], ln2_b [D], fc1_w [F,D], fc1_b [F],
#              fc2_w [D,F], fc2_b [D],
#   lnf_g [D], lnf_b [D], proj_w [P_dim, D].
# Linear weights are [out, in]: y = x W^T + b.
# ---------------------------------------------------------------------------
_BLOCK_TENSORS = ("ln1_g", "ln1_b", "qkv_w", "qkv_b", "o_w", "o_b",
                  "ln2_g", "ln2_b", "fc1_w", "fc1_b", "fc2_w", "fc2_b")


def _block_shapes(c: ModelConfig) -> Dict[str, Tuple[int, ...]]:
    D, F = c.width, c.mlp
    return {"ln1_g": (D,), "ln1_b": (D,), "qkv_w": (3 * D, D), "qkv_b": (3 * D,),
            "o_w": (D, D), "o_b": (D,), "ln2_g": (D,), "ln2_b": (D,),
            "fc1_w": (F, D), "fc1_b": (F,), "fc2_w": (D, F), "fc2_b": (D,)}


def weight_layout(c: ModelConfig) -> List[Tuple[str, Tuple[int, ...]]]:
    """(name, shape) in blob order; block tensors are named '<layer>.<name>'."""
    D, P = c.width, c.patch
    out: List[Tuple[str, Tuple[int, ...]]] = [
        ("patch_w", (D, c.channels, P, P)), ("patch_b", (D,)), ("cls", (D,)),
        ("pos", (1 + c.base_grid * c.base_grid, D))]
    bs = _block_shapes(c)
    for l in range(c.layers):
        out += [(f"{l}.{n}", bs[n]) for n in _BLOCK_TENSORS]
    out += [("lnf_g", (D,)), ("lnf_b", (D,))]
    if c.pool == "map":
        F = c.mlp
        out += [("map_probe", (D,)), ("map_q_w", (D, D)), ("map_q_b", (D,)),
                ("map_kv_w", (2 * D, D)), ("map_kv_b", (2 * D,)), ("map_o_w", (D, D)),
                ("map_o_b", (D,)), ("map_ln_g", (D,)), ("map_ln_b", (D,)),
                ("map_fc1_w", (F, D)), ("map_fc1_b", (F,)), ("map_fc2_w", (D, F)),
                ("map_fc2_b", (D,))]
    out += [("proj_w", (c.proj_dim, D))]
    return out


def weight_count(c: ModelConfig) -> int:
    return int(sum(int(np.prod(s)) for _, s in weight_layout(c)))


_CHUNK = 1 << 22


def _fill_uniform(rng: np.random.Generator, out: np.ndarray) -> None:
    """Fill a float32 array with iid U[0,1) values on the 2^-24 grid.  Each
    64-bit PCG64 output gives two values (bits 63..40 and 39..16)."""
    flat = out.reshape(-1)
    n = flat.size
    for s in range(0, n, 2 * _CHUNK):
        m = min(2 * _CHUNK, n - s)
        raw = rng.bit_generator.random_raw((m + 1) // 2)
        u = np.empty(2 * raw.size, np.float32)
        u[0::2] = (raw >> np.uint64(40)).astype(np.float32)
        u[1::2] = ((raw >> np.uint64(16)) & np.uint64(0xFFFFFF)).astype(np.float32)
        u *= np.float32(2.0 ** -24)
        flat[s:s + m] = u[:m]


def _fill_normal(rng: np.random.Generator, out: np.ndarray, std: float) -> None:
    """Fill a float32 array with iid N(0, std^2) values (Box-Muller on two
    24-bit uniforms per 64-bit PCG64 output)."""
    flat = out.reshape(-1)
    n = flat.size
    for s in range(0, n, 2 * _CHUNK):
        m = min(2 * _CHUNK, n - s)
        raw = rng.bit_generator.random_raw((m + 1) // 2)
        u1 = ((raw >> np.uint64(40)).astype(np.float32) + np.float32(0.5)) \
            * np.float32(2.0 ** -24)
        u2 = ((raw >> np.uint64(16)) & np.uint64(0xFFFFFF)).astype(np.float32) \
            * np.float32(2.0 * np.pi * 2.0 ** -24)
        r = np.sqrt(np.float32(-2.0) * np.log(u1)) * np.float32(std)
        z = np.empty(2 * raw.size, np.float32)
        z[0::2] = r * np.cos(u2)
        z[1::2] = r * np.sin(u2)
        flat[s:s + m] = z[:m]


def make_blob(c: ModelConfig, seed: int, std: float = 0.02) -> np.ndarray:
    """Random-init weights as one flat FP32 blob in blob order.  Every linear
    weight, bias, CLS, position table, and (gamma - 1) and beta of each
    LayerNorm is N(0, std^2), so no value is exactly 0 or 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    blob = np.empty(weight_count(c), np.float32)
    _fill_normal(rng, blob, std)
    o = 0
    for name, shape in weight_layout(c):
        n = int(np.prod(shape))
        if name.endswith("_g"):
            blob[o:o + n] += np.float32(1.0)
        o += n
    return blob


def make_params(c: ModelConfig, seed: int, std: float = 0.02) -> Dict[str, object]:
    """`make_blob` viewed as {'patch_w':..., 'layers':[{...}], ...}."""
    return blob_to_params(c, make_blob(c, seed, std))


def params_to_blob(c: ModelConfig, p: Dict[str, object]) -> np.ndarray:
    parts = []
    for name, shape in weight_layout(c):
        if "." in name:
            l, n = name.split(".", 1)
            a = p["layers"][int(l)][n]
        else:
            a = p[name]
        a = np.asarray(a, dtype=np.float32)
        assert a.shape == tuple(shape), (name, a.shape, shape)
        parts.append(a.reshape(-1))
    return np.ascontiguousarray(np.concatenate(parts))


def blob_to_params(c: ModelConfig, blob: np.ndarray) -> Dict[str, object]:
    blob = np.asarray(blob, dtype=np.float32).reshape(-1)
    assert blob.size == weight_count(c)
    p: Dict[str, object] = {"layers": [dict() for _ in range(c.layers)]}
    o = 0
    for name, shape in weight_layout(c):
        n = int(np.prod(shape))
        a = blob[o:o + n].reshape(shape)
        o += n
        if "." in name:
            l, t = name.split(".", 1)
            p["layers"][int(l)][t] = a
        else:
            p[name] = a
    return p


# ---------------------------------------------------------------------------
# Images, texts, resolutions, requests.
# ---------------------------------------------------------------------------
def make_images(sizes: Sequence[Tuple[int, int]], seed: int,
                channels: int = 3) -> List[np.ndarray]:
    """One FP32 [C,H,W] array per (H, W), pixels iid U[0,1) (for RGB-D the
    depth plane is drawn the same way, as a normalised depth)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for (h, w) in sizes:
        a = np.empty((channels, h, w), np.float32)
        _fill_uniform(rng, a)
        out.append(a)
    return out


def make_texts(m: int, dim: int, seed: int) -> np.ndarray:
    """m text vectors uniform on the unit sphere (Gaussian, then divided by
    its norm), FP32 [m, dim]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((m, dim))
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    return g.astype(np.float32)


def draw_resolutions(n: int, choices: Sequence[int], seed: int) -> List[int]:
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = rng.integers(0, len(choices), size=n)
    return [int(choices[i]) for i in idx]


@dataclass
class Request:
    arrival_s: float
    sizes: List[Tuple[int, int]] = field(default_factory=list)


def draw_requests(n: int, qps: float, choices: Sequence[int], seed: int,
                  min_images: int = 1, max_images: int = 16) -> List[Request]:
    """Poisson arrivals at `qps` requests/s; each request holds U{min..max}
    images, all at one resolution drawn uniformly from `choices`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / qps, size=n)
    t = np.cumsum(gaps)
    counts = rng.integers(min_images, max_images + 1, size=n)
    res = rng.integers(0, len(choices), size=n)
    return [Request(float(t[i]), [(int(choices[res[i]]),) * 2] * int(counts[i]))
            for i in range(n)]



# ---------------------------------------------------------------------------
# Text tower (causal transformer over token ids).
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class TextConfig:
    """Dimensions of a text tower: token table rows, context length (position
    table rows), width D, L blocks, h heads, MLP width F, projection width."""
    name: str
    vocab: int
    ctx: int
    width: int
    layers: int
    heads: int
    mlp: int
    proj_dim: int
    ln_eps: float = 1e-5

    @property
    def head_dim(self) -> int:
        return self.width // self.heads


TEXT_MODELS: Dict[str, TextConfig] = {
    "tiny_text": TextConfig("tiny_text", vocab=1000, ctx=77, width=128, layers=2, heads=4,
                            mlp=512, proj_dim=128),
    # the CLIP ViT-L/14 text tower's shape
    "l14_text": TextConfig("l14_text", vocab=49408, ctx=77, width=768, layers=12, heads=12,
                           mlp=3072, proj_dim=768),
}


def text_weight_layout(c: TextConfig) -> List[Tuple[str, Tuple[int, ...]]]:
    """(name, shape) in blob order: tok_emb [V, D], pos [ctx, D], the blocks
    as for images, lnf_g, lnf_b, proj_w [P_dim, D]."""
    D, F = c.width, c.mlp
    bs = {"ln1_g": (D,), "ln1_b": (D,), "qkv_w": (3 * D, D), "qkv_b": (3 * D,),
          "o_w": (D, D), "o_b": (D,), "ln2_g": (D,), "ln2_b": (D,),
          "fc1_w": (F, D), "fc1_b": (F,), "fc2_w": (D, F), "fc2_b": (D,)}
    out: List[Tuple[str, Tuple[int, ...]]] = [("tok_emb", (c.vocab, D)), ("pos", (c.ctx, D))]
    for l in range(c.layers):
        out += [(f"{l}.{n}", bs[n]) for n in _BLOCK_TENSORS]
    out += [("lnf_g", (D,)), ("lnf_b", (D,)), ("proj_w", (c.proj_dim, D))]
    return out


def text_weight_count(c: TextConfig) -> int:
    return int(sum(int(np.prod(s)) for _, s in text_weight_layout(c)))


def make_text_blob(c: TextConfig, seed: int, std: float = 0.02) -> np.ndarray:
    """Random-init text weights in blob order, drawn like make_blob: N(0,
    std^2) everywhere, plus 1 on every LayerNorm gain."""
    rng = np.random.Generator(np.random.PCG64(seed))
    blob = np.empty(text_weight_count(c), np.float32)
    _fill_normal(rng, blob, std)
    o = 0
    for name, shape in text_weight_layout(c):
        n = int(np.prod(shape))
        if name.endswith("_g"):
            blob[o:o + n] += np.float32(1.0)
        o += n
    return blob


def text_blob_to_params(c: TextConfig, blob: np.ndarray) -> Dict[str, object]:
    blob = np.asarray(blob, dtype=np.float32).reshape(-1)
    assert blob.size == text_weight_count(c)
    p: Dict[str, object] = {"layers": [dict() for _ in range(c.layers)]}
    o = 0
    for name, shape in text_weight_layout(c):
        n = int(np.prod(shape))
        a = blob[o:o + n].reshape(shape)
        o += n
        if "." in name:
            l, t = name.split(".", 1)
            p["layers"][int(l)][t] = a
        else:
            p[name] = a
    return p


def draw_text_lengths(n: int, ctx: int, seed: int) -> List[int]:
    """Prompt-like token counts: U{5..20} (short class prompts), with one in
    ten sequences at the full context length."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lens = rng.integers(5, 21, size=n)
    full = rng.random(n) < 0.1
    return [int(ctx if f else min(l, ctx)) for l, f in zip(lens, full)]


def make_token_ids(lengths: Sequence[int], vocab: int, seed: int) -> List[np.ndarray]:
    """One int32 id sequence per length: start-of-text (vocab - 2), uniform
    ids below vocab - 2, end-of-text (vocab - 1) last; a length-1 sequence
    is just the end-of-text token."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for L in lengths:
        ids = rng.integers(0, vocab - 2, size=L).astype(np.int32)
        if L >= 2:
            ids[0] = vocab - 2
        ids[-1] = vocab - 1
        out.append(ids)
    return out
