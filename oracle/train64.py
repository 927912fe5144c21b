"""FP64 CPU oracle of contrastive training through the image encoder.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this module; only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  It shares no code with the HIP path.

What is computed: the gradient of a contrastive loss (CLIP, Radford et al.
2021, Sec. 2.3; SigLIP, Zhai et al. 2023, Eq. 1) of a batch of images
against given text embeddings, with respect to every parameter of the image
tower of vit64 (class-token pooling, or the attention-pooling head: a learned
query attending over every final-LayerNormed token, Lee et al. 2019, Sec.
3.2) -- the backward pass of the forward in vit64, written out by the chain
rule of each of its definitions:

  * L2 normalisation e_hat = e / |e|:  de = (de_hat - e_hat <e_hat, de_hat>) / |e|.
  * Linear y = x W^T + b:  dx = dy W,  dW = dy^T x,  db = sum over rows of dy.
  * LayerNorm (Ba et al. 2016, Sec. 3) y = x_hat * g + b with
    x_hat = (x - mean) / sqrt(var + eps):  dx = (dxh - mean(dxh) -
    x_hat * mean(dxh * x_hat)) / sqrt(var + eps), dxh = dy * g;
    dg = sum dy * x_hat,  db = sum dy.
  * GELU(z) = z Phi(z) (Hendrycks & Gimpel 2016, Sec. 2):
    GELU'(z) = Phi(z) + z phi(z), phi the standard normal density.
  * Attention (Vaswani et al. 2017, Sec. 3.2.1 Eq. 1) O = P V with
    P = softmax(S), S = Q K^T / sqrt(d):  dV = P^T dO,  dP = dO V^T,
    dS = P * (dP - rowsum(dP * P)),  dQ = dS K / sqrt(d),  dK = dS^T Q / sqrt(d)
    (the attention-pooling head: one query row per head, q = probe W_q^T + b_q,
    so dprobe = dq W_q, dW_q = dq probe^T).
  * Patch embedding and position table (ViT, Dosovitskiy et al. 2021,
    Sec. 3.1 Eq. 1, Sec. 3.2): the patch weights' gradient is the
    row-sum of outer products of token gradients with the normalised patch
    vectors; the class token and position row 0 take the class token's
    gradient; the base position grid takes the adjoint of the bilinear
    resampling, i.e. the transposed interpolation matrices.

Gradients are summed over the images of the batch.  Every function is plain
float64 NumPy with loops over images and heads.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence, Tuple

import numpy as np
from scipy.special import erf as _erf

from . import vit64 as V

F64 = np.float64


def layernorm_backward(x: np.ndarray, gamma: np.ndarray, dy: np.ndarray,
                       eps: float) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """dx, dgamma, dbeta of LayerNorm over the last axis (rows of x)."""
    x = np.asarray(x, F64)
    dy = np.asarray(dy, F64)
    mu = x.mean(axis=-1, keepdims=True)
    var = ((x - mu) ** 2).mean(axis=-1, keepdims=True)
    rstd = 1.0 / np.sqrt(var + eps)
    xh = (x - mu) * rstd
    dxh = dy * np.asarray(gamma, F64)
    dx = rstd * (dxh - dxh.mean(axis=-1, keepdims=True) -
                 xh * (dxh * xh).mean(axis=-1, keepdims=True))
    red = tuple(range(x.ndim - 1))
    return dx, (dy * xh).sum(axis=red), dy.sum(axis=red)


def gelu_grad(z: np.ndarray) -> np.ndarray:
    """d/dz of z Phi(z) = Phi(z) + z phi(z)."""
    z = np.asarray(z, F64)
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * phi


def attention_head_backward(q: np.ndarray, k: np.ndarray, v: np.ndarray,
                            do: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """dq, dk, dv of softmax(q k^T / sqrt(d)) v for one head of one image."""
    d = q.shape[1]
    c = 1.0 / math.sqrt(d)
    p = V.softmax((q @ k.T) * c, axis=-1)
    dv = p.T @ do
    dp = do @ v.T
    ds = p * (dp - (dp * p).sum(axis=-1, keepdims=True))
    return (ds @ k) * c, (ds.T @ q) * c, dv


def _zeros_like_params(params: Dict) -> Dict:
    out = {k: np.zeros(np.shape(v), F64) for k, v in params.items() if k != "layers"}
    out["layers"] = [{k: np.zeros(np.shape(v), F64) for k, v in lp.items()}
                     for lp in params["layers"]]
    return out


def _add(acc: Dict, g: Dict) -> None:
    for k, v in g.items():
        if k == "layers":
            for la, lg in zip(acc["layers"], v):
                for kk, vv in lg.items():
                    la[kk] += vv
        else:
            acc[k] += v


def map_forward(xl: np.ndarray, params: Dict, heads: int, eps: float) -> Dict:
    """The attention-pooling head of vit64.map_head on final-LayerNormed
    tokens xl [N, D], keeping every intermediate the backward needs; 'out'
    is the head's output."""
    xl = np.asarray(xl, F64)
    dm = xl.shape[1]
    d = dm // heads
    probe = np.asarray(params["map_probe"], F64)
    q = probe @ np.asarray(params["map_q_w"], F64).T + np.asarray(params["map_q_b"], F64)
    kv = xl @ np.asarray(params["map_kv_w"], F64).T + np.asarray(params["map_kv_b"], F64)
    o = np.zeros(dm)
    for h in range(heads):
        sl = slice(h * d, (h + 1) * d)
        o[sl] = V.attention_head(q[None, sl], kv[:, :dm][:, sl], kv[:, dm:][:, sl])[0]
    y = o @ np.asarray(params["map_o_w"], F64).T + np.asarray(params["map_o_b"], F64)
    zl = V.layernorm(y, params["map_ln_g"], params["map_ln_b"], eps)
    hpre = zl @ np.asarray(params["map_fc1_w"], F64).T + np.asarray(params["map_fc1_b"], F64)
    hg = V.gelu(hpre)
    out = y + hg @ np.asarray(params["map_fc2_w"], F64).T + np.asarray(params["map_fc2_b"], F64)
    return {"xl": xl, "q": q, "kv": kv, "o": o, "y": y, "zl": zl, "hpre": hpre, "hg": hg,
            "out": out}


def map_backward(dout: np.ndarray, s: Dict, params: Dict, heads: int, eps: float,
                 g: Dict) -> np.ndarray:
    """Backward of the attention-pooling head from d(out) [D]: adds the
    head's parameter gradients to g and returns d(xl) [N, D]."""
    dout = np.asarray(dout, F64)
    dm = dout.shape[0]
    d = dm // heads
    # out = y + GELU(zl W1^T + b1) W2^T + b2,  zl = LN(y)
    g["map_fc2_w"] += np.outer(dout, s["hg"])
    g["map_fc2_b"] += dout
    dh = (dout @ np.asarray(params["map_fc2_w"], F64)) * gelu_grad(s["hpre"])
    g["map_fc1_w"] += np.outer(dh, s["zl"])
    g["map_fc1_b"] += dh
    dzl = dh @ np.asarray(params["map_fc1_w"], F64)
    dyl, dg, db = layernorm_backward(s["y"][None], params["map_ln_g"], dzl[None], eps)
    g["map_ln_g"] += dg
    g["map_ln_b"] += db
    dy = dout + dyl[0]
    # y = o W_o^T + b_o
    g["map_o_w"] += np.outer(dy, s["o"])
    g["map_o_b"] += dy
    do = dy @ np.asarray(params["map_o_w"], F64)
    # one query per head over the N keys and values
    kv = s["kv"]
    dq = np.zeros(dm)
    dkv = np.zeros_like(kv)
    for h in range(heads):
        sl = slice(h * d, (h + 1) * d)
        dqh, dkh, dvh = attention_head_backward(s["q"][None, sl], kv[:, :dm][:, sl],
                                                kv[:, dm:][:, sl], do[None, sl])
        dq[sl] = dqh[0]
        dkv[:, :dm][:, sl] = dkh
        dkv[:, dm:][:, sl] = dvh
    # q = probe W_q^T + b_q;  kv = xl W_kv^T + b_kv
    g["map_q_w"] += np.outer(dq, np.asarray(params["map_probe"], F64))
    g["map_q_b"] += dq
    g["map_probe"] += dq @ np.asarray(params["map_q_w"], F64)
    g["map_kv_w"] += dkv.T @ s["xl"]
    g["map_kv_b"] += dkv.sum(axis=0)
    return dkv @ np.asarray(params["map_kv_w"], F64)


def encode_image_backward(img: np.ndarray, params: Dict, cfg,
                          d_emb: np.ndarray) -> Dict:
    """Gradient of <d_emb, e_hat(img)> with respect to every parameter (same
    structure as params), for the image tower with class-token or
    attention-pooling head."""
    pool = getattr(cfg, "pool", "cls")
    if pool not in ("cls", "map"):
        raise ValueError(f"unknown pooling {pool!r}")
    eps = cfg.ln_eps
    g = _zeros_like_params(params)
    # ---- forward, keeping what the backward needs
    xn = V.normalise_pixels(img, cfg.chan_mean, cfg.chan_std)
    gh, gw = V.patch_grid(xn.shape[1], xn.shape[2], cfg.patch)
    u = V.patchify(xn, cfg.patch)
    x = V.embed_tokens(img, params, cfg)
    saved = []
    for lp in params["layers"]:
        dm = x.shape[1]
        y1 = V.layernorm(x, lp["ln1_g"], lp["ln1_b"], eps)
        qkv = y1 @ np.asarray(lp["qkv_w"], F64).T + np.asarray(lp["qkv_b"], F64)
        d = dm // cfg.heads
        o = np.zeros((x.shape[0], dm))
        for h in range(cfg.heads):
            sl = slice(h * d, (h + 1) * d)
            o[:, sl] = V.attention_head(qkv[:, sl], qkv[:, dm:][:, sl], qkv[:, 2 * dm:][:, sl])
        hres = x + o @ np.asarray(lp["o_w"], F64).T + np.asarray(lp["o_b"], F64)
        y2 = V.layernorm(hres, lp["ln2_g"], lp["ln2_b"], eps)
        z1 = y2 @ np.asarray(lp["fc1_w"], F64).T + np.asarray(lp["fc1_b"], F64)
        gz = V.gelu(z1)
        saved.append((x, y1, qkv, o, hres, y2, z1, gz))
        x = hres + gz @ np.asarray(lp["fc2_w"], F64).T + np.asarray(lp["fc2_b"], F64)
    if pool == "map":
        mp = map_forward(V.layernorm(x, params["lnf_g"], params["lnf_b"], eps), params,
                         cfg.heads, eps)
        z = mp["out"]
    else:
        z = V.layernorm(x[0], params["lnf_g"], params["lnf_b"], eps)
    e = np.asarray(params["proj_w"], F64) @ z
    ne = max(np.linalg.norm(e), 1e-12)
    eh = e / ne
    # ---- backward
    dh_ = np.asarray(d_emb, F64)
    de = (dh_ - eh * (eh @ dh_)) / ne
    g["proj_w"] += np.outer(de, z)
    dz = np.asarray(params["proj_w"], F64).T @ de
    if pool == "map":
        dxl = map_backward(dz, mp, params, cfg.heads, eps, g)
        dx, dgf, dbf = layernorm_backward(x, params["lnf_g"], dxl, eps)
    else:
        dx0, dgf, dbf = layernorm_backward(x[0][None], params["lnf_g"], dz[None], eps)
        dx = np.zeros_like(x)
        dx[0] = dx0[0]
    g["lnf_g"] += dgf
    g["lnf_b"] += dbf
    for lp, gl, (xin, y1, qkv, o, hres, y2, z1, gz) in zip(
            reversed(params["layers"]), reversed(g["layers"]), reversed(saved)):
        dm = xin.shape[1]
        d = dm // cfg.heads
        # x_out = h + GELU(z1) W2^T + b2
        gl["fc2_w"] += dx.T @ gz
        gl["fc2_b"] += dx.sum(axis=0)
        dz1 = (dx @ np.asarray(lp["fc2_w"], F64)) * gelu_grad(z1)
        gl["fc1_w"] += dz1.T @ y2
        gl["fc1_b"] += dz1.sum(axis=0)
        dy2 = dz1 @ np.asarray(lp["fc1_w"], F64)
        dxl, dg2, db2 = layernorm_backward(hres, lp["ln2_g"], dy2, eps)
        gl["ln2_g"] += dg2
        gl["ln2_b"] += db2
        dh = dx + dxl
        # h = x + O Wo^T + bo
        gl["o_w"] += dh.T @ o
        gl["o_b"] += dh.sum(axis=0)
        do = dh @ np.asarray(lp["o_w"], F64)
        dqkv = np.zeros_like(qkv)
        for h in range(cfg.heads):
            sl = slice(h * d, (h + 1) * d)
            dq, dk, dv = attention_head_backward(qkv[:, sl], qkv[:, dm:][:, sl],
                                                 qkv[:, 2 * dm:][:, sl], do[:, sl])
            dqkv[:, sl] = dq
            dqkv[:, dm:][:, sl] = dk
            dqkv[:, 2 * dm:][:, sl] = dv
        gl["qkv_w"] += dqkv.T @ y1
        gl["qkv_b"] += dqkv.sum(axis=0)
        dy1 = dqkv @ np.asarray(lp["qkv_w"], F64)
        dxl, dg1, db1 = layernorm_backward(xin, lp["ln1_g"], dy1, eps)
        gl["ln1_g"] += dg1
        gl["ln1_b"] += db1
        dx = dh + dxl
    # tokens = [cls; u E^T + b] + interp(pos)
    g["cls"] += dx[0]
    g["pos"][0] += dx[0]
    D = dx.shape[1]
    mh = V._interp_matrix(cfg.base_grid, gh)
    mw = V._interp_matrix(cfg.base_grid, gw)
    dgrid = np.einsum("ri,rqd,qj->ijd", mh, dx[1:].reshape(gh, gw, D), mw)
    g["pos"][1:] += dgrid.reshape(-1, D)
    g["patch_w"] += (dx[1:].T @ u).reshape(np.shape(params["patch_w"]))
    g["patch_b"] += dx[1:].sum(axis=0)
    return g


def encode_backward(images: Sequence[np.ndarray], params: Dict, cfg,
                    d_emb: np.ndarray) -> Dict:
    """Gradients of sum_i <d_emb[i], e_hat(images[i])>, summed over images."""
    acc = _zeros_like_params(params)
    for im, de in zip(images, np.asarray(d_emb, F64)):
        _add(acc, encode_image_backward(im, params, cfg, de))
    return acc


def training_step(images: Sequence[np.ndarray], params: Dict, cfg, texts: np.ndarray,
                  head: str, scale: float, bias: float = 0.0):
    """Contrastive loss of the images' embeddings against matched texts and
    its gradients: (loss, parameter gradients, dL/dtexts, dL/dscale,
    dL/dbias)."""
    emb = V.encode(images, params, cfg)
    loss = V.contrastive_loss(emb, texts, head, scale, bias)
    de, dt, ds, db = V.contrastive_grads(emb, texts, head, scale, bias)
    return loss, encode_backward(images, params, cfg, de), dt, ds, db


def flatten_grads(grads: Dict, cfg, layout) -> np.ndarray:
    """Gradients as one float64 vector in the weight blob's order; `layout`
    is the (name, shape) list of the blob (block tensors '<layer>.<name>')."""
    out = []
    for name, shape in layout:
        if "." in name:
            l, t = name.split(".", 1)
            a = grads["layers"][int(l)][t]
        else:
            a = grads[name]
        assert tuple(np.shape(a)) == tuple(shape), (name, np.shape(a), shape)
        out.append(np.asarray(a, F64).reshape(-1))
    return np.concatenate(out)
