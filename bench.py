"""Throughput benchmark of the image-encoder hot path on one MI355X.

A step is one pass of the whole path over one batch: patch embedding, all
transformer blocks, pooling / projection / L2 norm (vl_encode_images), then
the logit GEMM and scoring head against the resident text embeddings
(vl_score).  Inputs are seeded synthetic tensors already resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload l14_336]

Prints one JSON line (rank 0).  Only one GPU is used: --gpus above 1 exits
with a message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

BF16_PEAK = 2.5e15       # MI355X dense BF16 MFMA, FLOP/s
FP8_PEAK = 5.0e15        # MI355X dense FP8 MFMA, FLOP/s
FP32_PEAK = 157.3e12     # MI355X FP32 vector, FLOP/s
HBM_PEAK = 8.0e12        # B/s


def flops_per_image(c: synth.ModelConfig, res: int) -> float:
    """Algorithmic FLOPs (2 per multiply-add, no padding credited)."""
    g = res // c.patch
    npch = g * g
    n = npch + 1
    D, F = c.width, c.mlp
    f = 2.0 * npch * c.channels * c.patch ** 2 * D
    per_layer = 2.0 * n * D * 3 * D + 4.0 * n * n * D + 2.0 * n * D * D + 4.0 * n * D * F
    f += c.layers * per_layer
    f += 2.0 * D * c.proj_dim
    return f


def op_flops(c: synth.ModelConfig, sizes, op: str) -> float:
    """Algorithmic FLOPs of one layer's worth of an encoder operation over the
    whole batch (one launch, or two for a two-part batch)."""
    D, F = c.width, c.mlp
    toks = [1 + (h // c.patch) * (w // c.patch) for h, w in sizes]
    T = sum(toks)
    return {
        "qkv_gemm": 2.0 * T * D * 3 * D,
        "oproj_gemm": 2.0 * T * D * D,
        "fc1_gemm": 2.0 * T * D * F,
        "fc2_gemm": 2.0 * T * F * D,
        "attention": sum(4.0 * n * n * D for n in toks),
        "patch_embed": sum(2.0 * (n - 1) * c.channels * c.patch ** 2 * D for n in toks),
    }.get(op, 0.0)


def traffic_from_profile(op: str, workload: str, configs=None):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None when there is none, the kernel source changed since, or the op now
    runs another tile configuration.  FETCH_SIZE / WRITE_SIZE are each scaled
    by the factor a plain copy of known size measured in the same run."""
    path = os.path.join(ROOT, "profiles", f"traffic_{op}_{workload}.md")
    if not os.path.exists(path):
        return None
    # one record per measured tile configuration; the op's configuration
    # picks its record (without a known configuration: the last record)
    rec = None
    for line in open(path):
        line = line.strip()
        if line.startswith("{") and '"fetch_kib"' in line:
            r = json.loads(line)
            if configs is None or r.get("config") in configs:
                rec = r
    if rec is None:
        return None
    src = os.path.join(ROOT, "paper_2505_00690_amd", "csrc", rec["source"])
    if not os.path.exists(src):
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return (rec["fetch_kib"] * rec["fetch_factor"] + rec["write_kib"] * rec["write_factor"]) * 1024.0


# ------------------------------------------------ profile summaries
# The committed profiles/ summaries are written from rocprofv3 output by
# these two functions (python bench.py --summarize-kernels DIR /
# --summarize-traffic FETCH_DIR WRITE_DIR): kernel times per name and, for the
# block kernels, per workgroup count; and per GEMM tile configuration the
# FETCH_SIZE / WRITE_SIZE per dispatch, calibrated by a plain copy of known
# size in the same run.
_OPS = {"1": "qkv_gemm", "2": "oproj_gemm", "3": "fc1_gemm", "4": "fc2_gemm"}


def _csv(dirpath: str, suffix: str):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(dirpath, "**", "*" + suffix), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {dirpath}")
    return list(csv.DictReader(open(files[0])))


def _gemm_config(name: str):
    """(op, tile configuration name, kernel source) of a BF16 or MXFP8
    block-GEMM kernel name."""
    import re
    m = re.search(r"k_gemm_bf16_dl<(\d+), (\d+), (\d+), (\d+), false, (\d), \d, (\d)>", name)
    if m and m.group(5) in _OPS:
        bm, bn, wm, wn, op, st = m.groups()
        pre = "DL3" if st == "3" else "DL"
        return _OPS[op], f"{pre}_{bm}x{bn}_W{wm}x{wn}", "gemm_kernels.hpp"
    m = re.search(r"k_gemm_mx<(\d+), (\d+), (\d+), (\d+), (\d), \d>", name)
    if m and m.group(5) in _OPS:
        bm, bn, wm, wn, op = m.groups()
        return _OPS[op], f"MX_{bm}x{bn}_W{wm}x{wn}", "gemm_mx.hpp"
    return None


def summarize_kernels(dirpath: str) -> str:
    rows = _csv(dirpath, "kernel_stats.csv")
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        t = float(r["TotalDurationNs"])
        out.append(f"| `{r['Name'].split('(')[0].replace('void ', '')}` | {r['Calls']} | "
                   f"{t / 1e6:.3f} | {float(r['AverageNs']) / 1e3:.1f} | {100 * t / tot:.1f} |")
    trace = _csv(dirpath, "kernel_trace.csv")
    groups = {}
    for r in trace:
        n = r["Kernel_Name"].split("(")[0].replace("void ", "")
        if not any(k in n for k in ("k_gemm_bf16_dl", "k_gemm_mx", "k_attn_bf16", "k_layernorm")):
            continue
        wg = int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        groups.setdefault((n, wg), []).append(d)
    out += ["", "Block kernels by workgroup count:", "",
            "| kernel | workgroups | launches | avg us |", "|---|---|---|---|"]
    for (n, wg), ds in sorted(groups.items()):
        out.append(f"| `{n}` | {wg} | {len(ds)} | {sum(ds) / len(ds):.1f} |")
    return "\n".join(out)


def summarize_traffic(fetch_dir: str, write_dir: str, copy_mib: int = 256) -> str:
    """One JSON record per (GEMM op, tile configuration): mean FETCH_SIZE /
    WRITE_SIZE per dispatch (KiB) and the copy calibration factors."""
    def per_kernel(dirpath, counter):
        acc = {}
        for r in _csv(dirpath, "counter_collection.csv"):
            if r["Counter_Name"] != counter:
                continue
            acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        # the calibration copy is the largest copy dispatch of the run
        cal = max((max(v) for k, v in acc.items() if "copyBuffer" in k), default=None)
        if cal is None:
            raise SystemExit(f"no calibration copy in the {counter} run")
        return ({k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()},
                cal)
    fetch, nf, fcal = per_kernel(fetch_dir, "FETCH_SIZE")
    write, _, wcal = per_kernel(write_dir, "WRITE_SIZE")
    kib = copy_mib * 1024
    ff, wf = kib / fcal, kib / wcal
    out = []
    for k in sorted(fetch):
        oc = _gemm_config(k)
        if oc is None or k not in write:
            continue
        src = oc[2]
        sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2505_00690_amd", "csrc", src),
                                  "rb").read()).hexdigest()
        rec = {"op": oc[0], "fetch_kib": round(fetch[k], 1), "write_kib": round(write[k], 1),
               "fetch_factor": round(ff, 4), "write_factor": round(wf, 4),
               "copy_fetch_kib": round(fcal, 1), "copy_write_kib": round(wcal, 1),
               "copy_kib": kib, "kernel": k.split("(")[0].replace("void vl::", ""),
               "config": oc[1], "dispatches": nf[k], "source": src, "source_sha256": sha}
        out.append(json.dumps(rec))
    return "\n".join(out)


def summarize_counters(*dirs: str) -> str:
    """Per kernel of one or more rocprofv3 --pmc runs: dispatches and the
    mean per dispatch of every counter collected, with the derived ratios
    the counters give (MFMA busy share of SIMD cycles, share of wave cycles
    spent waiting on any dependency, BF16 MFMA FLOPs issued)."""
    vals, disp = {}, {}
    for d in dirs:
        for r in _csv(d, "counter_collection.csv"):
            n = r["Kernel_Name"].split("(")[0].replace("void ", "")
            if not n.startswith("vl::"):
                continue
            vals.setdefault(n, {}).setdefault(r["Counter_Name"], []).append(
                float(r["Counter_Value"]))
            disp.setdefault(n, set()).add((d, r["Dispatch_Id"]))
    out = ["| kernel | dispatches | MFMA busy % | waiting % of wave cycles | "
           "BF16 MFMA GFLOP per dispatch |", "|---|---|---|---|---|"]
    for n in sorted(vals, key=lambda k: -sum(vals[k].get("SQ_WAVE_CYCLES", [0]))):
        c = {k: sum(v) / len(v) for k, v in vals[n].items()}
        util = c.get("MfmaUtil")
        wait = (100.0 * c["SQ_WAIT_INST_ANY"] / c["SQ_WAVE_CYCLES"]
                if c.get("SQ_WAVE_CYCLES") else None)
        fl = c.get("SQ_INSTS_VALU_MFMA_MOPS_BF16")
        f = lambda x, fmt: "-" if x is None else format(x, fmt)  # noqa: E731
        out.append(f"| `{n}` | {len(disp[n]) // max(1, len(dirs))} | {f(util, '.1f')} | "
                   f"{f(wait, '.1f')} | {f(None if fl is None else fl * 512 / 1e9, '.2f')} |")
    return "\n".join(out)


def cpu_baseline(wl: synth.Workload, blob: np.ndarray, images, texts, n_sample: int,
                 precision: str = None, one_thread: bool = True):
    """The FP64 oracle as it stands, on the host cores, over a bounded
    sample of the same workload: encode + score of n_sample images."""
    from oracle import vit64 as O
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()
                       if i.get("user_api") == "blas"] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    c = synth.MODELS[wl.model]
    precision = precision or wl.precision
    params = O.weights_for(synth.blob_to_params(c, blob), precision)
    sample = images[:n_sample]
    t0 = time.perf_counter()
    emb = O.encode(sample, params, c, act="mx" if precision == "mxfp8" else "none")
    O.score(emb, texts, wl.head, wl.scale, wl.bias)
    dt = time.perf_counter() - t0
    out = {"value": n_sample / dt, "unit": "images/s", "cores": int(threads), "kind": "oracle",
           "cpu": _cpu_model(),
           "sample": f"{n_sample} of {len(images)} images of the workload "
                     f"({wl.model}, {images[0].shape[1]}x{images[0].shape[2]}), FP64 encode + "
                     f"{wl.head} scoring vs {len(texts)} texts; {dt:.1f} s"}
    if one_thread:
        # the same oracle on one BLAS thread, one image
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1):
                t0 = time.perf_counter()
                O.encode(sample[:1], params, c, act="mx" if precision == "mxfp8" else "none")
                dt1 = time.perf_counter() - t0
            out["value_1thread"] = 1.0 / dt1
            out["sample_1thread"] = f"1 image on 1 BLAS thread; {dt1:.1f} s"
        except ImportError:  # pragma: no cover
            pass
    return out, emb


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_error(got: np.ndarray, ref: np.ndarray, precision: str) -> dict:
    """Error of GPU embeddings against the FP64 oracle's on the same images:
    per-image relative error ||e - e_ref|| / ||e_ref|| and cosine."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    rel = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    cos = (got * ref).sum(1) / np.linalg.norm(got, axis=1) / np.linalg.norm(ref, axis=1)
    bar = "rel err <= 1e-4" if precision == "fp32" else "cos >= 0.999"
    return {"precision": precision, "images": int(len(ref)), "max_rel_err": float(rel.max()),
            "min_cos": float(cos.min()), "bar": bar}


def top1_agreement(top_a: np.ndarray, top_ref: np.ndarray, emb_a: np.ndarray,
                   emb_ref: np.ndarray, texts: np.ndarray, scale: float, slack: float) -> dict:
    """Top-1 agreement of a reduced-precision path with the FP32 path: raw,
    and over the images whose FP32 top-1/top-2 logit gap exceeds 2 * scale *
    (||e_a - e_ref|| + slack), where no embedding error of that size can
    change the choice (slack: the FP32 path's own bound against the oracle)."""
    l = scale * (np.asarray(emb_ref, np.float64) @ np.asarray(texts, np.float64).T)
    srt = np.sort(l, axis=1)
    gap = srt[:, -1] - srt[:, -2]
    d = np.linalg.norm(np.asarray(emb_a, np.float64) - np.asarray(emb_ref, np.float64), axis=1)
    cert = gap > 2.0 * scale * (d + slack)
    agree = np.asarray(top_a) == np.asarray(top_ref)
    return {"images": int(len(agree)), "raw": float(agree.mean()),
            "certified_images": int(cert.sum()),
            "certified_agree": float(agree[cert].mean()) if cert.any() else None,
            "vs": "fp32 GPU path",
            "note": "random unit texts: most top-1/top-2 logit gaps lie below the change the "
                    "BF16 embedding error can make, so raw agreement measures ties; only "
                    "certified images are decided by the model"}


def text_leg(torch, vl, n_texts: int, steps: int, seed: int = 3002, split: bool = True):
    """The text tower: CLIP ViT-L/14-shaped (width 768, 12 causal blocks,
    context 77), BF16, HIP graphs; n_texts prompt-length token sequences
    (U{5..20} tokens, one in ten at 77) encoded in one call, as the texts the
    scoring head keeps resident are produced."""
    c = synth.TEXT_MODELS["l14_text"]
    w = torch.from_numpy(synth.make_text_blob(c, seed)).cuda()
    lens = synth.draw_text_lengths(n_texts, c.ctx, seed + 1)
    ids = torch.from_numpy(np.concatenate(synth.make_token_ids(lens, c.vocab, seed + 2))).cuda()
    enc = vl.TextEncoder(c, w, "bf16", graphs=True)
    if split:
        vl.vl_model_set_option(enc.handle, vl.VL_OPT_SPLIT, 1)
    del w
    out = torch.empty((n_texts, c.proj_dim), dtype=torch.float32, device="cuda")
    for _ in range(2):
        enc.encode(ids, lens, out=out)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        enc.encode(ids, lens, out=out)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    T = int(sum(lens))
    D, F = c.width, c.mlp
    flops = c.layers * (2.0 * T * D * (3 * D + D + 2 * F) + sum(2.0 * n * (n + 1) * D for n in lens))
    enc.close()
    return {"value": n_texts / (ms / 1e3), "unit": "texts/s", "ms_per_call": ms,
            "texts": n_texts, "tokens": T, "model": c.name, "precision": "bf16",
            "tflops": flops / (ms / 1e3) / 1e12, "steps": steps, "two_part_split": split}


def rgbd_leg(torch, vl, steps: int, n_env: int = 256, w_seed: int = 1006, i_seed: int = 2006,
             split: bool = True):
    """The navigation benchmark's observation batch: one RGB-D 128x128 frame
    (4 planes) per environment for 256 environments on one GPU, encoded by
    a ViT-S/16-shaped tower in BF16 with HIP graphs (the policy network
    itself is not specified, so the encoder size is a choice)."""
    c = synth.MODELS["rgbd_s16"]
    w = torch.from_numpy(synth.make_blob(c, w_seed)).cuda()
    imgs = synth.make_images([(128, 128)] * n_env, i_seed, channels=c.channels)
    pix = torch.from_numpy(np.concatenate([im.reshape(-1) for im in imgs])).cuda()
    sizes = [(128, 128)] * n_env
    enc = vl.Encoder(c, w, "bf16", graphs=True, split=split)
    vl.vl_model_set_option(enc.handle, vl.VL_OPT_GRAPH_BUCKETS, 0)   # one fixed batch
    del w
    out = torch.empty((n_env, c.proj_dim), dtype=torch.float32, device="cuda")
    for _ in range(2):
        enc.encode(pix, sizes, out=out)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(steps):
        enc.encode(pix, sizes, out=out)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / steps
    flops = n_env * flops_per_image(c, 128)
    enc.close()
    return {"value": n_env / (ms / 1e3), "unit": "observations/s", "ms_per_batch": ms,
            "environments": n_env, "frame": "4x128x128", "model": c.name, "precision": "bf16",
            "tflops": flops / (ms / 1e3) / 1e12, "steps": steps, "two_part_split": split}


def train_leg(torch, vl, steps: int, model: str = "l14", res: int = 336, batch: int = 32,
              w_seed: int = 1002, i_seed: int = 2002, t_seed: int = 3007):
    """Contrastive training step through the image tower: the training
    forward (activations kept), the sigmoid loss of the batch against its
    matched texts (SigLIP, scale 10, bias -10) with its embedding gradient,
    and the backward pass to every weight gradient; BF16 operands, FP32
    accumulation.  The optimizer update is the caller's and is not timed.
    FLOPs credited: 3x the forward's (the usual training count; the score
    recomputations of the attention backward are not credited)."""
    c = synth.MODELS[model]
    w = torch.from_numpy(synth.make_blob(c, w_seed)).cuda()
    sizes = [(res, res)] * batch
    imgs = synth.make_images(sizes, i_seed, channels=c.channels)
    pix = torch.from_numpy(np.concatenate([im.reshape(-1) for im in imgs])).cuda()
    texts = torch.from_numpy(synth.make_texts(batch, c.proj_dim, t_seed)).cuda()
    tr = vl.Trainer(c, w, "bf16", split=True)   # the forward as two overlapped halves
    del w
    emb = torch.empty((batch, c.proj_dim), dtype=torch.float32, device="cuda")
    grads = torch.empty(vl.vl_weights_count(c), dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    de = torch.empty_like(emb)
    dt = torch.empty_like(texts)
    dsb = torch.empty(2, dtype=torch.float32, device="cuda")

    def step(evs=None):
        if evs:
            evs[0].record()
        tr.forward(pix, sizes, out=emb)
        if evs:
            evs[1].record()
        vl.vl_contrastive_loss_noalloc(emb, texts, "sigmoid", 10.0, -10.0, loss, de, dt, dsb)
        if evs:
            evs[2].record()
        tr.backward(pix, sizes, de, grads_out=grads)
        if evs:
            evs[3].record()

    for _ in range(2):
        step()
    torch.cuda.synchronize()
    ph = np.zeros(3)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(steps):
        step()
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / steps
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    step(evs)
    torch.cuda.synchronize()
    for k in range(3):
        ph[k] = evs[k].elapsed_time(evs[k + 1])
    flops = 3.0 * batch * flops_per_image(c, res)
    g = grads.cpu().numpy()
    tr.close()
    return {"value": batch / (ms / 1e3), "unit": "images/s", "ms_per_step": ms,
            "model": c.name, "resolution": res, "batch": batch, "precision": "bf16",
            "loss": "sigmoid (scale 10, bias -10), matched random texts",
            "schedule": "forward as two overlapped halves; weight gradients on a second "
                        "stream beside the input-gradient chain",
            "ms_forward": ph[0], "ms_loss": ph[1], "ms_backward": ph[2],
            "tflops_3x_forward": flops / (ms / 1e3) / 1e12,
            "grads_finite": bool(np.isfinite(g).all()), "steps": steps,
            "loss_value": float(loss.item())}


def serving_leg(torch, vl, n_requests: int, warmup_requests: int, slots: int,
                budget_gib: float, max_batch_images: int, graphs: bool = True):
    """The serving workload: ViT-L/14 with e4m3 per-row weights and BF16
    activations, 8192 resident texts, Poisson requests of 1-16 images at one
    of {224, 336, 384, 448} each.  Closed-loop capacity first (every request
    queued at t=0), then open-loop Poisson arrivals at 0.5x and 0.8x of that
    capacity; nearest-rank p50/p99 of arrival-to-completion latency.  With
    graphs, every batch replays the HIP graph of its capacity bucket on its
    slot (captured on the bucket's first batch); each run reports the share
    of its batches that replayed an existing graph."""
    from paper_2505_00690_amd.serve import GpuExecutor, RealClock, Request, Scheduler
    wl = synth.WORKLOADS["l14_serve"]
    c = synth.MODELS[wl.model]
    seeds = synth.seeds_for(wl)
    w = torch.from_numpy(synth.make_blob(c, seeds["weights"])).cuda()
    enc = vl.Encoder(c, w, wl.precision)
    del w
    texts = torch.from_numpy(synth.make_texts(wl.n_texts, c.proj_dim, seeds["texts"])).cuda()
    # A pool of 32 distinct images per resolution; requests draw from it.
    pool = {r: [torch.from_numpy(im.reshape(-1)).cuda()
                for im in synth.make_images([(r, r)] * 32, seeds["images"] + r)]
            for r in wl.resolutions}
    # tune the GEMM tiles once on a representative batch (32 images, mixed sizes)
    tsizes = [(r, r) for r in wl.resolutions for _ in range(8)]
    enc.autotune(torch.cat([pool[h][k % 32] for k, (h, _) in enumerate(tsizes)]), tsizes, reps=2)
    if graphs:   # after tuning: the tile choice is part of what a graph holds
        vl.vl_model_set_option(enc.handle, vl.VL_OPT_GRAPHS, 1)
    ex = GpuExecutor(enc, texts, wl.head, wl.scale, wl.bias, slots, keep_workspaces=graphs)
    budget = int(budget_gib * 2 ** 30)
    sched = Scheduler(ex, budget, slots=slots, max_batch_images=max_batch_images)

    def make(n, qps, seed):
        out = []
        for i, r in enumerate(synth.draw_requests(n, qps, wl.resolutions, seed)):
            res = r.sizes[0][0]
            out.append(Request(i, r.arrival_s, r.sizes,
                               [pool[res][(i * 7 + k) % 32] for k in range(len(r.sizes))]))
        return out

    def run(reqs):
        g0 = enc.graph_stats()
        st = sched.run(reqs, RealClock())
        torch.cuda.synchronize()
        g1 = enc.graph_stats()
        keep = [x for x in st.results if x.rid >= warmup_requests]
        lat = sorted(x.latency for x in keep)
        imgs = sum(x.n_images for x in st.results)
        from paper_2505_00690_amd.serve import percentile
        return {"images_per_s": imgs / st.wall, "requests_per_s": len(st.results) / st.wall,
                "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
                "batches": st.batches, "max_inflight": st.max_inflight,
                "peak_workspace_gib": st.peak_budget / 2 ** 30, "requests": len(st.results),
                "graph_captures": g1["captures"] - g0["captures"],
                "graph_hit_rate": (1.0 - (g1["captures"] - g0["captures"]) / st.batches
                                   if graphs and st.batches else None)}

    run(make(64, 1e9, seeds["arrivals"] + 99))   # warm-up (plans, allocator)
    cap = run(make(max(200, n_requests // 3), 1e9, seeds["arrivals"]))
    out = {"workload": "l14_serve", "precision": wl.precision, "slots": slots,
           "graphs": graphs,
           "budget_gib": budget_gib, "max_batch_images": max_batch_images,
           "capacity": cap, "open_loop": []}
    for frac in (0.5, 0.8):
        qps = frac * cap["requests_per_s"]
        r = run(make(n_requests, qps, seeds["arrivals"] + int(frac * 10)))
        r["qps"] = qps
        r["load"] = frac
        out["open_loop"].append(r)
    enc.close()
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="l14_336", choices=["tiny_fp32", "b16_224", "l14_336",
                                                             "b16_mixed"])
    ap.add_argument("--precision", default=None,
                    help="fp32 | bf16 | fp8w | mxfp8 (default: workload's)")
    ap.add_argument("--no-graphs", action="store_true")
    ap.add_argument("--bucket-graphs", action="store_true",
                    help="replay the timed batch from its capacity bucket's graph (the serving "
                         "mode) instead of a graph keyed on the exact batch")
    ap.add_argument("--no-autotune", action="store_true", help="use the built-in tile heuristic")
    ap.add_argument("--gemm-tiles", default="",
                    help="fixed tile configurations instead of autotuning, e.g. "
                         "fc1_gemm=DL_256x256_W4x2,qkv_gemm=DL_256x256_W4x2 (other ops: heuristic)")
    ap.add_argument("--no-split", action="store_true",
                    help="time the batch as one part (default for BF16 / FP8 / MXFP8: two "
                         "parts of consecutive images overlapped on two streams)")
    ap.add_argument("--fp32-steps", type=int, default=2, help="steps of the plain FP32 path")
    ap.add_argument("--cpu-sample", type=int, default=None, help="images for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-1thread", action="store_true",
                    help="skip the one-thread oracle figure (one image)")
    ap.add_argument("--timing-steps", type=int, default=3)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving (p50/p99) leg")
    ap.add_argument("--no-text", action="store_true", help="skip the text-tower leg")
    ap.add_argument("--no-rgbd", action="store_true", help="skip the RGB-D observation leg")
    ap.add_argument("--text-steps", type=int, default=5)
    ap.add_argument("--summarize-kernels", metavar="DIR", default=None,
                    help="print the kernel-time tables of a rocprofv3 --kernel-trace --stats "
                         "output directory and exit")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR", default=None,
                    help="print per-kernel SQ counter ratios of rocprofv3 --pmc runs")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    default=None, help="print the GEMM traffic records of two rocprofv3 "
                    "--pmc runs (FETCH_SIZE, WRITE_SIZE) and exit")
    ap.add_argument("--no-attn-resident", action="store_true",
                    help="stream key / value tiles per 128-query block for every image")
    ap.add_argument("--fused-ln", action="store_true",
                    help="fold the LayerNorms into the GEMMs (measured slower; off by default)")
    ap.add_argument("--no-train", action="store_true",
                    help="skip the contrastive training-step leg")
    ap.add_argument("--train-steps", type=int, default=3)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this many MiB first, so "
                         "a counter run can scale FETCH_SIZE / WRITE_SIZE by a copy of known size")
    ap.add_argument("--serve-requests", type=int, default=1200)
    ap.add_argument("--serve-slots", type=int, default=2)
    ap.add_argument("--serve-eager", action="store_true",
                    help="serving leg without graph replay (eager launches)")
    ap.add_argument("--serve-budget-gib", type=float, default=16.0)
    ap.add_argument("--serve-max-batch", type=int, default=32,
                    help="images per serving batch at most (32: same capacity as 64, "
                         "shorter tail latency)")
    args = ap.parse_args(argv)
    if args.summarize_kernels:
        print(summarize_kernels(args.summarize_kernels))
        return 0
    if args.summarize_counters:
        print(summarize_counters(*args.summarize_counters))
        return 0
    if args.summarize_traffic:
        print(summarize_traffic(*args.summarize_traffic, args.copy_calibration_mib or 256))
        return 0

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (images are "
              "independent, so each GPU would encode its share of a batch with its own "
              "weight replica).",
              file=sys.stderr)
        return 2

    import torch
    from paper_2505_00690_amd import vl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    wl = synth.WORKLOADS[args.workload]
    prec = args.precision or wl.precision
    c = synth.MODELS[wl.model]
    seeds = synth.seeds_for(wl)
    if len(wl.resolutions) == 1:
        sizes = [(wl.resolutions[0],) * 2] * wl.n_images
    else:
        sizes = [(r, r) for r in synth.draw_resolutions(wl.n_images, wl.resolutions,
                                                        seeds["resolutions"])]
    t0 = time.time()
    blob = synth.make_blob(c, seeds["weights"])
    images = synth.make_images(sizes, seeds["images"])
    texts = synth.make_texts(wl.n_texts, c.proj_dim, seeds["texts"])
    print(f"# inputs generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    if args.copy_calibration_mib > 0:
        n_el = args.copy_calibration_mib * 2 ** 20 // 4
        src = torch.ones(n_el, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"# copy calibration: {args.copy_calibration_mib} MiB read + written",
              file=sys.stderr, flush=True)
        del src, dst
    w = torch.from_numpy(blob).to(dev)
    pix = torch.from_numpy(np.concatenate([im.reshape(-1) for im in images])).to(dev)
    tx = torch.from_numpy(texts).to(dev)
    n = len(sizes)
    emb = torch.empty((n, c.proj_dim), dtype=torch.float32, device=dev)
    scores = torch.empty((n, wl.n_texts), dtype=torch.float32, device=dev)
    top1 = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    split = prec != "fp32" and not args.no_split
    named = None
    if args.gemm_tiles:
        named = {}
        for item in args.gemm_tiles.split(","):
            op, cfg = item.split("=")
            named[op.strip()] = {str(b): cfg.strip() for b in range(vl.VL_N_M_BUCKETS)}

    def make_encoder(two_parts: bool):
        e = vl.Encoder(c, w, prec, graphs=not args.no_graphs, split=two_parts,
                       fused_ln=args.fused_ln)
        if args.no_attn_resident:
            vl.vl_model_set_option(e.handle, vl.VL_OPT_ATTN_RESIDENT, 0)
        if not args.bucket_graphs:   # a fixed batch: graphs keyed on it exactly
            vl.vl_model_set_option(e.handle, vl.VL_OPT_GRAPH_BUCKETS, 0)
        t = None
        if prec != "fp32" and named:
            e.set_tuning(named)
            t = named
            print(f"# fixed GEMM tiles: {args.gemm_tiles}", file=sys.stderr, flush=True)
        elif prec != "fp32" and not args.no_autotune:
            t = e.autotune(pix, sizes, reps=3)
            print(f"# autotuned GEMM tiles ({'two parts' if two_parts else 'one part'}): {t}",
                  file=sys.stderr, flush=True)
        return e, t

    enc, tuned = make_encoder(split)

    def step(e):
        e.encode(pix, sizes, out=emb)
        vl.vl_score(emb, tx, wl.head, wl.scale, wl.bias, scores, top1)

    for _ in range(args.warmup):
        step(enc)
    torch.cuda.synchronize()
    emb_main = emb.cpu().numpy()
    top_main = top1.cpu().numpy()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step(enc)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    value = n / (ms / 1e3)
    print(f"# {prec}: {ms:.3f} ms/step, {value:.1f} images/s", file=sys.stderr, flush=True)
    # The spread of single steps, after the timed region: each of `args.steps`
    # more steps between its own pair of events on the call's stream.
    pev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in pev:
        a.record(stream)
        step(enc)
        b.record(stream)
    torch.cuda.synchronize()
    from paper_2505_00690_amd.serve import percentile
    per_step = [a.elapsed_time(b) for a, b in pev]
    step_spread = {"steps": len(per_step), "p10_ms": percentile(per_step, 10),
                   "p50_ms": percentile(per_step, 50), "p90_ms": percentile(per_step, 90)}

    # Per-operation device time: events around every launch, on its stream.
    # It is taken on the one-part schedule: with two parts the kernels of one
    # part run beside the other's, so a launch's duration no longer measures
    # that kernel alone (the roofline below is a per-kernel rate).
    tenc, ttuned = (make_encoder(False) if split else (enc, tuned))
    if split:
        for _ in range(2):
            step(tenc)
    vl.vl_model_set_option(tenc.handle, vl.VL_OPT_TIMING, 1)
    vl.vl_model_op_times(tenc.handle, reset=True)
    for _ in range(args.timing_steps):
        step(tenc)
    torch.cuda.synchronize()
    ops = vl.vl_model_op_times(tenc.handle, reset=True)
    vl.vl_model_set_option(tenc.handle, vl.VL_OPT_TIMING, 0)
    if split:
        tenc.close()
        del tenc
    breakdown = {k: round(v[0] / args.timing_steps, 4) for k, v in ops.items() if v[1]}
    gemm_like = ["qkv_gemm", "oproj_gemm", "fc1_gemm", "fc2_gemm", "attention"]
    dom = max(gemm_like, key=lambda k: ops[k][0])
    avg_s = ops[dom][0] / ops[dom][1] / 1e3
    # (a two-part batch launches every op twice per layer: per-launch work is
    # the op's work per step over its launches per step)
    flops_launch = op_flops(c, sizes, dom) * c.layers / (ops[dom][1] / args.timing_steps)
    achieved = flops_launch / avg_s
    fp8_note = prec == "fp8w"
    roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved / 1e12,
                "peak": BF16_PEAK / 1e12, "unit": "TFLOP/s", "frac": achieved / BF16_PEAK,
                "avg_launch_ms": avg_s * 1e3,
                "flops_per_launch": flops_launch,
                "traffic": traffic_from_profile(
                    dom, args.workload + ("_mxfp8" if prec == "mxfp8" else ""),
                    set(ttuned[dom].values()) if ttuned and dom in ttuned else None),
                "schedule": "one part (the timed steps run two overlapped parts)" if split
                            else "one part"}
    if prec == "fp32":
        roofline.update({"peak": FP32_PEAK / 1e12, "frac": achieved / FP32_PEAK, "bound": "alu"})
    if prec == "mxfp8" and dom != "attention":
        roofline.update({"peak": FP8_PEAK / 1e12, "frac": achieved / FP8_PEAK})

    total_flops = sum(flops_per_image(c, h) for h, _ in sizes)
    result = {
        "metric": "images/sec ViT-L/14@336 bf16 vs fp32 plain, same GPU; p50/p99 latency @ QPS",
        "value": value, "unit": "images/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"fp32": "f32", "bf16": "bf16", "fp8w": "fp8w-bf16a", "mxfp8": "mxfp8"}[prec],
        "data": "synthetic (seeded U[0,1] pixels, N(0,0.02^2) weights, unit random texts)",
        "config": {"workload": args.workload, "model": wl.model, "batch": n,
                   "resolutions": sorted(set(h for h, _ in sizes)), "precision": prec,
                   "head": wl.head, "n_texts": wl.n_texts, "graphs": (False if args.no_graphs else
                                                "capacity bucket" if args.bucket_graphs else "exact"),
                   "two_part_split": split,
                   "fused_layernorm": prec in ("bf16", "fp8w") and args.fused_ln,
                   "gemm_tiles": tuned, "gemm_tiles_one_part": ttuned},
        "encoder_tflops": total_flops / (ms / 1e3) / 1e12,
        "mfu_bf16": total_flops / (ms / 1e3) / BF16_PEAK,
        "op_ms_per_step": breakdown,
        "step_ms_spread": step_spread,
        "roofline": roofline,
    }
    if fp8_note:
        result["roofline"]["note"] = "weight-only e4m3: MFMA runs in BF16"

    if args.fp32_steps > 0 and prec != "fp32":
        del enc
        torch.cuda.synchronize()
        enc32 = vl.Encoder(c, w, "fp32", graphs=not args.no_graphs)
        step(enc32)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.fp32_steps):
            step(enc32)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms32 = ev0.elapsed_time(ev1) / args.fp32_steps
        result["fp32_path"] = {"value": n / (ms32 / 1e3), "unit": "images/s",
                               "ms_per_step": ms32, "steps": args.fp32_steps,
                               "speedup_of_value": ms32 / ms}
        emb32 = emb.cpu().numpy()
        result["top1_agreement"] = top1_agreement(top_main, top1.cpu().numpy(), emb_main,
                                                  emb32, texts, wl.scale, 1e-4)
        del enc32

    if not args.no_text:
        result["text_tower"] = text_leg(torch, vl, wl.n_texts, args.text_steps,
                                        split=not args.no_split)
        print(f"# text tower: {json.dumps(result['text_tower'])}", file=sys.stderr, flush=True)

    if not args.no_rgbd:
        result["rgbd_observations"] = rgbd_leg(torch, vl, args.text_steps,
                                               split=not args.no_split)
        print(f"# rgbd: {json.dumps(result['rgbd_observations'])}", file=sys.stderr, flush=True)

    if not args.no_train:
        result["train_step"] = train_leg(torch, vl, args.train_steps)
        print(f"# train step: {json.dumps(result['train_step'])}", file=sys.stderr, flush=True)

    if not args.no_serve:
        result["serving"] = serving_leg(torch, vl, args.serve_requests, 100, args.serve_slots,
                                        args.serve_budget_gib, args.serve_max_batch,
                                        graphs=not args.serve_eager)
        print(f"# serving: {json.dumps(result['serving'])}", file=sys.stderr, flush=True)

    if not args.no_cpu_baseline:
        k = args.cpu_sample or {"tiny_fp32": 8, "b16_224": 8, "l14_336": 4, "b16_mixed": 6}[
            args.workload]
        result["cpu_baseline"], ref = cpu_baseline(wl, blob, images, texts, k, prec,
                                                   one_thread=not args.no_cpu_1thread)
        # error against the FP64 oracle beside the throughput, on the same
        # sample: the timed path, and the plain FP32 path on two images
        errs = [oracle_error(emb_main[:k], ref, prec)]
        if prec != "fp32" and "fp32_path" in result:
            from oracle import vit64 as O
            p32 = O.weights_for(synth.blob_to_params(c, blob), "fp32")
            ref32 = O.encode(images[:2], p32, c)
            errs.append(oracle_error(emb32[:2], ref32, "fp32"))
        result["oracle_err"] = errs
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
