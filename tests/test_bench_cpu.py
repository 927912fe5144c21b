"""Host logic of bench.py: the single-GPU guard, the algorithmic FLOP model
and how a committed counter summary is matched to the kernel it describes."""
import hashlib
import json
import os

import bench
import synth


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_flop_model_matches_the_layer_shapes():
    c = synth.MODELS["l14"]
    sizes = [(336, 336)] * 32
    T = 32 * (1 + (336 // 14) ** 2)
    D, F = c.width, c.mlp
    assert bench.op_flops(c, sizes, "fc1_gemm") == 2.0 * T * D * F
    assert bench.op_flops(c, sizes, "qkv_gemm") == 2.0 * T * D * 3 * D
    assert bench.op_flops(c, sizes, "attention") == 32 * 4.0 * 577 ** 2 * D
    per_image = bench.flops_per_image(c, 336)
    layer_ops = sum(bench.op_flops(c, sizes, op) for op in
                    ("qkv_gemm", "oproj_gemm", "fc1_gemm", "fc2_gemm", "attention"))
    # the per-image model adds the patch embedding and the projection
    extra = 32 * (2.0 * 576 * 3 * 14 ** 2 * D + 2.0 * D * c.proj_dim)
    assert abs(32 * per_image - (c.layers * layer_ops + extra)) <= 1e-9 * 32 * per_image


def _profile(root, source_text, records):
    os.makedirs(os.path.join(root, "profiles"))
    os.makedirs(os.path.join(root, "paper_2505_00690_amd", "csrc"))
    with open(os.path.join(root, "paper_2505_00690_amd", "csrc", "k.hpp"), "w") as f:
        f.write(source_text)
    sha = hashlib.sha256(b"kernel v1").hexdigest()
    lines = ["# summary", ""]
    for cfg, fetch, write in records:
        lines.append(json.dumps({"fetch_kib": fetch, "write_kib": write, "fetch_factor": 2.0,
                                 "write_factor": 1.0, "config": cfg, "source": "k.hpp",
                                 "source_sha256": sha}))
        lines.append("")
    with open(os.path.join(root, "profiles", "traffic_fc1_gemm_w.md"), "w") as f:
        f.write("\n".join(lines))


def test_traffic_record_follows_the_tile_configuration(tmp_path, monkeypatch):
    _profile(str(tmp_path), "kernel v1", [("A", 100.0, 10.0), ("B", 200.0, 20.0)])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    f = bench.traffic_from_profile
    assert f("fc1_gemm", "w", {"A"}) == (100.0 * 2 + 10.0) * 1024
    assert f("fc1_gemm", "w", {"B"}) == (200.0 * 2 + 20.0) * 1024
    assert f("fc1_gemm", "w", {"C"}) is None          # configuration never measured
    assert f("fc1_gemm", "w") == (200.0 * 2 + 20.0) * 1024
    assert f("fc2_gemm", "w") is None                 # no summary for the op


def test_traffic_record_dropped_once_the_kernel_source_changes(tmp_path, monkeypatch):
    _profile(str(tmp_path), "kernel v2", [("A", 100.0, 10.0)])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profile("fc1_gemm", "w", {"A"}) is None


def test_oracle_error_and_top1_agreement_host_logic():
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(5))
    ref = rng.standard_normal((6, 16))
    ref /= np.linalg.norm(ref, axis=1, keepdims=True)
    got = ref + 1e-3 * rng.standard_normal(ref.shape)
    e = bench.oracle_error(got, ref, "bf16")
    rel = np.linalg.norm(got - ref, axis=1)
    assert abs(e["max_rel_err"] - rel.max()) < 1e-15 and e["images"] == 6
    assert 0.999 < e["min_cos"] < 1.0
    texts = rng.standard_normal((40, 16))
    texts /= np.linalg.norm(texts, axis=1, keepdims=True)
    top_ref = np.argmax(ref @ texts.T, axis=1)
    top_a = top_ref.copy()
    top_a[0] = (top_a[0] + 1) % 40                 # one disagreement
    r = bench.top1_agreement(top_a, top_ref, got, ref, texts, 10.0, 1e-4)
    assert r["images"] == 6 and abs(r["raw"] - 5 / 6) < 1e-12
    # a row is certified only when its logit gap beats 2 * scale * (||d|| + slack)
    l = 10.0 * ref @ texts.T
    s = np.sort(l, axis=1)
    cert = (s[:, -1] - s[:, -2]) > 2 * 10.0 * (np.linalg.norm(got - ref, axis=1) + 1e-4)
    assert r["certified_images"] == int(cert.sum())


def test_traffic_summary_from_counter_csvs(tmp_path):
    """--summarize-traffic: the largest copy dispatch calibrates each counter,
    GEMM kernel names map to (op, tile configuration), values are averaged
    per dispatch."""
    import csv
    import json as _json

    import bench

    def write(d, counter, rows):
        d.mkdir()
        with open(d / "p_counter_collection.csv", "w", newline="") as f:
            w = csv.writer(f)
            w.writerow(["Kernel_Name", "Counter_Name", "Counter_Value"])
            for name, v in rows:
                w.writerow([name, counter, v])
    k = "void vl::k_gemm_bf16_dl<256, 256, 4, 2, false, 3, 2, 2>(unsigned short const*, int)"
    other = "void vl::k_layernorm<16, true>(float const*)"
    write(tmp_path / "f", "FETCH_SIZE", [("__amd_rocclr_copyBuffer", 4.0),
                                         ("__amd_rocclr_copyBuffer", 131072.0),
                                         (k, 100.0), (k, 300.0), (other, 7.0)])
    write(tmp_path / "w", "WRITE_SIZE", [("__amd_rocclr_copyBuffer", 262144.0), (k, 50.0),
                                         (k, 50.0)])
    recs = [_json.loads(l) for l in
            bench.summarize_traffic(str(tmp_path / "f"), str(tmp_path / "w")).splitlines()]
    assert len(recs) == 1
    r = recs[0]
    assert r["op"] == "fc1_gemm" and r["config"] == "DL_256x256_W4x2"
    assert r["fetch_kib"] == 200.0 and r["write_kib"] == 50.0 and r["dispatches"] == 2
    assert r["fetch_factor"] == 2.0 and r["write_factor"] == 1.0


def test_gemm_kernel_names_map_to_op_configuration_and_source():
    """The summarisers' kernel-name parser: BF16 tile kernels (two- and
    three-stage), MXFP8 tile kernels (their own source file), and names that
    are not block GEMMs."""
    import bench
    assert bench._gemm_config("void vl::k_gemm_bf16_dl<160, 256, 1, 8, false, 4, 2, 3>(x)") == (
        "fc2_gemm", "DL3_160x256_W1x8", "gemm_kernels.hpp")
    assert bench._gemm_config("void vl::k_gemm_bf16_dl<256, 256, 2, 4, false, 1, 2, 2>(x)") == (
        "qkv_gemm", "DL_256x256_W2x4", "gemm_kernels.hpp")
    assert bench._gemm_config("void vl::k_gemm_mx<192, 256, 2, 4, 3, 2>(x)") == (
        "fc1_gemm", "MX_192x256_W2x4", "gemm_mx.hpp")
    assert bench._gemm_config("void vl::k_gemm_mx<160, 256, 1, 8, 2, 2>(x)") == (
        "oproj_gemm", "MX_160x256_W1x8", "gemm_mx.hpp")
    # e4m3-weight variants, the weight-gradient ops and other kernels are not block GEMMs
    assert bench._gemm_config("void vl::k_gemm_bf16_dl<256, 256, 2, 4, true, 3, 2, 2>(x)") is None
    assert bench._gemm_config("void vl::k_gemm_bf16_dl<256, 256, 2, 4, false, 7, 2, 2>(x)") is None
    assert bench._gemm_config("void vl::k_layernorm<16, true>(float const*)") is None
