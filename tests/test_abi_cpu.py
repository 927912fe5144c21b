"""The C-ABI library loads without a GPU, exports every symbol declared in
include/vl.h, and rejects invalid arguments before touching the device."""
import ctypes
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "vl.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(vl_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def V():
    from paper_2505_00690_amd import vl
    vl.lib()
    return vl


def test_every_declared_symbol_is_exported(V):
    declared = _declared_functions()
    assert len(declared) >= 10
    lib = V.lib()
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(V.EXPORTED_SYMBOLS)


def test_abi_version_and_status_strings(V):
    assert V.vl_abi_version() == 2
    assert V.vl_status_string(0) == "ok"
    assert V.vl_status_string(3) == "workspace too small"


def test_weights_count_matches_blob_layout(V):
    for c in synth.MODELS.values():
        assert V.vl_weights_count(c) == synth.weight_count(c)
    bad = synth.ModelConfig("bad", 16, 100, 1, 3, 512, 128, 4)   # width % heads != 0
    assert V.vl_weights_count(bad) == 0


def test_invalid_arguments_rejected_on_host(V):
    lib = V.lib()
    cfg = V.VlConfig.from_model(synth.MODELS["tiny"])
    h = ctypes.c_void_p()
    st = lib.vl_model_create(ctypes.byref(cfg), 1, None, 0, None, ctypes.byref(h))
    assert st == 1 and "NULL" in V.vl_last_error_message()
    st = lib.vl_model_create(ctypes.byref(cfg), 7, ctypes.c_void_p(256), 0, None, ctypes.byref(h))
    assert st == 1
    st = lib.vl_model_create(ctypes.byref(cfg), 1, ctypes.c_void_p(256), 5, None, ctypes.byref(h))
    assert st == 1 and "expected" in V.vl_last_error_message()
    # head_dim 128 is not supported
    c2 = V.VlConfig.from_model(synth.ModelConfig("x", 16, 256, 1, 2, 512, 128, 4))
    n = lib.vl_weights_count(ctypes.byref(c2))
    st = lib.vl_model_create(ctypes.byref(c2), 1, ctypes.c_void_p(256), n, None, ctypes.byref(h))
    assert st == 2
    # scoring argument checks happen before any launch
    p = ctypes.c_void_p(256)
    assert lib.vl_score(p, 4, p, 10, 128, 0, 1.0, 0.0, p, None, None) == 1   # n_texts % 4
    assert "n_texts" in V.vl_last_error_message()
    assert lib.vl_score(p, 4, p, 16, 102, 0, 1.0, 0.0, p, None, None) == 1   # dim % 4
    assert "dim" in V.vl_last_error_message()
    # dim = 100 meets the documented dim % 4: only n_texts is then reported
    assert lib.vl_score(p, 4, p, 10, 100, 0, 1.0, 0.0, p, None, None) == 1
    assert "n_texts" in V.vl_last_error_message()
    assert lib.vl_score(p, 4, p, 16, 128, 0, 1.0, 0.0, ctypes.c_void_p(260), None, None) == 1
    assert lib.vl_score(p, 0, p, 16, 128, 0, 1.0, 0.0, p, None, None) == 1
    assert lib.vl_score(p, 4, p, 16, 128, 5, 1.0, 0.0, p, None, None) == 1   # head
    assert lib.vl_score(None, 4, p, 16, 128, 0, 1.0, 0.0, p, None, None) == 1
    assert lib.vl_encode_images(None, p, None, None, 1, p, p, 0, None) == 1
    assert lib.vl_encode_workspace_bytes(None, 1, None, None) == 0


def test_next_row_entry_points_validate_on_host(V):
    """Argument checks of the text tower, attention pooling, MXFP8 and
    contrastive-loss entry points happen before anything touches a device."""
    lib = V.lib()
    p = ctypes.c_void_p(256)
    h = ctypes.c_void_p()
    # text tower
    tc = synth.TEXT_MODELS["tiny_text"]
    assert V.vl_text_weights_count(tc) == synth.text_weight_count(tc)
    cfg = V.VlTextConfig.from_model(tc)
    assert lib.vl_text_model_create(ctypes.byref(cfg), 1, p, 5, None, ctypes.byref(h)) == 1
    bad = V.VlTextConfig.from_model(synth.TextConfig("b", 10, 2000, 128, 1, 4, 512, 128))
    assert lib.vl_text_weights_count(ctypes.byref(bad)) == 0            # ctx > 1024
    assert lib.vl_encode_texts(None, p, None, 1, p, p, 0, None) == 1
    assert lib.vl_text_workspace_bytes(None, 1, None) == 0
    # attention pooling adds exactly its tensors to the image blob
    for name in ("tiny_map", "b16_map"):
        assert V.vl_weights_count(synth.MODELS[name]) == synth.weight_count(synth.MODELS[name])
    ic = V.VlConfig.from_model(synth.MODELS["tiny"])
    ic.pool = 7
    assert lib.vl_weights_count(ctypes.byref(ic)) == 0
    ic = V.VlConfig.from_model(synth.MODELS["tiny"])
    ic.channels = 5
    assert lib.vl_weights_count(ctypes.byref(ic)) == 0
    # MXFP8
    assert lib.vl_mx_quantize(p, 4, 100, p, p, None) == 1               # cols % 128
    assert lib.vl_mx_gemm(p, p, p, p, 4, 48, 128, p, p, -1, None) == 1  # N % 32
    assert lib.vl_mx_gemm(p, p, p, p, 4, 64, 100, p, p, -1, None) == 1  # K % 128
    assert lib.vl_mx_gemm(p, p, p, p, 4, 64, 128, p, p, 0, None) == 1   # a BF16 config id
    # contrastive losses
    f = lambda *a: lib.vl_contrastive_loss(*a)  # noqa: E731
    assert f(p, p, 8, 100, 0, 10.0, 0.0, p, p, p, p, p, 1 << 30, None) == 1     # dim % 16
    assert f(p, p, 0, 128, 0, 10.0, 0.0, p, p, p, p, p, 1 << 30, None) == 1     # n
    assert f(p, p, 8, 128, 0, 0.0, 0.0, p, p, p, p, p, 1 << 30, None) == 1      # scale
    assert f(p, p, 8, 128, 9, 10.0, 0.0, p, p, p, p, p, 1 << 30, None) == 1     # head
    assert f(p, p, 8, 128, 0, 10.0, 0.0, p, p, p, p, p, 16, None) == 3          # workspace
    assert V.vl_contrastive_workspace_bytes(8, 128) > 0
    assert V.vl_contrastive_workspace_bytes(0, 128) == 0
    # the allocation-free variant: same checks, and sizes past its static
    # scratch are refused before the device is touched
    g = lambda *a: lib.vl_contrastive_loss_noalloc(*a)  # noqa: E731
    assert g(p, p, 8, 100, 0, 10.0, 0.0, p, p, p, p, None) == 1                 # dim % 16
    assert g(p, p, 0, 128, 0, 10.0, 0.0, p, p, p, p, None) == 1                 # n
    assert g(p, p, 8, 128, 0, -1.0, 0.0, p, p, p, p, None) == 1                 # scale
    assert g(p, p, 8, 128, 2, 10.0, 0.0, p, p, p, p, None) == 1                 # head
    assert g(None, p, 8, 128, 0, 10.0, 0.0, p, p, p, p, None) == 1              # NULL
    assert V.vl_contrastive_workspace_bytes(2528, 768) <= V.VL_NOALLOC_SCRATCH_BYTES
    assert V.vl_contrastive_workspace_bytes(2529, 768) > V.VL_NOALLOC_SCRATCH_BYTES
    assert g(p, p, 2529, 768, 0, 10.0, 0.0, p, p, p, p, None) == 3
    assert "scratch" in V.vl_last_error_message()


def test_attention_entry_point_validates_on_host(V):
    """vl_attention's documented constraints, each checked on its own."""
    lib = V.lib()
    p = ctypes.c_void_p(256)
    L = (ctypes.c_int32 * 2)(65, 577)
    nb = lib.vl_attention_workspace_bytes(2, L)
    assert nb >= 2 * 32 + (1 + 5) * 8 and nb % 256 == 0
    assert lib.vl_attention_workspace_bytes(0, L) == 0
    assert lib.vl_attention_workspace_bytes(1, (ctypes.c_int32 * 1)(0)) == 0
    assert lib.vl_attention_workspace_bytes(1, (ctypes.c_int32 * 1)(4097)) == 0
    assert lib.vl_attention_workspace_bytes(1, (ctypes.c_int32 * 1)(4096)) > 0
    f = lambda *a: lib.vl_attention(*a)  # noqa: E731
    assert f(p, 1, L, 2, 0, 64, 0, p, p, nb, None) == 1          # heads
    assert f(p, 1, L, 2, 65, 64, 0, p, p, nb, None) == 1         # heads <= 64
    assert f(p, 1, L, 2, 4, 48, 0, p, p, nb, None) == 2          # head_dim 32 / 64
    assert f(p, 2, L, 2, 4, 64, 0, p, p, nb, None) == 1          # precision
    assert f(None, 1, L, 2, 4, 64, 0, p, p, nb, None) == 1
    assert f(p, 1, L, 2, 4, 64, 0, ctypes.c_void_p(264), p, nb, None) == 1    # out alignment
    assert f(p, 1, L, 2, 4, 64, 0, p, ctypes.c_void_p(384), nb, None) == 1    # ws alignment
    assert f(p, 1, L, 2, 4, 64, 0, p, p, nb - 1, None) == 3      # workspace too small
    assert f(p, 1, (ctypes.c_int32 * 2)(65, 0), 2, 4, 64, 0, p, p, nb, None) == 1


def test_attention_backward_entry_point_validates_on_host(V):
    """vl_attention_backward's documented constraints, each checked on its
    own, and its workspace size from its parts."""
    lib = V.lib()
    p = ctypes.c_void_p(256)
    L = (ctypes.c_int32 * 2)(65, 577)
    T, heads, d = 642, 4, 64
    nb = lib.vl_attention_backward_workspace_bytes(2, L, heads, d)
    up = lambda x: (x + 255) // 256 * 256  # noqa: E731
    # descriptors (2 x 32 B, (2 + 10) 64-token and (1 + 5) 128-token blocks
    # of 8 B), log-sum-exp and D [T, heads] FP32, dO in BF16 [T, heads d]
    want = up(64 + 12 * 8 + 6 * 8) + 2 * up(4 * T * heads) + up(2 * T * heads * d)
    assert nb == want, (nb, want)
    assert lib.vl_attention_backward_workspace_bytes(0, L, heads, d) == 0
    assert lib.vl_attention_backward_workspace_bytes(2, L, 0, d) == 0
    assert lib.vl_attention_backward_workspace_bytes(2, L, heads, 48) == 0
    assert lib.vl_attention_backward_workspace_bytes(1, (ctypes.c_int32 * 1)(4097), heads, d) == 0
    f = lambda *a: lib.vl_attention_backward(*a)  # noqa: E731
    assert f(p, p, p, 1, L, 2, 0, 64, p, p, nb, None) == 1       # heads
    assert f(p, p, p, 1, L, 2, 65, 64, p, p, nb, None) == 1      # heads <= 64
    assert f(p, p, p, 1, L, 2, 4, 48, p, p, nb, None) == 2       # head_dim 32 / 64
    assert f(p, p, p, 2, L, 2, 4, 64, p, p, nb, None) == 1       # precision
    assert f(p, None, p, 1, L, 2, 4, 64, p, p, nb, None) == 1    # O
    assert f(p, p, ctypes.c_void_p(260), 1, L, 2, 4, 64, p, p, nb, None) == 1   # dO alignment
    assert f(p, p, p, 1, L, 2, 4, 64, p, ctypes.c_void_p(384), nb, None) == 1   # ws alignment
    assert f(p, p, p, 1, L, 2, 4, 64, p, p, nb - 1, None) == 3   # workspace too small
    assert f(p, p, p, 1, (ctypes.c_int32 * 2)(65, 0), 2, 4, 64, p, p, nb, None) == 1


def test_tuning_file_entry_points_validate_on_host(V, tmp_path):
    lib = V.lib()
    assert lib.vl_model_save_tuning(None, str(tmp_path / "t.json").encode()) == 1
    assert lib.vl_model_load_tuning(None, str(tmp_path / "t.json").encode()) == 1


def test_binding_checks_buffer_sizes_before_the_call(V):
    """The C ABI cannot see the size of a device buffer; the binding checks
    every tensor against the shapes the call implies and raises ValueError
    (checked here with host tensors, before any device pointer is taken)."""
    import torch
    emb = torch.zeros((3, 128))
    texts = torch.zeros((16, 128))
    with pytest.raises(ValueError, match="scores_out"):
        V.vl_score(emb, texts, "softmax", 100.0, 0.0, torch.zeros((3, 15)))
    with pytest.raises(ValueError, match="scores_out"):
        V.vl_score(emb, texts, "softmax", 100.0, 0.0, torch.zeros((3, 16), dtype=torch.float64))
    with pytest.raises(ValueError, match="top1_out"):
        V.vl_score(emb, texts, "softmax", 100.0, 0.0, torch.zeros((3, 16)),
                   torch.zeros(2, dtype=torch.int32))
    with pytest.raises(ValueError, match="width"):
        V.vl_score(emb, torch.zeros((16, 64)), "softmax", 100.0, 0.0, torch.zeros((3, 16)))
    sizes_h, sizes_w = [64, 48], [64, 80]
    need = 3 * (64 * 64 + 48 * 80)
    ws = torch.zeros(16, dtype=torch.uint8)
    with pytest.raises(ValueError, match="pixels"):
        V.vl_encode_images(None, torch.zeros(need - 1), sizes_h, sizes_w, torch.zeros((2, 128)),
                           ws, proj_dim=128)
    with pytest.raises(ValueError, match="emb_out"):
        V.vl_encode_images(None, torch.zeros(need), sizes_h, sizes_w, torch.zeros((2, 64)), ws,
                           proj_dim=128)
    with pytest.raises(ValueError, match="emb_out"):
        V.vl_encode_images(None, torch.zeros(need), sizes_h, sizes_w, torch.zeros((3, 128)), ws)
    with pytest.raises(ValueError, match="pixels"):      # four planes need more pixels
        V.vl_encode_images(None, torch.zeros(need), sizes_h, sizes_w, torch.zeros((2, 128)), ws,
                           channels=4)
    with pytest.raises(ValueError, match="differ"):
        V.vl_encode_images(None, torch.zeros(need), [64], [64, 80], torch.zeros((2, 128)), ws)
    with pytest.raises(ValueError, match="qkv"):
        V.vl_attention(torch.zeros((10, 3 * 128)), [5, 4], 2, 64, False, torch.zeros((9, 128)))
    with pytest.raises(ValueError, match="out"):
        V.vl_attention(torch.zeros((9, 3 * 128)), [5, 4], 2, 64, False, torch.zeros((9, 64)))
    with pytest.raises(ValueError, match="emb_out"):
        V.vl_encode_texts(None, torch.zeros(9, dtype=torch.int32), [5, 4], torch.zeros((3, 128)),
                          ws)
