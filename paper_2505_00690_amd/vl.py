"""Python binding of libvl.so (ctypes).  Argument marshalling only: every
step of the encoder and of the scoring head runs in the library's HIP
kernels.  PyTorch supplies device memory and streams.

The functions mirror the C ABI in include/vl.h one to one (same names, same
argument order, tensors in place of device pointers); `Encoder` is a thin
convenience wrapper that owns a model handle and a workspace tensor.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

__all__ = [
    "VlError", "VlConfig", "lib", "library_path", "VL_FP32", "VL_BF16", "VL_FP8W_BF16A",
    "VL_HEAD_SOFTMAX", "VL_HEAD_SIGMOID", "VL_OPT_GRAPHS", "VL_OPT_TIMING", "VL_OPT_SPLIT",
    "VL_OPT_GRAPH_BUCKETS", "VL_OPT_KMAJOR_WGRAD",
    "VL_N_OPS", "OP_NAMES", "vl_model_op_times", "PRECISIONS", "HEADS",
    "vl_abi_version", "vl_weights_count", "vl_model_create", "vl_model_destroy",
    "vl_model_set_option", "vl_encode_workspace_bytes", "vl_encode_images", "vl_score",
    "vl_status_string", "vl_last_error_message", "Encoder", "EXPORTED_SYMBOLS",
    "vl_gemm_config_count", "vl_gemm_config_name", "vl_model_get_tuning",
    "vl_model_set_tuning", "vl_model_autotune", "GEMM_OPS", "VL_MXFP8", "vl_mx_quantize",
    "vl_mx_gemm", "VlTextConfig", "vl_text_weights_count", "vl_text_model_create",
    "vl_text_workspace_bytes", "vl_encode_texts", "TextEncoder", "VL_POOL_CLS", "VL_POOL_MAP",
    "POOLS", "vl_contrastive_workspace_bytes", "vl_contrastive_loss",
    "vl_attention_workspace_bytes", "vl_attention", "vl_model_save_tuning",
    "vl_model_load_tuning", "vl_contrastive_loss_noalloc", "VL_NOALLOC_SCRATCH_BYTES",
    "vl_train_workspace_bytes", "vl_encode_images_train", "vl_encode_images_backward", "Trainer",
    "vl_bf16_round", "vl_fp8_quantize_rows", "vl_model_graph_stats",
    "vl_attention_backward_workspace_bytes", "vl_attention_backward",
]

VL_FP32, VL_BF16, VL_FP8W_BF16A, VL_MXFP8 = 0, 1, 2, 3
VL_HEAD_SOFTMAX, VL_HEAD_SIGMOID = 0, 1
VL_OPT_GRAPHS, VL_OPT_TIMING, VL_OPT_SPLIT, VL_OPT_FUSED_LN, VL_OPT_ATTN_RESIDENT = 0, 1, 2, 3, 4
VL_OPT_GRAPH_BUCKETS = 5
VL_OPT_KMAJOR_WGRAD = 6
VL_N_OPS = 8
OP_NAMES = ("patch_embed", "layernorm", "qkv_gemm", "attention", "oproj_gemm", "fc1_gemm",
            "fc2_gemm", "pool_proj_l2")
PRECISIONS = {"fp32": VL_FP32, "bf16": VL_BF16, "fp8w": VL_FP8W_BF16A, "mxfp8": VL_MXFP8}
HEADS = {"softmax": VL_HEAD_SOFTMAX, "sigmoid": VL_HEAD_SIGMOID}
VL_POOL_CLS, VL_POOL_MAP = 0, 1
POOLS = {"cls": VL_POOL_CLS, "map": VL_POOL_MAP}

EXPORTED_SYMBOLS = (
    "vl_abi_version", "vl_status_string", "vl_last_error_message", "vl_weights_count",
    "vl_model_create", "vl_model_destroy", "vl_model_set_option",
    "vl_encode_workspace_bytes", "vl_encode_images", "vl_score", "vl_model_op_times",
    "vl_mx_quantize", "vl_mx_gemm", "vl_text_weights_count", "vl_text_model_create",
    "vl_text_workspace_bytes", "vl_encode_texts", "vl_contrastive_workspace_bytes",
    "vl_contrastive_loss", "vl_attention_workspace_bytes", "vl_attention",
    "vl_gemm_config_count", "vl_gemm_config_name", "vl_model_get_tuning",
    "vl_model_set_tuning", "vl_model_autotune", "vl_model_save_tuning", "vl_model_load_tuning",
    "vl_contrastive_loss_noalloc", "vl_train_workspace_bytes", "vl_encode_images_train",
    "vl_encode_images_backward", "vl_bf16_round", "vl_fp8_quantize_rows", "vl_model_graph_stats",
    "vl_attention_backward_workspace_bytes", "vl_attention_backward",
)
VL_NOALLOC_SCRATCH_BYTES = 64 << 20
VL_N_GEMM_OPS, VL_N_M_BUCKETS = 5, 25
GEMM_OPS = ("patch_embed", "qkv_gemm", "oproj_gemm", "fc1_gemm", "fc2_gemm")


def library_path() -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvl.so")


class VlError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"vl status {status}: {message}")
        self.status = status


class VlConfig(ctypes.Structure):
    _fields_ = [
        ("patch", ctypes.c_int32), ("width", ctypes.c_int32), ("layers", ctypes.c_int32),
        ("heads", ctypes.c_int32), ("mlp", ctypes.c_int32), ("proj_dim", ctypes.c_int32),
        ("base_grid", ctypes.c_int32), ("ln_eps", ctypes.c_float),
        ("chan_mean", ctypes.c_float * 4), ("chan_std", ctypes.c_float * 4),
        ("channels", ctypes.c_int32), ("pool", ctypes.c_int32),
    ]

    @classmethod
    def from_model(cls, c) -> "VlConfig":
        ch = int(getattr(c, "channels", 3))
        mean = list(c.chan_mean)[:ch] + [0.0] * (4 - ch)
        std = list(c.chan_std)[:ch] + [1.0] * (4 - ch)
        return cls(int(c.patch), int(c.width), int(c.layers), int(c.heads), int(c.mlp),
                   int(c.proj_dim), int(c.base_grid), float(c.ln_eps),
                   (ctypes.c_float * 4)(*mean), (ctypes.c_float * 4)(*std), ch,
                   POOLS[getattr(c, "pool", "cls")])


class VlTextConfig(ctypes.Structure):
    _fields_ = [
        ("vocab", ctypes.c_int32), ("ctx", ctypes.c_int32), ("width", ctypes.c_int32),
        ("layers", ctypes.c_int32), ("heads", ctypes.c_int32), ("mlp", ctypes.c_int32),
        ("proj_dim", ctypes.c_int32), ("ln_eps", ctypes.c_float),
    ]

    @classmethod
    def from_model(cls, c) -> "VlTextConfig":
        return cls(int(c.vocab), int(c.ctx), int(c.width), int(c.layers), int(c.heads),
                   int(c.mlp), int(c.proj_dim), float(c.ln_eps))


_LIB: Optional[ctypes.CDLL] = None
_vp, _i32, _sz, _f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_size_t, ctypes.c_float
_pi32 = ctypes.POINTER(ctypes.c_int32)


def lib() -> ctypes.CDLL:
    """Load libvl.so from the package directory; raise if it is not built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it first "
                           "(python -m paper_2505_00690_amd.build)")
    L = ctypes.CDLL(path)
    L.vl_abi_version.restype = _i32
    L.vl_abi_version.argtypes = []
    L.vl_status_string.restype = ctypes.c_char_p
    L.vl_status_string.argtypes = [ctypes.c_int]
    L.vl_last_error_message.restype = ctypes.c_char_p
    L.vl_last_error_message.argtypes = []
    L.vl_weights_count.restype = _sz
    L.vl_weights_count.argtypes = [ctypes.POINTER(VlConfig)]
    L.vl_model_create.restype = ctypes.c_int
    L.vl_model_create.argtypes = [ctypes.POINTER(VlConfig), ctypes.c_int, _vp, _sz, _vp,
                                  ctypes.POINTER(_vp)]
    L.vl_model_destroy.restype = None
    L.vl_model_destroy.argtypes = [_vp]
    L.vl_model_set_option.restype = ctypes.c_int
    L.vl_model_set_option.argtypes = [_vp, ctypes.c_int, ctypes.c_int64]
    L.vl_encode_workspace_bytes.restype = _sz
    L.vl_encode_workspace_bytes.argtypes = [_vp, _i32, _pi32, _pi32]
    L.vl_encode_images.restype = ctypes.c_int
    L.vl_encode_images.argtypes = [_vp, _vp, _pi32, _pi32, _i32, _vp, _vp, _sz, _vp]
    L.vl_model_op_times.restype = ctypes.c_int
    L.vl_model_op_times.argtypes = [_vp, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
    L.vl_model_graph_stats.restype = ctypes.c_int
    L.vl_model_graph_stats.argtypes = [_vp, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64), _pi32]
    L.vl_gemm_config_count.restype = _i32
    L.vl_gemm_config_count.argtypes = []
    L.vl_gemm_config_name.restype = ctypes.c_char_p
    L.vl_gemm_config_name.argtypes = [_i32]
    L.vl_model_get_tuning.restype = ctypes.c_int
    L.vl_model_get_tuning.argtypes = [_vp, _pi32]
    L.vl_model_set_tuning.restype = ctypes.c_int
    L.vl_model_set_tuning.argtypes = [_vp, _pi32]
    L.vl_model_autotune.restype = ctypes.c_int
    L.vl_model_autotune.argtypes = [_vp, _vp, _pi32, _pi32, _i32, _vp, _vp, _sz, _i32, _vp]
    L.vl_model_save_tuning.restype = ctypes.c_int
    L.vl_model_save_tuning.argtypes = [_vp, ctypes.c_char_p]
    L.vl_model_load_tuning.restype = ctypes.c_int
    L.vl_model_load_tuning.argtypes = [_vp, ctypes.c_char_p]
    L.vl_mx_quantize.restype = ctypes.c_int
    L.vl_mx_quantize.argtypes = [_vp, _i32, _i32, _vp, _vp, _vp]
    L.vl_text_weights_count.restype = _sz
    L.vl_text_weights_count.argtypes = [ctypes.POINTER(VlTextConfig)]
    L.vl_text_model_create.restype = ctypes.c_int
    L.vl_text_model_create.argtypes = [ctypes.POINTER(VlTextConfig), ctypes.c_int, _vp, _sz, _vp,
                                       ctypes.POINTER(_vp)]
    L.vl_text_workspace_bytes.restype = _sz
    L.vl_text_workspace_bytes.argtypes = [_vp, _i32, _pi32]
    L.vl_encode_texts.restype = ctypes.c_int
    L.vl_encode_texts.argtypes = [_vp, _vp, _pi32, _i32, _vp, _vp, _sz, _vp]
    L.vl_contrastive_workspace_bytes.restype = _sz
    L.vl_contrastive_workspace_bytes.argtypes = [_i32, _i32]
    L.vl_contrastive_loss.restype = ctypes.c_int
    L.vl_contrastive_loss.argtypes = [_vp, _vp, _i32, _i32, ctypes.c_int, _f32, _f32, _vp, _vp,
                                      _vp, _vp, _vp, _sz, _vp]
    L.vl_bf16_round.restype = ctypes.c_int
    L.vl_bf16_round.argtypes = [_vp, ctypes.c_int64, _i32, _vp, _vp]
    L.vl_fp8_quantize_rows.restype = ctypes.c_int
    L.vl_fp8_quantize_rows.argtypes = [_vp, _i32, _i32, _vp, _vp, _vp]
    L.vl_train_workspace_bytes.restype = _sz
    L.vl_train_workspace_bytes.argtypes = [_vp, _i32, _pi32, _pi32]
    L.vl_encode_images_train.restype = ctypes.c_int
    L.vl_encode_images_train.argtypes = [_vp, _vp, _pi32, _pi32, _i32, _vp, _vp, _sz, _vp]
    L.vl_encode_images_backward.restype = ctypes.c_int
    L.vl_encode_images_backward.argtypes = [_vp, _vp, _pi32, _pi32, _i32, _vp, _vp, _vp, _sz,
                                            _vp]
    L.vl_contrastive_loss_noalloc.restype = ctypes.c_int
    L.vl_contrastive_loss_noalloc.argtypes = [_vp, _vp, _i32, _i32, ctypes.c_int, _f32, _f32,
                                              _vp, _vp, _vp, _vp, _vp]
    L.vl_attention_workspace_bytes.restype = _sz
    L.vl_attention_workspace_bytes.argtypes = [_i32, _pi32]
    L.vl_attention.restype = ctypes.c_int
    L.vl_attention.argtypes = [_vp, ctypes.c_int, _pi32, _i32, _i32, _i32, _i32, _vp, _vp, _sz,
                               _vp]
    L.vl_attention_backward_workspace_bytes.restype = _sz
    L.vl_attention_backward_workspace_bytes.argtypes = [_i32, _pi32, _i32, _i32]
    L.vl_attention_backward.restype = ctypes.c_int
    L.vl_attention_backward.argtypes = [_vp, _vp, _vp, ctypes.c_int, _pi32, _i32, _i32, _i32,
                                        _vp, _vp, _sz, _vp]
    L.vl_mx_gemm.restype = ctypes.c_int
    L.vl_mx_gemm.argtypes = [_vp, _vp, _vp, _vp, _i32, _i32, _i32, _vp, _vp, _i32, _vp]
    L.vl_score.restype = ctypes.c_int
    L.vl_score.argtypes = [_vp, _i32, _vp, _i32, _i32, ctypes.c_int, _f32, _f32, _vp, _vp, _vp]
    _LIB = L
    return L


def _check(st: int) -> None:
    if st != 0:
        raise VlError(st, lib().vl_last_error_message().decode())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t: Optional[torch.Tensor], dtype=None, name="tensor") -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _i32_array(xs: Sequence[int]):
    return (ctypes.c_int32 * len(xs))(*[int(x) for x in xs])


def vl_abi_version() -> int:
    return int(lib().vl_abi_version())


def vl_status_string(status: int) -> str:
    return lib().vl_status_string(int(status)).decode()


def vl_last_error_message() -> str:
    return lib().vl_last_error_message().decode()


def vl_weights_count(cfg) -> int:
    c = cfg if isinstance(cfg, VlConfig) else VlConfig.from_model(cfg)
    return int(lib().vl_weights_count(ctypes.byref(c)))


def vl_model_create(cfg, precision, weights: torch.Tensor, stream=None) -> ctypes.c_void_p:
    c = cfg if isinstance(cfg, VlConfig) else VlConfig.from_model(cfg)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    handle = ctypes.c_void_p()
    _check(lib().vl_model_create(ctypes.byref(c), prec, _ptr(weights, torch.float32, "weights"),
                                 weights.numel(), _stream(stream), ctypes.byref(handle)))
    return handle


def vl_model_destroy(handle) -> None:
    lib().vl_model_destroy(handle)


def vl_model_set_option(handle, option: int, value: int) -> None:
    _check(lib().vl_model_set_option(handle, int(option), int(value)))


def vl_model_op_times(handle, reset: bool = False):
    """{op name: (total ms, launches)} of the timed launches so far."""
    ms = (ctypes.c_double * VL_N_OPS)()
    n = (ctypes.c_int64 * VL_N_OPS)()
    _check(lib().vl_model_op_times(handle, ms, n, 1 if reset else 0))
    return {OP_NAMES[i]: (float(ms[i]), int(n[i])) for i in range(VL_N_OPS)}


def vl_model_graph_stats(handle) -> dict:
    """Graph cache counters: {"captures", "replays", "cached"}."""
    c, r = ctypes.c_int64(0), ctypes.c_int64(0)
    k = ctypes.c_int32(0)
    _check(lib().vl_model_graph_stats(handle, ctypes.byref(c), ctypes.byref(r), ctypes.byref(k)))
    return {"captures": int(c.value), "replays": int(r.value), "cached": int(k.value)}


def vl_gemm_config_count() -> int:
    return int(lib().vl_gemm_config_count())


def vl_gemm_config_name(cfg: int) -> Optional[str]:
    r = lib().vl_gemm_config_name(int(cfg))
    return r.decode() if r else None


def vl_model_get_tuning(handle):
    """Tuning table as a list of VL_N_GEMM_OPS rows of VL_N_M_BUCKETS ids."""
    t = (ctypes.c_int32 * (VL_N_GEMM_OPS * VL_N_M_BUCKETS))()
    _check(lib().vl_model_get_tuning(handle, t))
    return [list(t[i * VL_N_M_BUCKETS:(i + 1) * VL_N_M_BUCKETS]) for i in range(VL_N_GEMM_OPS)]


def vl_model_set_tuning(handle, table) -> None:
    flat = [int(v) for row in table for v in row]
    if len(flat) != VL_N_GEMM_OPS * VL_N_M_BUCKETS:
        raise ValueError("tuning table has the wrong size")
    _check(lib().vl_model_set_tuning(handle, (ctypes.c_int32 * len(flat))(*flat)))


def vl_model_save_tuning(handle, path: str) -> None:
    _check(lib().vl_model_save_tuning(handle, os.fsencode(path)))


def vl_model_load_tuning(handle, path: str) -> None:
    _check(lib().vl_model_load_tuning(handle, os.fsencode(path)))


def _need(t: torch.Tensor, name: str, shape=None, numel=None, dtype=None) -> None:
    """Host-side size check of a tensor handed to the library, which cannot
    check device buffer sizes itself (an undersized buffer would be read or
    written out of bounds)."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs at least {numel}")


def vl_model_autotune(handle, pixels: torch.Tensor, heights: Sequence[int],
                      widths: Sequence[int], emb_out: torch.Tensor, workspace: torch.Tensor,
                      reps: int = 5, stream=None, channels: int = 3,
                      proj_dim: Optional[int] = None) -> None:
    _check_encode_args(pixels, heights, widths, emb_out, channels, proj_dim)
    _check(lib().vl_model_autotune(handle, _ptr(pixels, torch.float32, "pixels"),
                                   _i32_array(heights), _i32_array(widths), len(heights),
                                   _ptr(emb_out, torch.float32, "emb_out"),
                                   _ptr(workspace, None, "workspace"),
                                   workspace.numel() * workspace.element_size(), int(reps),
                                   _stream(stream)))


def vl_encode_workspace_bytes(handle, heights: Sequence[int], widths: Sequence[int]) -> int:
    return int(lib().vl_encode_workspace_bytes(handle, len(heights), _i32_array(heights),
                                               _i32_array(widths)))


def _check_encode_args(pixels, heights, widths, emb_out, channels, proj_dim) -> None:
    if len(heights) != len(widths):
        raise ValueError("heights and widths differ in length")
    n = len(heights)
    _need(pixels, "pixels", dtype=torch.float32,
          numel=int(channels) * sum(int(h) * int(w) for h, w in zip(heights, widths)))
    _need(emb_out, "emb_out", dtype=torch.float32)
    if emb_out.dim() != 2 or emb_out.shape[0] != n or \
            (proj_dim is not None and emb_out.shape[1] != int(proj_dim)):
        raise ValueError(f"emb_out must be [{n}, {proj_dim if proj_dim else 'proj_dim'}], "
                         f"got {tuple(emb_out.shape)}")


def vl_encode_images(handle, pixels: torch.Tensor, heights: Sequence[int],
                     widths: Sequence[int], emb_out: torch.Tensor, workspace: torch.Tensor,
                     stream=None, channels: int = 3, proj_dim: Optional[int] = None) -> None:
    """channels / proj_dim: the model's, for the host-side size checks of
    pixels (channels * sum(H * W) floats) and emb_out ([n, proj_dim])."""
    _check_encode_args(pixels, heights, widths, emb_out, channels, proj_dim)
    _check(lib().vl_encode_images(handle, _ptr(pixels, torch.float32, "pixels"),
                                  _i32_array(heights), _i32_array(widths), len(heights),
                                  _ptr(emb_out, torch.float32, "emb_out"),
                                  _ptr(workspace, None, "workspace"),
                                  workspace.numel() * workspace.element_size(), _stream(stream)))


def vl_text_weights_count(cfg) -> int:
    c = cfg if isinstance(cfg, VlTextConfig) else VlTextConfig.from_model(cfg)
    return int(lib().vl_text_weights_count(ctypes.byref(c)))


def vl_text_model_create(cfg, precision, weights: torch.Tensor, stream=None) -> ctypes.c_void_p:
    c = cfg if isinstance(cfg, VlTextConfig) else VlTextConfig.from_model(cfg)
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    handle = ctypes.c_void_p()
    _check(lib().vl_text_model_create(ctypes.byref(c), prec,
                                      _ptr(weights, torch.float32, "weights"), weights.numel(),
                                      _stream(stream), ctypes.byref(handle)))
    return handle


def vl_text_workspace_bytes(handle, lengths: Sequence[int]) -> int:
    return int(lib().vl_text_workspace_bytes(handle, len(lengths), _i32_array(lengths)))


def vl_encode_texts(handle, ids: torch.Tensor, lengths: Sequence[int], emb_out: torch.Tensor,
                    workspace: torch.Tensor, stream=None) -> None:
    if ids.numel() != sum(int(x) for x in lengths):
        raise ValueError("ids must hold sum(lengths) tokens")
    if emb_out.dim() != 2 or emb_out.shape[0] != len(lengths):
        raise ValueError(f"emb_out must be [{len(lengths)}, proj_dim], got {tuple(emb_out.shape)}")
    _check(lib().vl_encode_texts(handle, _ptr(ids, torch.int32, "ids"), _i32_array(lengths),
                                 len(lengths), _ptr(emb_out, torch.float32, "emb_out"),
                                 _ptr(workspace, None, "workspace"),
                                 workspace.numel() * workspace.element_size(), _stream(stream)))


def vl_contrastive_workspace_bytes(n: int, dim: int) -> int:
    return int(lib().vl_contrastive_workspace_bytes(n, dim))


def vl_contrastive_loss(emb: torch.Tensor, texts: torch.Tensor, head, scale: float,
                        bias: float = 0.0, stream=None):
    """Loss and gradients of n matched pairs; returns (loss [1], d_emb,
    d_texts, d_scale_bias [2]) as new device tensors."""
    h = HEADS[head] if isinstance(head, str) else int(head)
    n, dim = emb.shape
    if texts.shape != emb.shape:
        raise ValueError("emb and texts must have the same shape")
    dev = emb.device
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    de = torch.empty_like(emb)
    dt = torch.empty_like(texts)
    dsb = torch.empty(2, dtype=torch.float32, device=dev)
    nb = vl_contrastive_workspace_bytes(n, dim)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    _check(lib().vl_contrastive_loss(_ptr(emb, torch.float32, "emb"),
                                     _ptr(texts, torch.float32, "texts"), n, dim, h,
                                     float(scale), float(bias), _ptr(loss), _ptr(de), _ptr(dt),
                                     _ptr(dsb), _ptr(ws), nb, _stream(stream)))
    return loss, de, dt, dsb


def vl_contrastive_loss_noalloc(emb: torch.Tensor, texts: torch.Tensor, head, scale: float,
                                bias: float, loss: torch.Tensor, d_emb: torch.Tensor,
                                d_texts: torch.Tensor, d_scale_bias: torch.Tensor,
                                stream=None) -> None:
    """vl_contrastive_loss into caller-provided outputs, with the library's
    static per-device scratch instead of a workspace (nothing is allocated,
    here or in the library).  Calls in flight together on one GPU race."""
    h = HEADS[head] if isinstance(head, str) else int(head)
    if emb.dim() != 2 or texts.shape != emb.shape:
        raise ValueError("emb and texts must both be [n, dim]")
    n, dim = emb.shape
    for name, t, shape in (("loss", loss, (1,)), ("d_emb", d_emb, (n, dim)),
                           ("d_texts", d_texts, (n, dim)), ("d_scale_bias", d_scale_bias, (2,))):
        if tuple(t.shape) != shape:
            raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
    _check(lib().vl_contrastive_loss_noalloc(
        _ptr(emb, torch.float32, "emb"), _ptr(texts, torch.float32, "texts"), n, dim, h,
        float(scale), float(bias), _ptr(loss, torch.float32, "loss"),
        _ptr(d_emb, torch.float32, "d_emb"), _ptr(d_texts, torch.float32, "d_texts"),
        _ptr(d_scale_bias, torch.float32, "d_scale_bias"), _stream(stream)))


def vl_score(emb: torch.Tensor, texts: torch.Tensor, head, scale: float, bias: float,
             scores_out: torch.Tensor, top1_out: Optional[torch.Tensor] = None,
             stream=None) -> None:
    h = HEADS[head] if isinstance(head, str) else int(head)
    if emb.dim() != 2 or texts.dim() != 2:
        raise ValueError("emb and texts must be 2-D")
    n, dim = emb.shape
    m = texts.shape[0]
    if texts.shape[1] != dim:
        raise ValueError("emb and texts differ in width")
    _need(scores_out, "scores_out", shape=(n, m), dtype=torch.float32)
    if top1_out is not None:
        _need(top1_out, "top1_out", shape=(n,), dtype=torch.int32)
    _check(lib().vl_score(_ptr(emb, torch.float32, "emb"), n, _ptr(texts, torch.float32, "texts"),
                          m, dim, h, float(scale), float(bias),
                          _ptr(scores_out, torch.float32, "scores_out"),
                          _ptr(top1_out, torch.int32, "top1_out"), _stream(stream)))


def vl_attention_workspace_bytes(lengths: Sequence[int]) -> int:
    return int(lib().vl_attention_workspace_bytes(len(lengths), _i32_array(lengths)))


def vl_attention(qkv: torch.Tensor, lengths: Sequence[int], heads: int, head_dim: int,
                 causal: bool, out: torch.Tensor, workspace: Optional[torch.Tensor] = None,
                 stream=None) -> None:
    """Multi-head attention of packed sequences: qkv [T, 3 * heads * head_dim]
    (BF16 or FP32) -> out [T, heads * head_dim] of the same dtype."""
    T = sum(int(x) for x in lengths)
    D = int(heads) * int(head_dim)
    if qkv.dtype not in (torch.bfloat16, torch.float32):
        raise ValueError("qkv must be bfloat16 or float32")
    if tuple(qkv.shape) != (T, 3 * D):
        raise ValueError(f"qkv must be [{T}, {3 * D}], got {tuple(qkv.shape)}")
    if tuple(out.shape) != (T, D) or out.dtype != qkv.dtype:
        raise ValueError(f"out must be [{T}, {D}] {qkv.dtype}")
    prec = VL_BF16 if qkv.dtype == torch.bfloat16 else VL_FP32
    nb = vl_attention_workspace_bytes(lengths)
    if nb == 0:
        raise VlError(1, "invalid sequence lengths")
    if workspace is None:
        workspace = torch.empty(nb, dtype=torch.uint8, device=qkv.device)
    elif workspace.numel() * workspace.element_size() < nb:
        raise ValueError("workspace too small")
    _check(lib().vl_attention(_ptr(qkv, None, "qkv"), prec, _i32_array(lengths), len(lengths),
                              int(heads), int(head_dim), 1 if causal else 0, _ptr(out, None, "out"),
                              _ptr(workspace, None, "workspace"),
                              workspace.numel() * workspace.element_size(), _stream(stream)))


def vl_attention_backward_workspace_bytes(lengths: Sequence[int], heads: int,
                                          head_dim: int) -> int:
    return int(lib().vl_attention_backward_workspace_bytes(len(lengths), _i32_array(lengths),
                                                           int(heads), int(head_dim)))


def vl_attention_backward(qkv: torch.Tensor, out: torch.Tensor, d_out: torch.Tensor,
                          lengths: Sequence[int], heads: int, head_dim: int,
                          d_qkv: torch.Tensor, workspace: Optional[torch.Tensor] = None,
                          stream=None) -> None:
    """Backward of unmasked vl_attention: qkv [T, 3D] and its output out [T, D]
    (BF16 or FP32), d_out [T, D] FP32 -> d_qkv [T, 3D] of qkv's dtype."""
    T = sum(int(x) for x in lengths)
    D = int(heads) * int(head_dim)
    if qkv.dtype not in (torch.bfloat16, torch.float32):
        raise ValueError("qkv must be bfloat16 or float32")
    if tuple(qkv.shape) != (T, 3 * D):
        raise ValueError(f"qkv must be [{T}, {3 * D}], got {tuple(qkv.shape)}")
    if tuple(out.shape) != (T, D) or out.dtype != qkv.dtype:
        raise ValueError(f"out must be [{T}, {D}] {qkv.dtype}")
    if tuple(d_out.shape) != (T, D) or d_out.dtype != torch.float32:
        raise ValueError(f"d_out must be [{T}, {D}] float32")
    if tuple(d_qkv.shape) != (T, 3 * D) or d_qkv.dtype != qkv.dtype:
        raise ValueError(f"d_qkv must be [{T}, {3 * D}] {qkv.dtype}")
    prec = VL_BF16 if qkv.dtype == torch.bfloat16 else VL_FP32
    nb = vl_attention_backward_workspace_bytes(lengths, heads, head_dim)
    if nb == 0:
        raise VlError(1, "invalid sequence lengths, heads or head_dim")
    if workspace is None:
        workspace = torch.empty(nb, dtype=torch.uint8, device=qkv.device)
    elif workspace.numel() * workspace.element_size() < nb:
        raise ValueError("workspace too small")
    _check(lib().vl_attention_backward(
        _ptr(qkv, None, "qkv"), _ptr(out, None, "out"), _ptr(d_out, torch.float32, "d_out"), prec,
        _i32_array(lengths), len(lengths), int(heads), int(head_dim), _ptr(d_qkv, None, "d_qkv"),
        _ptr(workspace, None, "workspace"), workspace.numel() * workspace.element_size(),
        _stream(stream)))


def vl_mx_quantize(src: torch.Tensor, codes_out: torch.Tensor, scales_out: torch.Tensor,
                   stream=None) -> None:
    """MXFP8 encoding of FP32 rows src [rows, cols] into codes_out (uint8
    [rows, cols]) and scales_out (uint8, (cols/128) * rows * 4 bytes,
    block-major as include/vl.h describes)."""
    rows, cols = src.shape
    if codes_out.shape != src.shape or scales_out.numel() != (cols // 128) * rows * 4:
        raise ValueError("codes_out / scales_out have the wrong size")
    _check(lib().vl_mx_quantize(_ptr(src, torch.float32, "src"), rows, cols,
                                _ptr(codes_out, torch.uint8, "codes_out"),
                                _ptr(scales_out, torch.uint8, "scales_out"), _stream(stream)))


def vl_mx_gemm(a: torch.Tensor, sa: torch.Tensor, b: torch.Tensor, sb: torch.Tensor,
               bias: torch.Tensor, c: torch.Tensor, cfg: int = -1, stream=None) -> None:
    """c += A . B^T + bias for MXFP8 operands (codes a [M, K], b [N, K] and
    their scale arrays as vl_mx_quantize writes them)."""
    M, K = a.shape
    N = b.shape[0]
    if b.shape[1] != K or c.shape != (M, N) or bias.shape != (N,):
        raise ValueError("shape mismatch")
    if sa.numel() != K // 128 * M * 4 or sb.numel() != K // 128 * N * 4:
        raise ValueError("scale arrays have the wrong size")
    _check(lib().vl_mx_gemm(_ptr(a, torch.uint8, "a"), _ptr(sa, torch.uint8, "sa"),
                            _ptr(b, torch.uint8, "b"), _ptr(sb, torch.uint8, "sb"), M, N, K,
                            _ptr(bias, torch.float32, "bias"), _ptr(c, torch.float32, "c"),
                            int(cfg), _stream(stream)))


def vl_bf16_round(src: torch.Tensor, dst: torch.Tensor, method: int = 0, stream=None) -> None:
    """FP32 -> BF16 bit patterns (int16 / uint16 tensor of src's size)."""
    if src.numel() != dst.numel() or dst.element_size() != 2:
        raise ValueError("dst must hold src.numel() 16-bit values")
    _check(lib().vl_bf16_round(_ptr(src, torch.float32, "src"), src.numel(), int(method),
                               _ptr(dst, None, "dst"), _stream(stream)))


def vl_fp8_quantize_rows(src: torch.Tensor, codes: torch.Tensor, scales: torch.Tensor,
                         stream=None) -> None:
    rows, cols = src.shape
    _need(codes, "codes", shape=(rows, cols), dtype=torch.uint8)
    _need(scales, "scales", shape=(rows,), dtype=torch.float32)
    _check(lib().vl_fp8_quantize_rows(_ptr(src, torch.float32, "src"), rows, cols,
                                      _ptr(codes), _ptr(scales), _stream(stream)))


def vl_train_workspace_bytes(handle, heights: Sequence[int], widths: Sequence[int]) -> int:
    return int(lib().vl_train_workspace_bytes(handle, len(heights), _i32_array(heights),
                                              _i32_array(widths)))


def vl_encode_images_train(handle, pixels: torch.Tensor, heights: Sequence[int],
                           widths: Sequence[int], emb_out: torch.Tensor, workspace: torch.Tensor,
                           stream=None, channels: int = 3, proj_dim=None) -> None:
    _check_encode_args(pixels, heights, widths, emb_out, channels, proj_dim)
    _check(lib().vl_encode_images_train(handle, _ptr(pixels, torch.float32, "pixels"),
                                        _i32_array(heights), _i32_array(widths), len(heights),
                                        _ptr(emb_out, torch.float32, "emb_out"),
                                        _ptr(workspace, None, "workspace"),
                                        workspace.numel() * workspace.element_size(),
                                        _stream(stream)))


def vl_encode_images_backward(handle, pixels: torch.Tensor, heights: Sequence[int],
                              widths: Sequence[int], d_emb: torch.Tensor, grads_out: torch.Tensor,
                              workspace: torch.Tensor, n_weights: int, stream=None,
                              channels: int = 3, proj_dim=None) -> None:
    _check_encode_args(pixels, heights, widths, d_emb, channels, proj_dim)
    _need(grads_out, "grads_out", dtype=torch.float32, numel=int(n_weights))
    _check(lib().vl_encode_images_backward(handle, _ptr(pixels, torch.float32, "pixels"),
                                           _i32_array(heights), _i32_array(widths), len(heights),
                                           _ptr(d_emb, torch.float32, "d_emb"),
                                           _ptr(grads_out, torch.float32, "grads_out"),
                                           _ptr(workspace, None, "workspace"),
                                           workspace.numel() * workspace.element_size(),
                                           _stream(stream)))


class Encoder:
    """Owns a model handle built from an FP32 weight blob on the device, plus
    a reusable workspace tensor."""

    def __init__(self, cfg, weights: torch.Tensor, precision: str = "bf16",
                 graphs: bool = False, stream=None, split: bool = False,
                 fused_ln: bool = False):
        self.cfg = cfg
        self.precision = precision
        self.handle = vl_model_create(cfg, precision, weights, stream)
        if graphs:
            vl_model_set_option(self.handle, VL_OPT_GRAPHS, 1)
        if split:
            vl_model_set_option(self.handle, VL_OPT_SPLIT, 1)
        if fused_ln:
            vl_model_set_option(self.handle, VL_OPT_FUSED_LN, 1)
        self._ws: Optional[torch.Tensor] = None
        self.device = weights.device
        self._channels = int(getattr(cfg, "channels", 3))

    def close(self) -> None:
        if self.handle is not None and self.handle.value:
            vl_model_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, sizes: Sequence[Tuple[int, int]]) -> int:
        return vl_encode_workspace_bytes(self.handle, [h for h, _ in sizes], [w for _, w in sizes])

    def workspace(self, nbytes: int) -> torch.Tensor:
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._ws

    def autotune(self, pixels: torch.Tensor, sizes: Sequence[Tuple[int, int]],
                 reps: int = 5, cache: Optional[str] = None) -> dict:
        """Time every GEMM tile configuration on this batch shape and keep
        the fastest; returns {op: {bucket: config name}} of the table.  With
        `cache` (a JSON path), a table saved there for this device, precision
        and model shape is loaded instead of tuning, and a new one is saved."""
        n = len(sizes)
        out = torch.empty((n, self.cfg.proj_dim), dtype=torch.float32, device=self.device)
        ws = self.workspace(self.workspace_bytes(sizes))
        if cache and os.path.exists(cache):
            try:
                vl_model_load_tuning(self.handle, cache)
                return self.tuning()
            except VlError:
                pass                          # tuned elsewhere: tune again and rewrite
        vl_model_autotune(self.handle, pixels, [h for h, _ in sizes], [w for _, w in sizes],
                          out, ws, reps, channels=self._channels, proj_dim=self.cfg.proj_dim)
        if cache:
            vl_model_save_tuning(self.handle, cache)
        return self.tuning()

    def graph_stats(self) -> dict:
        return vl_model_graph_stats(self.handle)

    def tuning(self) -> dict:
        t = vl_model_get_tuning(self.handle)
        return {GEMM_OPS[i]: {str(b): vl_gemm_config_name(c) for b, c in enumerate(row) if c >= 0}
                for i, row in enumerate(t)}

    def set_tuning(self, named: dict) -> None:
        """Inverse of tuning(): {op: {bucket: config name}}."""
        ids = {vl_gemm_config_name(i): i for i in range(vl_gemm_config_count())}
        table = [[-1] * VL_N_M_BUCKETS for _ in range(VL_N_GEMM_OPS)]
        for op, row in named.items():
            for b, name in row.items():
                table[GEMM_OPS.index(op)][int(b)] = ids[name]
        vl_model_set_tuning(self.handle, table)

    def encode(self, pixels: torch.Tensor, sizes: Sequence[Tuple[int, int]],
               out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """pixels: flat FP32 device tensor holding the [C,H,W] images back to
        back; sizes: their (H, W).  Returns [n, proj_dim] unit embeddings."""
        n = len(sizes)
        if out is None:
            out = torch.empty((n, self.cfg.proj_dim), dtype=torch.float32, device=self.device)
        need = self.workspace_bytes(sizes)
        if need == 0:
            raise VlError(1, "invalid batch shapes")
        ws = self.workspace(need)
        vl_encode_images(self.handle, pixels, [h for h, _ in sizes], [w for _, w in sizes], out,
                         ws, stream, channels=self._channels, proj_dim=self.cfg.proj_dim)
        return out


class TextEncoder:
    """Owns a text-model handle built from an FP32 weight blob on the device,
    plus a reusable workspace tensor."""

    def __init__(self, cfg, weights: torch.Tensor, precision: str = "bf16",
                 graphs: bool = False, stream=None):
        self.cfg = cfg
        self.precision = precision
        self.handle = vl_text_model_create(cfg, precision, weights, stream)
        if graphs:
            vl_model_set_option(self.handle, VL_OPT_GRAPHS, 1)
        self._ws: Optional[torch.Tensor] = None
        self.device = weights.device

    def close(self) -> None:
        if self.handle is not None and self.handle.value:
            vl_model_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def encode(self, ids: torch.Tensor, lengths: Sequence[int],
               out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """ids: int32 device tensor of all sequences' token ids back to back;
        lengths: tokens per sequence.  Returns [n, proj_dim] unit embeddings."""
        n = len(lengths)
        if out is None:
            out = torch.empty((n, self.cfg.proj_dim), dtype=torch.float32, device=self.device)
        need = vl_text_workspace_bytes(self.handle, lengths)
        if need == 0:
            raise VlError(1, "invalid text lengths")
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        vl_encode_texts(self.handle, ids, lengths, out, self._ws, stream)
        return out


class Trainer(Encoder):
    """An Encoder that also runs the training forward and the backward pass
    (FP32 or BF16 models, class-token pooling, images at the base grid)."""

    def train_workspace_bytes(self, sizes: Sequence[Tuple[int, int]]) -> int:
        return vl_train_workspace_bytes(self.handle, [h for h, _ in sizes],
                                        [w for _, w in sizes])

    def forward(self, pixels: torch.Tensor, sizes: Sequence[Tuple[int, int]],
                out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        n = len(sizes)
        if out is None:
            out = torch.empty((n, self.cfg.proj_dim), dtype=torch.float32, device=self.device)
        need = self.train_workspace_bytes(sizes)
        if need == 0:
            raise VlError(1, "batch not supported for training")
        ws = self.workspace(need)
        vl_encode_images_train(self.handle, pixels, [h for h, _ in sizes], [w for _, w in sizes],
                               out, ws, stream, channels=self._channels,
                               proj_dim=self.cfg.proj_dim)
        return out

    def backward(self, pixels: torch.Tensor, sizes: Sequence[Tuple[int, int]],
                 d_emb: torch.Tensor, grads_out: Optional[torch.Tensor] = None,
                 stream=None) -> torch.Tensor:
        nw = vl_weights_count(self.cfg)
        if grads_out is None:
            grads_out = torch.empty(nw, dtype=torch.float32, device=self.device)
        ws = self.workspace(self.train_workspace_bytes(sizes))
        vl_encode_images_backward(self.handle, pixels, [h for h, _ in sizes],
                                  [w for _, w in sizes], d_emb, grads_out, ws, nw, stream,
                                  channels=self._channels, proj_dim=self.cfg.proj_dim)
        return grads_out
