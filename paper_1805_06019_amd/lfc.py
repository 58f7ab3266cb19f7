"""Python binding of liblfc.so (C ABI in include/lfc.h).

Argument marshalling only: every decode and render step runs in the HIP
kernels of the library.  Device buffers are torch CUDA tensors passed by
pointer, work goes on torch's current stream.  The functions raise
``LFCError`` on a non-OK status and raise at load time if the library has
not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblfc.so")
MAX_LEVELS = 6
NOALLOC_SCRATCH_BYTES = 32 << 20   # LFC_NOALLOC_SCRATCH_BYTES
LAYOUT_BLOCKS = 0
LAYOUT_IMAGES = 1

STATUS = {0: "LFC_OK", -1: "LFC_E_INVALID", -2: "LFC_E_CORRUPT", -3: "LFC_E_NOMEM", -4: "LFC_E_HIP",
          -5: "LFC_E_RANGE", -6: "LFC_E_UNSUPPORTED"}


class LFCError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class c_params(C.Structure):
    _fields_ = [
        ("grid_u", C.c_int32), ("grid_v", C.c_int32),
        ("width", C.c_int32), ("height", C.c_int32),
        ("block", C.c_int32), ("levels", C.c_int32),
        ("cluster", C.c_int32 * MAX_LEVELS),
        ("pix_threshold", C.c_int32), ("blk_threshold", C.c_int32),
        ("quant_bits", C.c_int32), ("range_mask", C.c_uint32),
    ]


class c_info(C.Structure):
    _fields_ = [
        ("params", c_params),
        ("padded_width", C.c_int32), ("padded_height", C.c_int32),
        ("n_blocks", C.c_int32), ("n_groups", C.c_int32),
        ("n_srv", C.c_int32), ("n_top", C.c_int32),
        ("stream_bytes", C.c_uint64), ("device_bytes", C.c_uint64),
        ("present_blocks", C.c_uint64),
    ]


class c_stats(C.Structure):
    _fields_ = [
        ("psnr", C.c_double), ("psnr_y", C.c_double), ("psnr_co", C.c_double), ("psnr_cg", C.c_double),
        ("present_blocks", C.c_uint64), ("code_hist", C.c_uint64 * 26), ("stream_bytes", C.c_uint64),
    ]


class c_view(C.Structure):
    _fields_ = [("u", C.c_float), ("v", C.c_float), ("s", C.c_float), ("t", C.c_float)]


class c_render_request(C.Structure):
    _fields_ = [("lf", C.c_int32), ("out_w", C.c_int32), ("out_h", C.c_int32), ("view", c_view)]


class c_control(C.Structure):
    _fields_ = [("mode", C.c_int32), ("min_confidence", C.c_float), ("lambda_q16", C.c_int64),
                ("d_mlp", C.c_void_p), ("stream", C.c_void_p), ("rows", C.c_int64),
                ("classes", C.c_void_p), ("ranges", C.c_void_p), ("features", C.c_void_p),
                ("search_classes", C.c_void_p), ("search_ranges", C.c_void_p), ("fallbacks", C.c_int64)]


CTL_GLOBAL, CTL_SEARCH, CTL_TABLE, CTL_MLP = 0, 1, 2, 3
CTL_CLASSES, CTL_DROP, CTL_RANGES, CTL_ABSENT, CTL_FEATURES = 10, 9, 27, 26, 16
MLP_PARAMS = 7653


class c_render_config(C.Structure):
    _fields_ = [("path", C.c_int32), ("tile_w", C.c_int32), ("tile_h", C.c_int32), ("disparity", C.c_float)]


TUNE_MAX = 16


class c_render_tuning(C.Structure):
    _fields_ = [("n_tried", C.c_int32), ("best", C.c_int32), ("cfg", c_render_config * TUNE_MAX),
                ("ms", C.c_float * TUNE_MAX)]


RENDER_AUTO, RENDER_TILES, RENDER_DECODED = 0, 1, 2


class c_decode_tuning(C.Structure):
    _fields_ = [("n_tried", C.c_int32), ("best", C.c_int32), ("tile_blocks", C.c_int32 * 16),
                ("staged", C.c_int32 * 16), ("ms", C.c_float * 16)]


class c_open_config(C.Structure):
    _fields_ = [("tile_blocks", C.c_int32)]


class c_decode_config(C.Structure):
    _fields_ = [("stage_cap_words", C.c_int64)]


class c_server_config(C.Structure):
    _fields_ = [("max_batch", C.c_int32), ("streams", C.c_int32), ("out_pool_bytes", C.c_int64),
                ("max_queue", C.c_int64), ("device_bytes_cap", C.c_int64)]


class c_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("max_batch_seen", C.c_int64), ("admission_waits", C.c_int64), ("pool_bytes_in_use", C.c_int64)]


@dataclass
class Params:
    """Encoding parameters; see lfc_params in include/lfc.h."""
    grid_u: int
    grid_v: int
    width: int
    height: int
    block: int = 4
    levels: int = 2
    cluster: tuple = (2,)
    pix_threshold: int = 0
    blk_threshold: int = 0
    quant_bits: int = 0
    range_mask: int = 0

    def to_c(self) -> c_params:
        p = c_params()
        p.grid_u, p.grid_v, p.width, p.height = self.grid_u, self.grid_v, self.width, self.height
        p.block, p.levels = self.block, self.levels
        for i in range(MAX_LEVELS):
            p.cluster[i] = self.cluster[i] if i < len(self.cluster) else 0
        p.pix_threshold, p.blk_threshold = self.pix_threshold, self.blk_threshold
        p.quant_bits, p.range_mask = self.quant_bits, self.range_mask
        return p

    @staticmethod
    def from_c(p: c_params) -> "Params":
        return Params(p.grid_u, p.grid_v, p.width, p.height, p.block, p.levels,
                      tuple(p.cluster[i] for i in range(max(p.levels - 1, 0))), p.pix_threshold,
                      p.blk_threshold, p.quant_bits, p.range_mask)


_lib = None


def load() -> C.CDLL:
    """Loads liblfc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        L.lfc_encode.argtypes = [vp, C.POINTER(c_params), C.POINTER(vp), C.POINTER(sz)]
        L.lfc_encode_ex.argtypes = [vp, C.POINTER(c_params), C.POINTER(vp), C.POINTER(sz), C.POINTER(c_stats)]
        L.lfc_free.argtypes = [vp]
        L.lfc_free.restype = None
        L.lfc_validate.argtypes = [vp, sz, C.POINTER(c_params)]
        L.lfc_open.argtypes = [vp, sz, vp, C.POINTER(vp)]
        L.lfc_open_ex.argtypes = [vp, sz, C.POINTER(c_open_config), vp, C.POINTER(vp)]
        L.lfc_decode_blocks_ex.argtypes = [vp, vp, i64, i32, vp, C.POINTER(c_decode_config), vp]
        L.lfc_info.argtypes = [vp, C.POINTER(c_info)]
        L.lfc_decode_blocks.argtypes = [vp, vp, i64, i32, vp, vp]
        L.lfc_decode_progressive.argtypes = [vp, vp, i64, i32, vp, vp]
        L.lfc_decode_rgb.argtypes = [vp, vp, vp]
        L.lfc_stage_needs.argtypes = [vp, vp, i64]
        L.lfc_stage_needs.restype = i64
        L.lfc_render_views.argtypes = [vp, vp, i32, i32, i32, vp, vp]
        L.lfc_tune_decode.argtypes = [vp, vp, i32, C.POINTER(c_decode_tuning), vp]
        L.lfc_tune_decode_rgb.argtypes = [vp, vp, i32, C.POINTER(c_decode_tuning), vp]
        L.lfc_encode_gpu.argtypes = [vp, C.POINTER(c_params), C.POINTER(vp), C.POINTER(sz), C.POINTER(c_stats), vp]
        L.lfc_control_rows.argtypes = [C.POINTER(c_params)]
        L.lfc_control_rows.restype = i64
        L.lfc_encode_ctl.argtypes = [vp, C.POINTER(c_params), C.POINTER(c_control), C.POINTER(vp), C.POINTER(sz),
                                     C.POINTER(c_stats)]
        L.lfc_mlp_infer.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
        L.lfc_mlp_infer_ex.argtypes = [vp, vp, i64, vp, vp, vp, vp, i32, vp]
        L.lfc_mlp_grad.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp]
        L.lfc_mlp_adam.argtypes = [vp, vp, vp, vp, vp, i32, C.c_float, C.c_float, C.c_float, C.c_float, vp]
        L.lfc_render_views_ex.argtypes = [vp, vp, i32, i32, i32, vp, C.POINTER(c_render_config), vp]
        L.lfc_render_views_noalloc.argtypes = [vp, vp, i32, i32, i32, vp, C.POINTER(c_render_config), vp]
        L.lfc_render_tune.argtypes = [vp, vp, i32, i32, i32, vp, i32, C.POINTER(c_render_tuning), vp]
        L.lfc_render_plan_create.argtypes = [vp, C.POINTER(c_render_config), vp, i32, i32, i32, vp, i32,
                                             C.POINTER(vp)]
        L.lfc_render_plan_launch.argtypes = [vp, vp]
        L.lfc_render_plan_info.argtypes = [vp, C.POINTER(c_render_config), C.POINTER(i32)]
        L.lfc_render_plan_destroy.argtypes = [vp]
        L.lfc_render_plan_destroy.restype = None
        L.lfc_check.argtypes = [vp, vp]
        L.lfc_close.argtypes = [vp]
        L.lfc_last_error.argtypes = []
        L.lfc_last_error.restype = C.c_char_p
        u64p, dp = C.POINTER(C.c_uint64), C.POINTER(C.c_double)
        L.lfc_batch_create.argtypes = [C.POINTER(vp)]
        L.lfc_batch_render.argtypes = [vp, C.POINTER(vp), i32, C.POINTER(c_render_request), i32, C.POINTER(vp), vp]
        L.lfc_batch_destroy.argtypes = [vp]
        L.lfc_batch_decode.argtypes = [vp, C.POINTER(vp), i32, vp, i64, vp, vp]
        L.lfc_batch_check.argtypes = [vp, vp]
        L.lfc_batch_plan_create.argtypes = [C.POINTER(vp), i32, C.POINTER(c_render_request), i32, C.POINTER(vp), i32,
                                            C.POINTER(vp)]
        L.lfc_batch_plan_launch.argtypes = [vp, vp]
        L.lfc_batch_plan_info.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.lfc_batch_plan_destroy.argtypes = [vp]
        L.lfc_batch_plan_destroy.restype = None
        L.lfc_server_create.argtypes = [C.POINTER(vp), i32, C.POINTER(c_server_config), C.POINTER(vp)]
        L.lfc_server_submit.argtypes = [vp, C.POINTER(c_render_request), u64p]
        L.lfc_server_wait.argtypes = [vp, C.c_uint64, i32, C.POINTER(vp), dp]
        L.lfc_server_release.argtypes = [vp, C.c_uint64]
        L.lfc_server_replay.argtypes = [vp, C.POINTER(c_render_request), dp, i32, dp]
        L.lfc_server_get_stats.argtypes = [vp, C.POINTER(c_server_stats)]
        L.lfc_server_destroy.argtypes = [vp]
        for f in ("lfc_encode", "lfc_encode_ex", "lfc_validate", "lfc_open", "lfc_open_ex", "lfc_info",
                  "lfc_decode_blocks", "lfc_decode_blocks_ex",
                  "lfc_render_views", "lfc_render_views_ex", "lfc_render_views_noalloc", "lfc_encode_ctl", "lfc_tune_decode", "lfc_tune_decode_rgb", "lfc_encode_gpu", "lfc_mlp_infer", "lfc_mlp_infer_ex", "lfc_mlp_grad",
                  "lfc_mlp_adam", "lfc_render_tune", "lfc_render_plan_create",
                  "lfc_render_plan_launch", "lfc_render_plan_info", "lfc_check", "lfc_close", "lfc_decode_progressive", "lfc_decode_rgb", "lfc_batch_create",
                  "lfc_batch_decode", "lfc_batch_check", "lfc_batch_render", "lfc_batch_plan_create",
                  "lfc_batch_plan_launch", "lfc_batch_plan_info",
                  "lfc_batch_destroy", "lfc_server_create", "lfc_server_submit", "lfc_server_wait",
                  "lfc_server_release", "lfc_server_replay", "lfc_server_get_stats", "lfc_server_destroy"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(st: int) -> None:
    if st != 0:
        raise LFCError(st, load().lfc_last_error().decode(errors="replace"))


def _stream_ptr(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def lfc_encode(rgb: np.ndarray, params: Params) -> bytes:
    """CompressLFI on the host: rgb uint8 [grid_v][grid_u][height][width][3]."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    if rgb.shape != (params.grid_v, params.grid_u, params.height, params.width, 3):
        raise ValueError(f"rgb shape {rgb.shape} does not match the parameters")
    out, n = C.c_void_p(), C.c_size_t()
    _check(load().lfc_encode(rgb.ctypes.data, C.byref(params.to_c()), C.byref(out), C.byref(n)))
    try:
        return C.string_at(out.value, n.value)
    finally:
        load().lfc_free(out)


def lfc_encode_ex(rgb: np.ndarray, params: Params, want_stream: bool = True):
    """lfc_encode plus the encoder's quality/rate statistics (eqs. 4-5).
    Returns (stream or None, stats dict)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    if rgb.shape != (params.grid_v, params.grid_u, params.height, params.width, 3):
        raise ValueError(f"rgb shape {rgb.shape} does not match the parameters")
    st = c_stats()
    out, n = C.c_void_p(), C.c_size_t()
    if want_stream:
        _check(load().lfc_encode_ex(rgb.ctypes.data, C.byref(params.to_c()), C.byref(out), C.byref(n),
                                    C.byref(st)))
    else:
        _check(load().lfc_encode_ex(rgb.ctypes.data, C.byref(params.to_c()), None, None, C.byref(st)))
    data = None
    if want_stream:
        try:
            data = C.string_at(out.value, n.value)
        finally:
            load().lfc_free(out)
    stats = dict(psnr=st.psnr, psnr_y=st.psnr_y, psnr_co=st.psnr_co, psnr_cg=st.psnr_cg,
                 present_blocks=st.present_blocks, code_hist=list(st.code_hist), stream_bytes=st.stream_bytes)
    return data, stats


def lfc_control_rows(params: Params) -> int:
    n = load().lfc_control_rows(C.byref(params.to_c()))
    if n < 0:
        raise LFCError(-1, "invalid parameters")
    return n


def lfc_encode_ctl(rgb: np.ndarray, params: Params, mode: int, lambda_q16: int = 0, classes=None, ranges=None,
                   mlp=None, min_confidence: float = 0.0, want_features: bool = False, want_search: bool = False,
                   want_stream: bool = True, cuda_stream=None):
    """Encoder under per-block control (include/lfc.h).  mlp: CUDA tensor of
    LFC_MLP_PARAMS bfloat16 bits (int16/uint16) for CTL_MLP.  Returns (stream
    or None, stats dict with the classes and ranges used, and the features,
    search classes and ranges when asked for, and the fallback count)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    if rgb.shape != (params.grid_v, params.grid_u, params.height, params.width, 3):
        raise ValueError(f"rgb shape {rgb.shape} does not match the parameters")
    ctl = c_control()
    ctl.mode, ctl.lambda_q16, ctl.min_confidence = mode, int(lambda_q16), float(min_confidence)
    keep = {}
    if mode != CTL_GLOBAL:
        rows = lfc_control_rows(params)
        ctl.rows = rows
        if mode == CTL_TABLE:
            keep["classes"] = np.ascontiguousarray(classes, dtype=np.int8)
            keep["ranges"] = np.ascontiguousarray(ranges, dtype=np.int8)
            if keep["classes"].size != rows or keep["ranges"].size != rows:
                raise ValueError("classes and ranges need one entry per control row")
        else:
            keep["classes"] = np.full(rows, -1, dtype=np.int8)
            keep["ranges"] = np.full(rows, -1, dtype=np.int8)
        ctl.classes, ctl.ranges = keep["classes"].ctypes.data, keep["ranges"].ctypes.data
        if want_features:
            keep["features"] = np.zeros((rows, CTL_FEATURES), dtype=np.float32)
            ctl.features = keep["features"].ctypes.data
        if want_search:
            keep["search_classes"] = np.full(rows, -1, dtype=np.int8)
            keep["search_ranges"] = np.full(rows, -1, dtype=np.int8)
            ctl.search_classes = keep["search_classes"].ctypes.data
            ctl.search_ranges = keep["search_ranges"].ctypes.data
    if mode == CTL_MLP and mlp is not None:
        ctl.d_mlp = mlp.data_ptr()
        ctl.stream = _stream_ptr(cuda_stream)
    st = c_stats()
    out, n = C.c_void_p(), C.c_size_t()
    if want_stream:
        _check(load().lfc_encode_ctl(rgb.ctypes.data, C.byref(params.to_c()), C.byref(ctl), C.byref(out),
                                     C.byref(n), C.byref(st)))
    else:
        _check(load().lfc_encode_ctl(rgb.ctypes.data, C.byref(params.to_c()), C.byref(ctl), None, None,
                                     C.byref(st)))
    data = None
    if want_stream:
        try:
            data = C.string_at(out.value, n.value)
        finally:
            load().lfc_free(out)
    stats = dict(psnr=st.psnr, psnr_y=st.psnr_y, psnr_co=st.psnr_co, psnr_cg=st.psnr_cg,
                 present_blocks=st.present_blocks, code_hist=list(st.code_hist), stream_bytes=st.stream_bytes,
                 fallbacks=ctl.fallbacks, **keep)
    return data, stats


MLP_FP32, MLP_BF16 = 0, 1


def mlp_infer(w, x, logits: bool = False, cuda_stream=None, precision: int = MLP_FP32):
    """Network inference on the GPU: w bf16 bits (CUDA int16/uint16
    [LFC_MLP_PARAMS]), x float32 CUDA [n][16].  Returns (threshold class,
    range class, confidence[, logits]) CUDA tensors."""
    import torch
    n = x.shape[0]
    cls = torch.empty(n, dtype=torch.int8, device="cuda")
    rng = torch.empty(n, dtype=torch.int8, device="cuda")
    conf = torch.empty(n, dtype=torch.float32, device="cuda")
    z = torch.empty((n, 37), dtype=torch.float32, device="cuda") if logits else None
    _check(load().lfc_mlp_infer_ex(w.data_ptr(), x.data_ptr(), n, cls.data_ptr(), rng.data_ptr(), conf.data_ptr(),
                                   z.data_ptr() if z is not None else None, precision, _stream_ptr(cuda_stream)))
    return (cls, rng, conf, z) if logits else (cls, rng, conf)


def mlp_grad(w, x, cls, rng, part=None, cuda_stream=None):
    """Mean loss and gradient over a batch (CUDA tensors); returns (grad
    float32 [LFC_MLP_PARAMS], loss float32 [1])."""
    import torch
    n = x.shape[0]
    nwg = (n + 127) // 128
    if part is None or part.numel() < nwg * (MLP_PARAMS + 1):
        part = torch.empty(nwg * (MLP_PARAMS + 1), dtype=torch.float32, device="cuda")
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(load().lfc_mlp_grad(w.data_ptr(), x.data_ptr(), cls.data_ptr(), rng.data_ptr(), n, part.data_ptr(),
                               grad.data_ptr(), loss.data_ptr(), _stream_ptr(cuda_stream)))
    return grad, loss


def mlp_adam(master, w, m, v, grad, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, cuda_stream=None):
    _check(load().lfc_mlp_adam(master.data_ptr(), w.data_ptr(), m.data_ptr(), v.data_ptr(), grad.data_ptr(), step,
                               lr, beta1, beta2, eps, _stream_ptr(cuda_stream)))


def lfc_encode_gpu(rgb, params: Params, want_stream: bool = True, cuda_stream=None):
    """lfc_encode_ex on the GPU.  rgb: uint8 [V][U][H][W][3], a CUDA tensor
    or a host array (copied to the device).  Returns (stream or None, stats)."""
    import torch
    if not isinstance(rgb, torch.Tensor):
        rgb = torch.from_numpy(np.ascontiguousarray(rgb, dtype=np.uint8)).cuda()
    assert rgb.dtype == torch.uint8 and rgb.is_cuda and rgb.is_contiguous()
    if tuple(rgb.shape) != (params.grid_v, params.grid_u, params.height, params.width, 3):
        raise ValueError(f"rgb shape {tuple(rgb.shape)} does not match the parameters")
    st = c_stats()
    out, n = C.c_void_p(), C.c_size_t()
    if want_stream:
        _check(load().lfc_encode_gpu(rgb.data_ptr(), C.byref(params.to_c()), C.byref(out), C.byref(n), C.byref(st),
                                     _stream_ptr(cuda_stream)))
    else:
        _check(load().lfc_encode_gpu(rgb.data_ptr(), C.byref(params.to_c()), None, None, C.byref(st),
                                     _stream_ptr(cuda_stream)))
    data = None
    if want_stream:
        try:
            data = C.string_at(out.value, n.value)
        finally:
            load().lfc_free(out)
    stats = dict(psnr=st.psnr, psnr_y=st.psnr_y, psnr_co=st.psnr_co, psnr_cg=st.psnr_cg,
                 present_blocks=st.present_blocks, code_hist=list(st.code_hist), stream_bytes=st.stream_bytes)
    return data, stats


def lfc_validate(stream: bytes) -> Params:
    p = c_params()
    buf = np.frombuffer(stream, dtype=np.uint8)
    _check(load().lfc_validate(buf.ctypes.data, buf.size, C.byref(p)))
    return Params.from_c(p)


class LightField:
    """An opened, device-resident compressed light field (wraps lfc_lf*)."""

    def __init__(self, handle: int):
        self.handle = handle
        self.info = lfc_info(self)

    @property
    def params(self) -> Params:
        return Params.from_c(self.info.params)

    def close(self) -> None:
        if self.handle:
            lfc_close(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lfc_open(stream: bytes, cuda_stream=None, tile_blocks: int = 0) -> LightField:
    """Opens a stream on the current device; tile_blocks: the whole-field
    decode's tile capacity (0: the default)."""
    buf = np.frombuffer(stream, dtype=np.uint8)
    h = C.c_void_p()
    if tile_blocks:
        cfg = c_open_config(tile_blocks)
        _check(load().lfc_open_ex(buf.ctypes.data, buf.size, C.byref(cfg), _stream_ptr(cuda_stream), C.byref(h)))
    else:
        _check(load().lfc_open(buf.ctypes.data, buf.size, _stream_ptr(cuda_stream), C.byref(h)))
    return LightField(h.value)


def lfc_info(lf: LightField) -> c_info:
    info = c_info()
    _check(load().lfc_info(lf.handle, C.byref(info)))
    return info


def lfc_decode_blocks(lf: LightField, req=None, layout: int = LAYOUT_BLOCKS, out=None, cuda_stream=None,
                      stage_cap_words: int | None = None):
    """Decodes blocks on the GPU.  req: int32 CUDA tensor [n][2] = (view, block)
    or None for every block.  Returns the int16 CUDA output tensor.
    stage_cap_words (images layout): None uses the handle's staging setting;
    -1 stages each strip in LDS as it needs; >= 0 caps the staging (0: none)."""
    import torch
    i = lf.info
    nv = i.params.grid_u * i.params.grid_v
    B = i.params.block
    if layout == LAYOUT_IMAGES:
        n = nv
        shape = (nv, 3, i.padded_height, i.padded_width)
    else:
        n = req.shape[0] if req is not None else nv * i.n_blocks
        shape = (n, 3, B, B)
    if req is not None:
        assert req.dtype == torch.int32 and req.is_cuda and req.is_contiguous() and req.dim() == 2
    if out is None:
        out = torch.empty(shape, dtype=torch.int16, device="cuda")
    assert out.dtype == torch.int16 and out.is_cuda and out.is_contiguous() and tuple(out.shape) == shape
    if stage_cap_words is None:
        _check(load().lfc_decode_blocks(lf.handle, req.data_ptr() if req is not None else None, n, layout,
                                        out.data_ptr(), _stream_ptr(cuda_stream)))
    else:
        cfg = c_decode_config(stage_cap_words)
        _check(load().lfc_decode_blocks_ex(lf.handle, req.data_ptr() if req is not None else None, n, layout,
                                           out.data_ptr(), C.byref(cfg), _stream_ptr(cuda_stream)))
    return out


def lfc_tune_decode(lf: LightField, reps: int = 5, out=None, cuda_stream=None):
    """Times the whole-field decode at several tile capacities and keeps the
    fastest in the handle; returns (kept capacity, [(capacity, ms)])."""
    import torch
    i = lf.info
    nv = i.params.grid_u * i.params.grid_v
    if out is None:
        out = torch.empty((nv, 3, i.padded_height, i.padded_width), dtype=torch.int16, device="cuda")
    res = c_decode_tuning()
    _check(load().lfc_tune_decode(lf.handle, out.data_ptr(), reps, C.byref(res), _stream_ptr(cuda_stream)))
    tried = [(int(res.tile_blocks[k]), float(res.ms[k])) for k in range(res.n_tried)]
    return tried[res.best][0], tried


def lfc_tune_decode_ex(lf: LightField, reps: int = 5, out=None, cuda_stream=None):
    """As lfc_tune_decode; returns ((kept capacity, kept staging), [(capacity, staged, ms)])."""
    import torch
    i = lf.info
    nv = i.params.grid_u * i.params.grid_v
    if out is None:
        out = torch.empty((nv, 3, i.padded_height, i.padded_width), dtype=torch.int16, device="cuda")
    res = c_decode_tuning()
    _check(load().lfc_tune_decode(lf.handle, out.data_ptr(), reps, C.byref(res), _stream_ptr(cuda_stream)))
    tried = [(int(res.tile_blocks[k]), bool(res.staged[k]), float(res.ms[k])) for k in range(res.n_tried)]
    return tried[res.best][:2], tried


def lfc_tune_decode_rgb(lf: LightField, reps: int = 5, out=None, cuda_stream=None):
    """Measured choice of the colour whole-field kernel's tile capacity (kept
    in the handle); returns (kept capacity, [(capacity, ms)])."""
    import torch
    i = lf.info
    shape = (i.params.grid_u * i.params.grid_v, i.padded_height, i.padded_width)
    if out is None:
        out = torch.empty(shape, dtype=torch.int32, device="cuda")
    assert out.dtype == torch.int32 and out.is_cuda and out.is_contiguous() and tuple(out.shape) == shape
    res = c_decode_tuning()
    _check(load().lfc_tune_decode_rgb(lf.handle, out.data_ptr(), reps, C.byref(res), _stream_ptr(cuda_stream)))
    tried = [(int(res.tile_blocks[k]), float(res.ms[k])) for k in range(res.n_tried)]
    return tried[res.best][0], tried


def lfc_stage_needs(lf: LightField) -> np.ndarray:
    """LDS words each strip of the whole-field decode needs: [strips][2] =
    (groups + schedule, schedule alone)."""
    L = load()
    n = L.lfc_stage_needs(lf.handle, None, 0)
    if n < 0:
        _check(int(n))
    out = np.zeros((n, 2), dtype=np.uint32)
    L.lfc_stage_needs(lf.handle, out.ctypes.data, n)
    return out


def lfc_decode_rgb(lf: LightField, out=None, cuda_stream=None):
    """Every view as 8-bit RGB: int32 CUDA tensor [nv][padded_height][padded_width]
    holding R | G << 8 | B << 16 per pixel."""
    import torch
    i = lf.info
    shape = (i.params.grid_u * i.params.grid_v, i.padded_height, i.padded_width)
    if out is None:
        out = torch.empty(shape, dtype=torch.int32, device="cuda")
    assert out.dtype == torch.int32 and out.is_cuda and out.is_contiguous() and tuple(out.shape) == shape
    _check(load().lfc_decode_rgb(lf.handle, out.data_ptr(), _stream_ptr(cuda_stream)))
    return out


def lfc_decode_progressive(lf: LightField, req, level: int, out=None, cuda_stream=None):
    """Progressive decompression: blocks [n][3][B][B] reconstructed down to
    tree level `level` only.  req: int32 CUDA tensor [n][2] or None (all)."""
    import torch
    i = lf.info
    B = i.params.block
    n = req.shape[0] if req is not None else i.params.grid_u * i.params.grid_v * i.n_blocks
    if req is not None:
        assert req.dtype == torch.int32 and req.is_cuda and req.is_contiguous() and req.dim() == 2
    if out is None:
        out = torch.empty((n, 3, B, B), dtype=torch.int16, device="cuda")
    assert out.dtype == torch.int16 and out.is_cuda and out.is_contiguous() and tuple(out.shape) == (n, 3, B, B)
    _check(load().lfc_decode_progressive(lf.handle, req.data_ptr() if req is not None else None, n, level,
                                         out.data_ptr(), _stream_ptr(cuda_stream)))
    return out


def _render_buffers(views, out_w: int, out_h: int, out):
    import torch
    assert views.dtype == torch.float32 and views.is_cuda and views.is_contiguous() and views.shape[-1] == 4
    n = views.shape[0]
    if out is None:
        out = torch.empty((n, 3, out_h, out_w), dtype=torch.float32, device="cuda")
    assert out.dtype == torch.float32 and out.is_cuda and out.is_contiguous()
    assert tuple(out.shape) == (n, 3, out_h, out_w)
    return n, out


def _config(cfg, disparity: float = 0.0):
    """None, or (path, tile_w, tile_h[, disparity]); a nonzero disparity
    alone gives the automatic shape refocused."""
    if cfg is None and disparity == 0.0:
        return None
    c = c_render_config(*(cfg if cfg is not None else (RENDER_AUTO, 0, 0)))
    if disparity != 0.0:
        c.disparity = disparity
    return C.byref(c)


def lfc_render_views(lf: LightField, views, out_w: int, out_h: int, out=None, cuda_stream=None, cfg=None,
                     disparity: float = 0.0):
    """Renders novel views: views float32 CUDA tensor [n][4] = (u, v, s, t).
    Returns float32 CUDA [n][3][out_h][out_w], RGB / 255.  cfg: None
    (automatic) or (path, tile_w, tile_h) with path RENDER_TILES or
    RENDER_DECODED; disparity refocuses (include/lfc.h)."""
    n, out = _render_buffers(views, out_w, out_h, out)
    if cfg is None and disparity == 0.0:
        _check(load().lfc_render_views(lf.handle, views.data_ptr(), n, out_w, out_h, out.data_ptr(),
                                       _stream_ptr(cuda_stream)))
    else:
        _check(load().lfc_render_views_ex(lf.handle, views.data_ptr(), n, out_w, out_h, out.data_ptr(),
                                          _config(cfg, disparity), _stream_ptr(cuda_stream)))
    return out


def lfc_render_views_noalloc(lf: LightField, views, out_w: int, out_h: int, out, cuda_stream=None, cfg=None,
                             disparity: float = 0.0):
    """lfc_render_views through the entry point that allocates nothing: the
    decoded path uses the library's static device scratch.  out must be given
    (float32 CUDA [n][3][out_h][out_w]); cfg and disparity as lfc_render_views."""
    n, out = _render_buffers(views, out_w, out_h, out)
    _check(load().lfc_render_views_noalloc(lf.handle, views.data_ptr(), n, out_w, out_h, out.data_ptr(),
                                           _config(cfg, disparity), _stream_ptr(cuda_stream)))
    return out


def lfc_render_tune(lf: LightField, views, out_w: int, out_h: int, out=None, reps: int = 5, cuda_stream=None):
    """Times every render launch shape on these views; returns (best config,
    [(config, ms per launch)]) with configs as (path, tile_w, tile_h)."""
    n, out = _render_buffers(views, out_w, out_h, out)
    res = c_render_tuning()
    _check(load().lfc_render_tune(lf.handle, views.data_ptr(), n, out_w, out_h, out.data_ptr(), reps,
                                  C.byref(res), _stream_ptr(cuda_stream)))
    tried = [((res.cfg[i].path, res.cfg[i].tile_w, res.cfg[i].tile_h), float(res.ms[i])) for i in range(res.n_tried)]
    return tried[res.best][0], tried


class RenderPlan:
    """One render with its launch shape and buffers fixed, optionally
    captured in a HIP graph (launch() is then one graph launch).  The views
    tensor is read at each launch; rewrite it in place between launches."""

    def __init__(self, lf: LightField, views, out_w: int, out_h: int, out=None, cfg=None, graph: bool = True,
                 disparity: float = 0.0):
        n, self.out = _render_buffers(views, out_w, out_h, out)
        self.views, self.lf = views, lf
        h = C.c_void_p()
        _check(load().lfc_render_plan_create(lf.handle, _config(cfg, disparity), views.data_ptr(), n, out_w, out_h,
                                             self.out.data_ptr(), int(graph), C.byref(h)))
        self.handle = h.value

    def launch(self, cuda_stream=None):
        _check(load().lfc_render_plan_launch(self.handle, _stream_ptr(cuda_stream)))
        return self.out

    def info(self):
        c, g = c_render_config(), C.c_int32()
        _check(load().lfc_render_plan_info(self.handle, C.byref(c), C.byref(g)))
        return (c.path, c.tile_w, c.tile_h), bool(g.value)

    def close(self) -> None:
        h, self.handle = self.handle, None
        if h:
            load().lfc_render_plan_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lfc_check(lf: LightField, cuda_stream=None) -> None:
    _check(load().lfc_check(lf.handle, _stream_ptr(cuda_stream)))


def lfc_close(lf: LightField) -> None:
    h, lf.handle = lf.handle, None
    if h:
        _check(load().lfc_close(h))


def _requests(reqs) -> "C.Array":
    """reqs: sequence of (lf index, out_w, out_h, (u, v, s, t))."""
    arr = (c_render_request * len(reqs))()
    for k, (li, w, h, v) in enumerate(reqs):
        arr[k].lf, arr[k].out_w, arr[k].out_h = int(li), int(w), int(h)
        arr[k].view.u, arr[k].view.v, arr[k].view.s, arr[k].view.t = (float(x) for x in v)
    return arr


def _handles(lfs) -> "C.Array":
    return (C.c_void_p * len(lfs))(*[lf.handle for lf in lfs])


class Batch:
    """Staging for batched renders across light fields (wraps lfc_batch*)."""

    def __init__(self):
        h = C.c_void_p()
        _check(load().lfc_batch_create(C.byref(h)))
        self.handle = h.value

    def render(self, lfs, reqs, outs=None, cuda_stream=None):
        """Renders reqs = [(lf index, out_w, out_h, (u, v, s, t))] of the light
        fields lfs in one launch per block size.  Returns the float32 CUDA
        outputs [3][out_h][out_w], one per request."""
        import torch
        if outs is None:
            outs = [torch.empty((3, h, w), dtype=torch.float32, device="cuda") for _, w, h, _ in reqs]
        for o, (_, w, h, _) in zip(outs, reqs):
            assert o.dtype == torch.float32 and o.is_cuda and o.is_contiguous() and tuple(o.shape) == (3, h, w)
        ptrs = (C.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        _check(load().lfc_batch_render(self.handle, _handles(lfs), len(lfs), _requests(reqs), len(reqs), ptrs,
                                       _stream_ptr(cuda_stream)))
        return outs

    def decode(self, lfs, req, out=None, cuda_stream=None):
        """Random access over several light fields (same block size): req
        int32 CUDA tensor [n][3] = (light-field index, view, block).  Returns
        int16 CUDA [n][3][B][B]."""
        import torch
        assert req.dtype == torch.int32 and req.is_cuda and req.is_contiguous() and req.dim() == 2
        n = req.shape[0]
        B = lfs[0].info.params.block
        if out is None:
            out = torch.empty((n, 3, B, B), dtype=torch.int16, device="cuda")
        assert out.dtype == torch.int16 and out.is_cuda and out.is_contiguous() and tuple(out.shape) == (n, 3, B, B)
        _check(load().lfc_batch_decode(self.handle, _handles(lfs), len(lfs), req.data_ptr(), n, out.data_ptr(),
                                       _stream_ptr(cuda_stream)))
        return out

    def check(self, cuda_stream=None) -> None:
        _check(load().lfc_batch_check(self.handle, _stream_ptr(cuda_stream)))

    def close(self) -> None:
        h, self.handle = self.handle, None
        if h:
            _check(load().lfc_batch_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """One batched render across light fields fixed once (wraps
    lfc_batch_plan*): the request table is built at creation and, with
    graph, the launches are captured in a HIP graph (launch() is then one
    graph launch).  reqs as Batch.render."""

    def __init__(self, lfs, reqs, outs=None, graph: bool = True):
        import torch
        if outs is None:
            outs = [torch.empty((3, h, w), dtype=torch.float32, device="cuda") for _, w, h, _ in reqs]
        for o, (_, w, h, _) in zip(outs, reqs):
            assert o.dtype == torch.float32 and o.is_cuda and o.is_contiguous() and tuple(o.shape) == (3, h, w)
        self.lfs, self.outs = list(lfs), outs
        ptrs = (C.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        h = C.c_void_p()
        _check(load().lfc_batch_plan_create(_handles(lfs), len(lfs), _requests(reqs), len(reqs), ptrs, int(graph),
                                            C.byref(h)))
        self.handle = h.value

    def launch(self, cuda_stream=None):
        _check(load().lfc_batch_plan_launch(self.handle, _stream_ptr(cuda_stream)))
        return self.outs

    def info(self):
        """(light fields on the decoded colour path, graph in use)."""
        k, g = C.c_int32(), C.c_int32()
        _check(load().lfc_batch_plan_info(self.handle, C.byref(k), C.byref(g)))
        return int(k.value), bool(g.value)

    def close(self) -> None:
        h, self.handle = self.handle, None
        if h:
            load().lfc_batch_plan_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop over resident light fields (wraps lfc_server*)."""

    def __init__(self, lfs, max_batch: int = 64, streams: int = 2, out_pool_bytes: int = 1 << 30,
                 max_queue: int = 0, device_bytes_cap: int = 0):
        self.lfs = list(lfs)   # the handles must outlive the server
        cfg = c_server_config(max_batch, streams, out_pool_bytes, max_queue, device_bytes_cap)
        h = C.c_void_p()
        _check(load().lfc_server_create(_handles(self.lfs), len(self.lfs), C.byref(cfg), C.byref(h)))
        self.handle = h.value

    def submit(self, lf: int, out_w: int, out_h: int, view) -> int:
        t = C.c_uint64()
        _check(load().lfc_server_submit(self.handle, _requests([(lf, out_w, out_h, view)]), C.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1):
        """Returns (device pointer of the float32 [3][out_h][out_w] result, latency ms)."""
        p, lat = C.c_void_p(), C.c_double()
        _check(load().lfc_server_wait(self.handle, ticket, timeout_ms, C.byref(p), C.byref(lat)))
        return p.value, lat.value

    def fetch(self, ticket: int, out_w: int, out_h: int, timeout_ms: int = -1):
        """Waits, copies the result into a new CUDA tensor, releases it.

        The copy has finished before the release: a device-to-device
        hipMemcpy may return while it is still running, and the server may
        hand the released pool memory to the next request at once."""
        import torch
        ptr, lat = self.wait(ticket, timeout_ms)
        out = torch.empty((3, out_h, out_w), dtype=torch.float32, device="cuda")
        hip = C.CDLL("libamdhip64.so")
        hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        hip.hipStreamSynchronize.argtypes = [C.c_void_p]
        stream = torch.cuda.current_stream().cuda_stream
        st = hip.hipMemcpyAsync(out.data_ptr(), ptr, out.numel() * 4, 3, stream)   # device to device
        if st == 0:
            st = hip.hipStreamSynchronize(stream)
        self.release(ticket)
        if st != 0:
            raise LFCError(-4, f"device copy failed ({st})")
        return out, lat

    def release(self, ticket: int) -> None:
        _check(load().lfc_server_release(self.handle, ticket))

    def replay(self, reqs, arrival_ms) -> np.ndarray:
        """Submits reqs[i] at arrival_ms[i] (from now), discards the results,
        returns the latencies (ms) from arrival to completion."""
        n = len(reqs)
        arr = np.ascontiguousarray(arrival_ms, dtype=np.float64)
        lat = np.zeros(n, dtype=np.float64)
        _check(load().lfc_server_replay(self.handle, _requests(reqs), arr.ctypes.data_as(C.POINTER(C.c_double)), n,
                                        lat.ctypes.data_as(C.POINTER(C.c_double))))
        return lat

    def stats(self) -> dict:
        st = c_server_stats()
        _check(load().lfc_server_get_stats(self.handle, C.byref(st)))
        return {f: getattr(st, f) for f, _ in c_server_stats._fields_}

    def close(self) -> None:
        h, self.handle = self.handle, None
        if h:
            _check(load().lfc_server_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
