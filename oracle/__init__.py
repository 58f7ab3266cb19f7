"""RLFC reference oracle -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``oracle/liboracle.so`` (plain C, see ``oracle.h``).
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the library in
``paper_1805_06019_amd``; the two meet only in the seeded input generator.

Every function follows a passage of Pratapa & Manocha, "RLFC: Random Access
Light Field Compression using Key Views and Bounded Integer Sequence
Encoding" (I3D 2019, arXiv 1805.06019); the C source names the passage.

Parity unpinned: the quantiser (the paper defers it to its supplementary
Section 3) and bpp/PSNR against the paper's Tables 1-4.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
MAX_LEVELS = 6


class _Params(C.Structure):
    _fields_ = [
        ("grid_u", C.c_int32), ("grid_v", C.c_int32),
        ("width", C.c_int32), ("height", C.c_int32),
        ("block", C.c_int32), ("levels", C.c_int32),
        ("cluster", C.c_int32 * MAX_LEVELS),
        ("pix_threshold", C.c_int32), ("blk_threshold", C.c_int32),
        ("quant_bits", C.c_int32), ("range_mask", C.c_uint32),
    ]


class _Control(C.Structure):
    _fields_ = [("mode", C.c_int32), ("lambda_q16", C.c_int64),
                ("classes_in", C.c_void_p), ("ranges_in", C.c_void_p),
                ("classes_out", C.c_void_p), ("ranges_out", C.c_void_p), ("features_out", C.c_void_p)]


CTL_GLOBAL, CTL_SEARCH, CTL_TABLE = 0, 1, 2


class _Geom(C.Structure):
    _fields_ = [
        ("wp", C.c_int32), ("hp", C.c_int32),
        ("nbx", C.c_int32), ("nby", C.c_int32), ("nb", C.c_int32), ("ng", C.c_int32),
        ("n_srv", C.c_int32), ("n_top", C.c_int32),
        ("lu", C.c_int32 * MAX_LEVELS), ("lv", C.c_int32 * MAX_LEVELS),
    ]


@dataclass
class Params:
    """Encoding parameters (Sec. 3.1-3.3; Alg. 1 'enc')."""
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

    def c(self) -> _Params:
        p = _Params()
        p.grid_u, p.grid_v, p.width, p.height = self.grid_u, self.grid_v, self.width, self.height
        p.block, p.levels = self.block, self.levels
        for i in range(MAX_LEVELS):
            p.cluster[i] = self.cluster[i] if i < len(self.cluster) else 0
        p.pix_threshold, p.blk_threshold = self.pix_threshold, self.blk_threshold
        p.quant_bits, p.range_mask = self.quant_bits, self.range_mask
        return p


@dataclass
class Geom:
    wp: int
    hp: int
    nbx: int
    nby: int
    nb: int
    ng: int
    n_srv: int
    n_top: int
    lu: list = field(default_factory=list)
    lv: list = field(default_factory=list)


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.orc_geometry.argtypes = [C.POINTER(_Params), C.POINTER(_Geom)]
        L.orc_ycocg_forward.argtypes = [vp, i64, vp]
        L.orc_ycocg_forward.restype = None
        L.orc_ycocg_inverse.argtypes = [vp, i64, vp]
        L.orc_ycocg_inverse.restype = None
        L.orc_bise_range.argtypes = [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_bise_bits.argtypes = [C.c_int, C.c_int]
        L.orc_bise_encode.argtypes = [vp, C.c_int, C.c_int, vp, i64]
        L.orc_bise_decode.argtypes = [vp, i64, C.c_int, C.c_int, vp]
        L.orc_zigzag.argtypes = [i32]
        L.orc_zigzag.restype = i32
        L.orc_unzigzag.argtypes = [i32]
        L.orc_unzigzag.restype = i32
        L.orc_quantize.argtypes = [i32, C.c_int]
        L.orc_quantize.restype = i32
        L.orc_tree_tables.argtypes = [C.POINTER(_Params), vp, vp]
        L.orc_rkv_tree.argtypes = [vp, C.POINTER(_Params), vp]
        L.orc_encode.argtypes = [vp, C.POINTER(_Params), C.POINTER(C.c_void_p), C.POINTER(i64), vp, vp, vp]
        L.orc_encode_ctl.argtypes = [vp, C.POINTER(_Params), C.POINTER(_Control), C.POINTER(C.c_void_p),
                                     C.POINTER(i64), vp, vp, vp]
        L.orc_free.argtypes = [vp]
        L.orc_free.restype = None
        L.orc_read_header.argtypes = [vp, i64, C.POINTER(_Params), C.POINTER(_Geom)]
        L.orc_decode_block.argtypes = [vp, i64, i32, i32, vp]
        L.orc_decode_requests.argtypes = [vp, i64, i64, vp, vp]
        L.orc_decode_block_level.argtypes = [vp, i64, i32, i32, i32, vp]
        L.orc_decode_all.argtypes = [vp, i64, i32, i32, vp]
        L.orc_render.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, i32, i32, i32, vp]
        L.orc_render_focal.argtypes = [vp, i32, i32, i32, i32, i32, i32, vp, i32, i32, i32, C.c_float, vp]
        L.orc_psnr.argtypes = [vp, vp, i32, i32, i32, i32, i32]
        L.orc_psnr.restype = C.c_double
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _check(st: int, what: str) -> None:
    if st != 0:
        raise OracleError(f"{what} failed with status {st}")


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def geometry(p: Params) -> Geom:
    g = _Geom()
    _check(lib().orc_geometry(C.byref(p.c()), C.byref(g)), "orc_geometry")
    return Geom(g.wp, g.hp, g.nbx, g.nby, g.nb, g.ng, g.n_srv, g.n_top,
                list(g.lu)[: p.levels], list(g.lv)[: p.levels])


# -- colour (Sec. 4) ---------------------------------------------------------

def ycocg_forward(rgb: np.ndarray) -> np.ndarray:
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    out = np.empty(rgb.shape, dtype=np.int16)
    lib().orc_ycocg_forward(_ptr(rgb), rgb.size // 3, _ptr(out))
    return out


def ycocg_inverse(ycc: np.ndarray) -> np.ndarray:
    ycc = np.ascontiguousarray(ycc, dtype=np.int16)
    out = np.empty(ycc.shape, dtype=np.uint8)
    lib().orc_ycocg_inverse(_ptr(ycc), ycc.size // 3, _ptr(out))
    return out


# -- BISE (Sec. 3.3) ---------------------------------------------------------

def bise_range(code: int):
    k, m, n = C.c_int(), C.c_int(), C.c_int()
    _check(lib().orc_bise_range(code, C.byref(k), C.byref(m), C.byref(n)), "orc_bise_range")
    return ("bits", "trit", "quint")[k.value], m.value, n.value


def bise_bits(code: int, S: int) -> int:
    r = lib().orc_bise_bits(code, S)
    if r < 0:
        raise OracleError(f"bise_bits({code},{S}) -> {r}")
    return r


def bise_encode(vals, code: int, bitpos: int = 0, nwords: int | None = None) -> np.ndarray:
    v = np.ascontiguousarray(vals, dtype=np.uint16)
    nbits = bise_bits(code, v.size)
    if nwords is None:
        nwords = (bitpos + nbits + 31) // 32 + 1
    words = np.zeros(nwords, dtype=np.uint32)
    r = lib().orc_bise_encode(_ptr(v), v.size, code, _ptr(words), bitpos)
    if r < 0:
        raise OracleError(f"bise_encode -> {r}")
    return words


def bise_decode(words: np.ndarray, S: int, code: int, bitpos: int = 0) -> np.ndarray:
    w = np.ascontiguousarray(words, dtype=np.uint32)
    out = np.zeros(S, dtype=np.uint16)
    r = lib().orc_bise_decode(_ptr(w), bitpos, S, code, _ptr(out))
    if r < 0:
        raise OracleError(f"bise_decode -> {r}")
    return out


def zigzag(v: int) -> int:
    return lib().orc_zigzag(v)


def unzigzag(z: int) -> int:
    return lib().orc_unzigzag(z)


def quantize(r: int, q: int) -> int:
    return lib().orc_quantize(r, q)


# -- tree (Sec. 3.1, 3.4) ----------------------------------------------------

def tree_tables(p: Params):
    nv = p.grid_u * p.grid_v
    path = np.zeros((nv, max(p.levels - 1, 1)), dtype=np.int32)
    root = np.zeros(nv, dtype=np.int32)
    _check(lib().orc_tree_tables(C.byref(p.c()), _ptr(path), _ptr(root)), "orc_tree_tables")
    return path[:, : p.levels - 1], root


def rkv_tree(rgb: np.ndarray, p: Params):
    g = geometry(p)
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    sizes = [g.lu[l] * g.lv[l] for l in range(p.levels)]
    img = 3 * g.hp * g.wp
    out = np.zeros(sum(sizes) * img, dtype=np.int32)
    _check(lib().orc_rkv_tree(_ptr(rgb), C.byref(p.c()), _ptr(out)), "orc_rkv_tree")
    levels, off = [], 0
    for l, n in enumerate(sizes):
        levels.append(out[off: off + n * img].reshape(g.lv[l], g.lu[l], 3, g.hp, g.wp))
        off += n * img
    return levels


# -- CompressLFI / DecompressLFIBlock (Alg. 1, Alg. 2) ------------------------

@dataclass
class Encoded:
    stream: bytes
    r0: np.ndarray      # closed-loop level-0 reconstruction [U*V][3][hp][wp]
    ycocg: np.ndarray   # padded YCoCg-R planes of the input, same layout
    hist: np.ndarray    # present blocks per range code


def encode(rgb: np.ndarray, p: Params, want_planes: bool = True) -> Encoded:
    """rgb is [V][U][H][W][3] uint8 (view index vi = v*U + u)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    assert rgb.shape == (p.grid_v, p.grid_u, p.height, p.width, 3), rgb.shape
    g = geometry(p)
    nv = p.grid_u * p.grid_v
    r0 = np.zeros((nv, 3, g.hp, g.wp), dtype=np.int16) if want_planes else None
    ycc = np.zeros((nv, 3, g.hp, g.wp), dtype=np.int16) if want_planes else None
    hist = np.zeros(26, dtype=np.int64)
    out = C.c_void_p()
    nbytes = C.c_int64()
    st = lib().orc_encode(_ptr(rgb), C.byref(p.c()), C.byref(out), C.byref(nbytes),
                          _ptr(r0) if r0 is not None else None,
                          _ptr(ycc) if ycc is not None else None, _ptr(hist))
    _check(st, "orc_encode")
    try:
        data = C.string_at(out.value, nbytes.value)
    finally:
        lib().orc_free(out)
    return Encoded(data, r0, ycc, hist)


def control_rows(p: Params) -> int:
    """Residual (node, block, channel) triples: one encoder decision each."""
    g = geometry(p)
    return sum(g.lu[l] * g.lv[l] for l in range(p.levels - 1)) * g.nb * 3


def encode_ctl(rgb: np.ndarray, p: Params, mode: int, lambda_q16: int = 0, classes=None, ranges=None,
               want_features: bool = False):
    """Encoder under per-block control (see oracle.h): returns (Encoded,
    threshold classes used, range classes used, features or None)."""
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    assert rgb.shape == (p.grid_v, p.grid_u, p.height, p.width, 3), rgb.shape
    g = geometry(p)
    nv = p.grid_u * p.grid_v
    rows = control_rows(p)
    r0 = np.zeros((nv, 3, g.hp, g.wp), dtype=np.int16)
    hist = np.zeros(26, dtype=np.int64)
    cls_out = np.full(rows, -1, dtype=np.int8)
    rng_out = np.full(rows, -1, dtype=np.int8)
    feat = np.zeros((rows, 16), dtype=np.float32) if want_features else None
    ctl = _Control()
    ctl.mode, ctl.lambda_q16 = mode, lambda_q16
    if mode == CTL_TABLE:
        classes = np.ascontiguousarray(classes, dtype=np.int8)
        ranges = np.ascontiguousarray(ranges, dtype=np.int8)
        assert classes.size == rows and ranges.size == rows
        ctl.classes_in, ctl.ranges_in = _ptr(classes), _ptr(ranges)
    ctl.classes_out, ctl.ranges_out = _ptr(cls_out), _ptr(rng_out)
    ctl.features_out = _ptr(feat) if feat is not None else None
    out = C.c_void_p()
    nbytes = C.c_int64()
    st = lib().orc_encode_ctl(_ptr(rgb), C.byref(p.c()), C.byref(ctl), C.byref(out), C.byref(nbytes),
                              _ptr(r0), None, _ptr(hist))
    _check(st, "orc_encode_ctl")
    try:
        data = C.string_at(out.value, nbytes.value)
    finally:
        lib().orc_free(out)
    return Encoded(data, r0, None, hist), cls_out, rng_out, feat


def _sbuf(stream: bytes) -> np.ndarray:
    return np.frombuffer(stream, dtype=np.uint8)


def read_header(stream: bytes):
    p, g = _Params(), _Geom()
    s = _sbuf(stream)
    _check(lib().orc_read_header(_ptr(s), s.size, C.byref(p), C.byref(g)), "orc_read_header")
    params = Params(p.grid_u, p.grid_v, p.width, p.height, p.block, p.levels,
                    tuple(p.cluster[i] for i in range(p.levels - 1)), p.pix_threshold,
                    p.blk_threshold, p.quant_bits, p.range_mask)
    geom = Geom(g.wp, g.hp, g.nbx, g.nby, g.nb, g.ng, g.n_srv, g.n_top,
                list(g.lu)[: p.levels], list(g.lv)[: p.levels])
    return params, geom


def decode_block(stream: bytes, vi: int, b: int) -> np.ndarray:
    p, _ = read_header(stream)
    s = _sbuf(stream)
    out = np.zeros((3, p.block, p.block), dtype=np.int16)
    _check(lib().orc_decode_block(_ptr(s), s.size, vi, b, _ptr(out)), "orc_decode_block")
    return out


def decode_requests(stream: bytes, req: np.ndarray, out: np.ndarray | None = None) -> np.ndarray:
    """decode_block for every (view, block) row of req (int32 [n][2]), in C:
    [n][3][B][B]."""
    p, _ = read_header(stream)
    s = _sbuf(stream)
    req = np.ascontiguousarray(req, dtype=np.int32).reshape(-1, 2)
    if out is None:
        out = np.zeros((req.shape[0], 3, p.block, p.block), dtype=np.int16)
    assert out.dtype == np.int16 and out.flags.c_contiguous and out.shape[0] == req.shape[0]
    _check(lib().orc_decode_requests(_ptr(s), s.size, req.shape[0], _ptr(req), _ptr(out)), "orc_decode_requests")
    return out


def decode_block_level(stream: bytes, vi: int, b: int, level: int) -> np.ndarray:
    """Progressive decompression (Sec. 3.6): block b of view vi reconstructed
    only down to tree level `level`."""
    p, _ = read_header(stream)
    s = _sbuf(stream)
    out = np.zeros((3, p.block, p.block), dtype=np.int16)
    _check(lib().orc_decode_block_level(_ptr(s), s.size, vi, b, level, _ptr(out)), "orc_decode_block_level")
    return out


def decode_all(stream: bytes, b0: int = 0, b1: int | None = None, out: np.ndarray | None = None):
    p, g = read_header(stream)
    s = _sbuf(stream)
    if b1 is None:
        b1 = g.nb
    if out is None:
        out = np.zeros((p.grid_u * p.grid_v, 3, g.hp, g.wp), dtype=np.int16)
    assert out.dtype == np.int16 and out.flags.c_contiguous
    _check(lib().orc_decode_all(_ptr(s), s.size, b0, b1, _ptr(out)), "orc_decode_all")
    return out


def render(lf: np.ndarray, U: int, V: int, W: int, H: int, views: np.ndarray, wo: int, ho: int,
           disparity: float = 0.0):
    """Sec. 3.6 two-plane interpolation; disparity != 0 refocuses it."""
    lf = np.ascontiguousarray(lf, dtype=np.int16)
    views = np.ascontiguousarray(views, dtype=np.float32).reshape(-1, 4)
    n = views.shape[0]
    hp, wp = lf.shape[2], lf.shape[3]
    out = np.zeros((n, 3, ho, wo), dtype=np.float32)
    if disparity == 0.0:
        st = lib().orc_render(_ptr(lf), U, V, W, H, wp, hp, _ptr(views), n, wo, ho, _ptr(out))
    else:
        st = lib().orc_render_focal(_ptr(lf), U, V, W, H, wp, hp, _ptr(views), n, wo, ho, disparity, _ptr(out))
    _check(st, "orc_render")
    return out


def psnr(ref: np.ndarray, dec: np.ndarray, W: int, H: int) -> float:
    ref = np.ascontiguousarray(ref, dtype=np.int16)
    dec = np.ascontiguousarray(dec, dtype=np.int16)
    assert ref.shape == dec.shape
    nv, _, hp, wp = ref.shape
    return lib().orc_psnr(_ptr(ref), _ptr(dec), nv, W, H, wp, hp)
