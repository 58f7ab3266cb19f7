"""Host-side tests of liblfc.so (no GPU needed).

* the library loads and exports every function include/lfc.h declares;
* lfc_encode, written independently of the oracle, produces byte-identical
  streams on every geometry and parameter set tried (two implementations of
  one deterministic reading of Alg. 1);
* lfc_validate accepts those streams and rejects corrupted ones (bit flips,
  truncation, bad codes, out-of-range digit fields) without crashing;
* parameter errors come back as LFC_E_INVALID with a message.
"""
import ctypes as C
import os
import re
import struct

import numpy as np
import pytest

import oracle
from paper_1805_06019_amd import lfc, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(lfc_[a-z_]+)\s*\(", txt)
    return sorted(set(names))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert {"lfc_encode", "lfc_open", "lfc_decode_blocks", "lfc_render_views", "lfc_close"} <= set(names)
    lib = C.CDLL(lfc.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def _both(lf, **kw):
    V, U, H, W, _ = lf.shape
    ok = dict(grid_u=U, grid_v=V, width=W, height=H)
    ok.update(kw)
    a = oracle.encode(lf, oracle.Params(**ok), want_planes=False).stream
    b = lfc.lfc_encode(lf, lfc.Params(**ok))
    return a, b


CASES = [
    # U, V, W, H, layers, disparity, sigma, params
    (8, 8, 64, 64, 3, 2.0, 2.0, dict(block=4, levels=2, cluster=(2,), blk_threshold=2)),
    (1, 1, 9, 7, 2, 0.0, 2.0, dict(block=4, levels=1, cluster=())),
    (3, 5, 13, 9, 3, 1.0, 2.0, dict(block=4, levels=2, cluster=(2,))),
    (17, 17, 16, 16, 4, 3.0, 1.5, dict(block=4, levels=3, cluster=(2, 3), blk_threshold=40, quant_bits=1)),
    (9, 9, 25, 18, 4, 1.0, 1.0, dict(block=4, levels=3, cluster=(2, 2), pix_threshold=2, blk_threshold=20, quant_bits=2)),
    (5, 4, 20, 12, 3, 2.0, 3.0, dict(block=8, levels=2, cluster=(3,), blk_threshold=100, quant_bits=3)),
    (6, 3, 10, 6, 3, 2.0, 3.0, dict(block=2, levels=3, cluster=(2, 2), pix_threshold=1, blk_threshold=3)),
    (7, 7, 12, 12, 3, 2.0, 2.0, dict(block=4, levels=4, cluster=(2, 2, 2), quant_bits=4, blk_threshold=10)),
    (4, 4, 16, 16, 3, 2.0, 2.0, dict(block=4, levels=2, cluster=(2,), range_mask=(1 << 12) - 1)),
    (4, 4, 16, 16, 3, 2.0, 2.0, dict(block=4, levels=2, cluster=(2,), range_mask=0x3F80000 | 0x7F000 | (0xF << 8))),
    (2, 2, 9, 9, 2, 1.0, 4.0, dict(block=8, levels=2, cluster=(2,))),
]


@pytest.mark.parametrize("case", CASES)
def test_encoder_byte_identical_to_oracle(case):
    U, V, W, H, layers, disp, sigma, kw = case
    lf = synth.light_field(synth.LFSpec(U, V, W, H, layers, disp, sigma, 1000 + U * 7 + W), threads=1)
    a, b = _both(lf, **kw)
    assert len(a) == len(b)
    assert a == b
    p = lfc.lfc_validate(b)
    assert (p.grid_u, p.grid_v, p.width, p.height, p.block, p.levels) == (U, V, W, H, kw["block"], kw["levels"])


def test_encoder_hand_derived_stream():
    lf = np.zeros((1, 2, 4, 4, 3), dtype=np.uint8)
    lf[0, 0] = 100
    lf[0, 1] = 104
    a, b = _both(lf, block=4, levels=2, cluster=(2,))
    assert a == b and len(b) == 268


def _stream():
    lf = synth.light_field(synth.LFSpec(8, 8, 32, 32, 3, 2.0, 2.0, 5), threads=1)
    return lfc.lfc_encode(lf, lfc.Params(8, 8, 32, 32, 4, 3, (2, 2), 0, 20, 1))


def test_validator_rejects_truncation_and_trailing_bytes():
    s = _stream()
    lfc.lfc_validate(s)
    for cut in (0, 10, 127, 128, 200, len(s) // 2, len(s) - 4, len(s) - 1):
        with pytest.raises(lfc.LFCError) as e:
            lfc.lfc_validate(s[:cut])
        assert e.value.status == -2
    with pytest.raises(lfc.LFCError):
        lfc.lfc_validate(s + b"\0\0\0\0")


def test_validator_survives_random_bit_flips():
    # flips in key-view samples or in BISE low bits give legal streams; the
    # validator must simply never crash and must report CORRUPT or accept
    s = bytearray(_stream())
    rng = np.random.default_rng(1)
    for trial in range(400):
        t = bytearray(s)
        for _ in range(rng.integers(1, 4)):
            pos = int(rng.integers(0, len(t)))
            t[pos] ^= 1 << int(rng.integers(0, 8))
        try:
            lfc.lfc_validate(bytes(t))
        except lfc.LFCError as e:
            assert e.status == -2


def test_validator_rejects_any_offset_flip():
    s = _stream()
    off, srv_off = _srv_words(s)
    off_off = struct.unpack_from("<Q", s, 112)[0]
    rng = np.random.default_rng(2)
    for trial in range(200):
        t = bytearray(s)
        pos = off_off + int(rng.integers(0, srv_off - off_off))
        t[pos] ^= 1 << int(rng.integers(0, 8))
        with pytest.raises(lfc.LFCError) as e:
            lfc.lfc_validate(bytes(t))
        assert e.value.status == -2


def _srv_words(s):
    ng = struct.unpack_from("<i", s, 96)[0]
    off_off, srv_off = struct.unpack_from("<QQ", s, 112)
    off = np.frombuffer(s, dtype=np.uint32, count=ng + 1, offset=off_off)
    return off, srv_off


def test_validator_rejects_bad_code_and_digit_field():
    s = bytearray(_stream())
    off, srv_off = _srv_words(bytes(s))
    gi = int(np.nonzero(np.diff(off.astype(np.int64)))[0][0])
    nbw = (struct.unpack_from("<i", s, 84)[0] + 31) // 32
    code_word = srv_off + 4 * (int(off[gi]) + nbw)
    t = bytearray(s)
    w = struct.unpack_from("<I", t, code_word)[0]
    struct.pack_into("<I", t, code_word, (w & ~31) | 27)   # first code := 27 (reserved)
    with pytest.raises(lfc.LFCError):
        lfc.lfc_validate(bytes(t))
    # a stream whose first stored block is a trit block with its first field
    # set to 255 (>= 3^5) must be rejected
    lf = np.zeros((1, 2, 4, 4, 3), dtype=np.uint8)
    lf[0, 0] = 100
    lf[0, 1] = 101
    s2 = bytearray(lfc.lfc_encode(lf, lfc.Params(2, 1, 4, 4, 4, 2, (2,), range_mask=1 << 13)))
    lfc.lfc_validate(bytes(s2))
    # group 0: bitmap word, code word, then the payload starting with the trit field
    struct.pack_into("<B", s2, 240 + 8, 255)
    with pytest.raises(lfc.LFCError):
        lfc.lfc_validate(bytes(s2))


@pytest.mark.parametrize("bad", [
    dict(block=3), dict(levels=0), dict(levels=7), dict(cluster=(1,)), dict(quant_bits=5),
    dict(blk_threshold=-1), dict(range_mask=1 << 26), dict(grid_u=0), dict(width=0),
])
def test_encoder_rejects_bad_parameters(bad):
    kw = dict(grid_u=2, grid_v=2, width=8, height=8, block=4, levels=2, cluster=(2,))
    kw.update(bad)
    p = lfc.Params(**kw)
    rgb = np.zeros((max(p.grid_v, 1), max(p.grid_u, 1), max(p.height, 1), max(p.width, 1), 3), dtype=np.uint8)
    lib = lfc.load()
    out, n = C.c_void_p(), C.c_size_t()
    st = lib.lfc_encode(rgb.ctypes.data, C.byref(p.to_c()), C.byref(out), C.byref(n))
    assert st == -1 and out.value is None
    assert lib.lfc_last_error()


def test_encoder_range_error():
    lf = synth.light_field(synth.LFSpec(4, 4, 16, 16, 3, 2.0, 2.0, 4), threads=1)
    with pytest.raises(lfc.LFCError) as e:
        lfc.lfc_encode(lf, lfc.Params(4, 4, 16, 16, 4, 2, (2,), range_mask=1))
    assert e.value.status == -5


def test_null_arguments():
    lib = lfc.load()
    assert lib.lfc_validate(None, 0, None) == -1
    assert lib.lfc_open(None, 0, None, None) == -1
    assert lib.lfc_decode_blocks(None, None, 0, 0, None, None) == -1
    assert lib.lfc_render_views(None, None, 0, 1, 1, None, None) == -1
    assert lib.lfc_info(None, None) == -1
    assert lib.lfc_check(None, None) == -1
    assert lib.lfc_close(None) == 0


@pytest.mark.parametrize("case", [CASES[0], CASES[3], CASES[4], CASES[1]])
def test_encoder_statistics_match_oracle(case):
    U, V, W, H, layers, disp, sigma, kw = case
    lf = synth.light_field(synth.LFSpec(U, V, W, H, layers, disp, sigma, 1000 + U * 7 + W), threads=1)
    ok = dict(grid_u=U, grid_v=V, width=W, height=H, **kw)
    enc = oracle.encode(lf, oracle.Params(**ok))
    stream, st = lfc.lfc_encode_ex(lf, lfc.Params(**ok))
    assert stream == enc.stream and st["stream_bytes"] == len(stream)
    assert abs(st["psnr"] - oracle.psnr(enc.ycocg, enc.r0, W, H)) < 1e-9
    assert st["code_hist"] == list(enc.hist) and st["present_blocks"] == enc.hist.sum()
    none, st2 = lfc.lfc_encode_ex(lf, lfc.Params(**ok), want_stream=False)
    assert none is None and st2 == st


def test_batch_and_server_argument_errors_on_host():
    # checks that come before any device call
    lib = lfc.load()
    assert lib.lfc_batch_render(None, None, 0, None, 1, None, None) == -1
    assert lib.lfc_batch_destroy(None) == 0
    assert lib.lfc_server_destroy(None) == 0
    fake = (C.c_void_p * 1)(1)
    out = C.c_void_p()
    for max_batch, streams, pool in ((0, 1, 1 << 20), (8, 0, 1 << 20), (8, 9, 1 << 20), (8, 1, 16)):
        cfg = lfc.c_server_config(max_batch, streams, pool)
        assert lib.lfc_server_create(fake, 1, C.byref(cfg), C.byref(out)) == -1
    cfg = lfc.c_server_config(8, 1, 1 << 20)
    assert lib.lfc_server_create(None, 1, C.byref(cfg), C.byref(out)) == -1
    assert lib.lfc_server_create(fake, 0, C.byref(cfg), C.byref(out)) == -1
    t = C.c_uint64()
    assert lib.lfc_server_submit(None, None, C.byref(t)) == -1
    assert lib.lfc_server_wait(None, 1, 0, None, None) == -1
    assert lib.lfc_server_release(None, 1) == -1
    assert lib.lfc_server_replay(None, None, None, 0, None) == -1
    assert lib.lfc_server_get_stats(None, None) == -1


def test_render_plan_and_tune_argument_errors_on_host():
    # checks that come before any device call
    lib = lfc.load()
    plan = C.c_void_p(123)
    assert lib.lfc_render_plan_create(None, None, None, 1, 8, 8, None, 1, C.byref(plan)) == -1
    assert plan.value is None   # cleared on failure
    assert lib.lfc_render_plan_create(None, None, None, 1, 8, 8, None, 1, None) == -1
    assert lib.lfc_render_plan_launch(None, None) == -1
    cfg, g = lfc.c_render_config(), C.c_int32()
    assert lib.lfc_render_plan_info(None, C.byref(cfg), C.byref(g)) == -1
    lib.lfc_render_plan_destroy(None)
    res = lfc.c_render_tuning()
    assert lib.lfc_render_tune(None, None, 1, 8, 8, None, 5, C.byref(res), None) == -1
    assert lib.lfc_render_tune(None, None, 1, 8, 8, None, 5, None, None) == -1
    assert lib.lfc_render_views_ex(None, None, 0, 1, 1, None, None, None) == -1


def test_decode_tuner_argument_errors_on_host():
    lib = lfc.load()
    res = lfc.c_decode_tuning()
    assert lib.lfc_tune_decode(None, None, 5, C.byref(res), None) == -1
