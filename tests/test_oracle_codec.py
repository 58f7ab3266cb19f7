"""Pins of the oracle's encoder and decoders (Alg. 1, Alg. 2, Sec. 3.2-3.5).

* the paper's lossless-integer claim (Sec. 4): with every threshold and the
  quantiser off, decode(encode(x)) is the YCoCg-R input exactly, on many
  geometries (odd grids, truncated clusters, ragged images, B = 2/4/8, L = 1..4);
* the closed-loop error bound (eq. 3 with the re-computed RKVs of Sec. 3.2,
  reading C5): the level-0 error depends only on the level-0 step, at any depth;
* decode definitions: the Alg. 2 per-block decoder, the group-wise whole-field
  decoder and the encoder's own reconstruction agree;
* a complete stream derived by hand (tests/golden/tiny_stream.txt);
* the degenerate one-view, one-level tree; the PSNR closed form (eqs. 4-5);
* the paper's rate/quality trend in the block threshold (Figs. 5-6).
"""
import os
import struct

import numpy as np
import pytest

import oracle
from paper_1805_06019_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_stream.txt")


def small_lf(U, V, W, H, seed, layers=3, disp=1.5, sigma=2.0):
    return synth.light_field(synth.LFSpec(U, V, W, H, layers, disp, sigma, seed), threads=1)


GEOMS = [
    # U, V, W, H, B, L, clusters
    (1, 1, 8, 8, 4, 1, ()),
    (1, 1, 5, 7, 2, 1, ()),
    (3, 5, 13, 9, 4, 2, (2,)),
    (8, 8, 16, 16, 4, 2, (2,)),
    (17, 17, 8, 8, 4, 3, (2, 3)),
    (9, 9, 10, 7, 4, 3, (2, 2)),
    (5, 4, 12, 12, 8, 2, (3,)),
    (6, 3, 6, 10, 2, 3, (2, 2)),
    (7, 7, 9, 9, 4, 4, (2, 2, 2)),
    (2, 2, 17, 3, 8, 2, (2,)),
]


@pytest.mark.parametrize("geom", GEOMS)
def test_lossless_at_zero_thresholds(geom):
    U, V, W, H, B, L, cl = geom
    lf = small_lf(U, V, W, H, seed=U * 31 + W)
    p = oracle.Params(U, V, W, H, B, L, cl)
    enc = oracle.encode(lf, p)
    dec = oracle.decode_all(enc.stream)
    assert np.array_equal(dec, enc.ycocg)
    # and the planes really are the YCoCg-R of the input on the W x H area
    ycc = oracle.ycocg_forward(lf.reshape(-1, 3)).reshape(V * U, H, W, 3).transpose(0, 3, 1, 2)
    assert np.array_equal(dec[:, :, :H, :W], ycc)
    # edge replication of the padding
    assert np.array_equal(dec[:, :, H:, :W], np.repeat(ycc[:, :, H - 1:H], dec.shape[2] - H, axis=2))
    assert np.array_equal(dec[:, :, :, W:], np.repeat(dec[:, :, :, W - 1:W], dec.shape[3] - W, axis=3))
    assert oracle.psnr(enc.ycocg, dec, W, H) == 100.0


def _present_leaf_blocks(stream, p, g):
    """(view, block, channel) -> bool: is the level-0 block stored?  Parses the
    stream layout only (bitmap words at each group's start)."""
    _, gg = oracle.read_header(stream)
    rkv_bytes = gg.n_top * gg.nb * 3 * p.block * p.block * 2
    off = np.frombuffer(stream, dtype=np.uint32, count=gg.ng + 1, offset=128 + rkv_bytes)
    srv = np.frombuffer(stream, dtype=np.uint32, offset=128 + rkv_bytes + 4 * (gg.ng + 1))
    path, _ = oracle.tree_tables(p)
    nv = p.grid_u * p.grid_v
    pres = np.zeros((nv, gg.nb, 3), dtype=bool)
    for gi in range(gg.ng):
        if off[gi] == off[gi + 1]:
            continue
        for vi in range(nv):
            s = path[vi, 0]
            pres[vi, gi // 3, gi % 3] = (srv[off[gi] + s // 32] >> (s % 32)) & 1
    return pres


@pytest.mark.parametrize("L,cl", [(2, (2,)), (3, (2, 2)), (4, (2, 2, 2))])
@pytest.mark.parametrize("tp,tb,q", [(0, 40, 0), (3, 20, 0), (0, 30, 2), (4, 60, 3)])
def test_closed_loop_error_bound_independent_of_depth(L, cl, tp, tb, q):
    U = V = 8
    W = H = 16
    B, S = 4, 16
    lf = small_lf(U, V, W, H, seed=77, layers=4, disp=2.0, sigma=3.0)
    p = oracle.Params(U, V, W, H, B, L, cl, tp, tb, q)
    enc = oracle.encode(lf, p)
    dec = oracle.decode_all(enc.stream)
    assert np.array_equal(dec, enc.r0)
    err = (dec.astype(np.int32) - enc.ycocg.astype(np.int32))
    nbx = W // B
    blocks = err.reshape(U * V, 3, H // B, B, nbx, B).transpose(0, 2, 4, 1, 3, 5).reshape(U * V, -1, 3, S)
    pres = _present_leaf_blocks(enc.stream, p, oracle.geometry(p))
    kept_bound = max(tp - 1, (1 << (q - 1)) if q else 0, 0)
    drop_bound = tb + S * max(0, tp - 1)
    absb = np.abs(blocks)
    assert np.all(absb[pres].max(axis=-1) <= kept_bound)
    # absent blocks: either below the energy threshold or quantised to zero
    absent = absb[~pres]
    ok = (absent.sum(axis=-1) <= drop_bound) | (absent.max(axis=-1) <= kept_bound)
    assert np.all(ok)
    assert pres.any() and (~pres).any()


@pytest.mark.parametrize("geom", [GEOMS[2], GEOMS[4], GEOMS[6], GEOMS[7]])
def test_per_block_decoder_matches_whole_field(geom):
    U, V, W, H, B, L, cl = geom
    lf = small_lf(U, V, W, H, seed=5 + U)
    p = oracle.Params(U, V, W, H, B, L, cl, 1, 25, 1)
    enc = oracle.encode(lf, p)
    dec = oracle.decode_all(enc.stream)
    assert np.array_equal(dec, enc.r0)
    g = oracle.geometry(p)
    for vi in range(U * V):
        for b in range(g.nb):
            blk = oracle.decode_block(enc.stream, vi, b)
            by, bx = divmod(b, g.nbx)
            assert np.array_equal(blk, dec[vi, :, by * B:(by + 1) * B, bx * B:(bx + 1) * B])
    # the request loop returns the same blocks in request order
    req = np.array([(vi, b) for vi in range(U * V) for b in range(g.nb)][::-1], dtype=np.int32)
    got = oracle.decode_requests(enc.stream, req)
    for k in range(0, len(req), 7):
        assert np.array_equal(got[k], oracle.decode_block(enc.stream, int(req[k, 0]), int(req[k, 1])))


def test_whole_field_block_ranges_compose():
    lf = small_lf(8, 8, 16, 12, seed=3)
    p = oracle.Params(8, 8, 16, 12, 4, 2, (2,), 0, 10, 0)
    enc = oracle.encode(lf, p)
    full = oracle.decode_all(enc.stream)
    part = np.zeros_like(full)
    g = oracle.geometry(p)
    for b0 in range(0, g.nb, 5):
        oracle.decode_all(enc.stream, b0, min(g.nb, b0 + 5), out=part)
    assert np.array_equal(part, full)


def _read_golden():
    rec = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        k, *vals = line.split()
        rec[k] = vals
    return rec


def test_hand_derived_stream():
    rec = _read_golden()
    lf = np.zeros((1, 2, 4, 4, 3), dtype=np.uint8)
    lf[0, 0] = 100
    lf[0, 1] = 104
    enc = oracle.encode(lf, oracle.Params(2, 1, 4, 4, 4, 2, (2,)))
    s = enc.stream
    assert len(s) == int(rec["total_bytes"][0])
    assert s[:4] == b"RLFC" and struct.unpack_from("<HH", s, 4) == (1, 128)
    words = list(struct.unpack_from("<30I", s, 8))
    assert words == [int(x) for x in rec["header"]]
    rkv = np.frombuffer(s, dtype=np.int16, count=48, offset=128)
    assert np.all(rkv[:16] == int(rec["rkv_y"][0]))
    assert np.all(rkv[16:32] == int(rec["rkv_co"][0])) and np.all(rkv[32:] == int(rec["rkv_cg"][0]))
    assert list(np.frombuffer(s, dtype=np.uint32, count=4, offset=224)) == [int(x) for x in rec["offsets"]]
    assert [int(x) for x in np.frombuffer(s, dtype=np.uint32, offset=240)] == [int(x, 16) for x in rec["srv"]]
    assert list(enc.hist[[1, 19]]) == [1, 1] and enc.hist.sum() == 2
    dec = oracle.decode_all(s)
    assert np.all(dec[0, 0] == 100) and np.all(dec[1, 0] == 104) and not dec[:, 1:].any()


def test_degenerate_single_view_single_level():
    lf = small_lf(1, 1, 12, 12, seed=9)
    p = oracle.Params(1, 1, 12, 12, 4, 1, ())
    enc = oracle.encode(lf, p)
    g = oracle.geometry(p)
    assert g.n_srv == 0 and g.n_top == 1
    rkv_bytes = g.nb * 3 * 16 * 2
    assert len(enc.stream) == 128 + rkv_bytes + 4 * (g.ng + 1) + 8
    off = np.frombuffer(enc.stream, dtype=np.uint32, count=g.ng + 1, offset=128 + rkv_bytes)
    assert not off.any()
    dec = oracle.decode_all(enc.stream)
    assert np.array_equal(dec, enc.ycocg)


def test_stream_layout_invariants():
    lf = small_lf(8, 8, 32, 32, seed=11)
    p = oracle.Params(8, 8, 32, 32, 4, 2, (2,), 0, 60, 1)
    enc = oracle.encode(lf, p)
    _, g = oracle.read_header(enc.stream)
    rkv_bytes = g.n_top * g.nb * 3 * 32
    off = np.frombuffer(enc.stream, dtype=np.uint32, count=g.ng + 1, offset=128 + rkv_bytes)
    srv = np.frombuffer(enc.stream, dtype=np.uint32, offset=128 + rkv_bytes + 4 * (g.ng + 1))
    assert np.all(np.diff(off.astype(np.int64)) >= 0)
    assert srv.size == off[-1] + 2 and not srv[-2:].any()
    nbw = (g.n_srv + 31) // 32
    for gi in range(g.ng):
        n = int(off[gi + 1]) - int(off[gi])
        if n == 0:
            continue
        bm = srv[off[gi]:off[gi] + nbw]
        present = sum(bin(int(x)).count("1") for x in bm)
        assert present > 0
        # high bitmap bits beyond the node count are clear
        assert int(bm[-1]) >> (g.n_srv - 32 * (nbw - 1)) == 0 if g.n_srv % 32 else True
    empty = np.sum(np.diff(off.astype(np.int64)) == 0)
    assert 0 < empty < g.ng


def test_psnr_closed_form():
    ref = np.zeros((2, 3, 4, 4), dtype=np.int16)
    dec = ref.copy()
    dec[:, 0] += 1                      # Y off by one everywhere, chroma exact
    py = 10 * np.log10(255.0 ** 2 / 1.0)
    assert abs(oracle.psnr(ref, dec, 4, 4) - (6 * py + 100 + 100) / 8) < 1e-9
    dec = ref.copy()
    dec[0, 1, :2, :] += 4               # view 0, Co: MSE = 8 on the 4x4 area
    pco = 10 * np.log10(255.0 ** 2 / 8.0)
    expect = ((6 * 100 + pco + 100) / 8 + 100) / 2
    assert abs(oracle.psnr(ref, dec, 4, 4) - expect) < 1e-9
    # only the W x H area counts
    dec = ref.copy()
    dec[:, :, 3, :] = 50
    assert oracle.psnr(ref, dec, 4, 3) == 100.0


def test_rate_and_quality_fall_with_block_threshold():
    lf = small_lf(8, 8, 32, 32, seed=21, layers=4, sigma=2.5)
    bpp, psnr = [], []
    for tb in (0, 8, 24, 64, 160, 400):
        p = oracle.Params(8, 8, 32, 32, 4, 3, (2, 2), 0, tb, 0)
        enc = oracle.encode(lf, p)
        bpp.append(len(enc.stream) * 8 / (64 * 32 * 32))
        psnr.append(oracle.psnr(enc.ycocg, enc.r0, 32, 32))
    assert all(a >= b for a, b in zip(bpp, bpp[1:])), bpp
    assert all(a >= b for a, b in zip(psnr, psnr[1:])), psnr
    assert bpp[0] > bpp[-1] and psnr[0] > psnr[-1]


def test_range_mask_restricts_codes():
    lf = small_lf(4, 4, 16, 16, seed=4)
    only_bits = (1 << 12) - 1
    enc = oracle.encode(lf, oracle.Params(4, 4, 16, 16, 4, 2, (2,), 0, 0, 0, only_bits))
    assert enc.hist[12:].sum() == 0 and enc.hist[:12].sum() > 0
    assert np.array_equal(oracle.decode_all(enc.stream), enc.ycocg)
    with pytest.raises(oracle.OracleError):
        oracle.encode(lf, oracle.Params(4, 4, 16, 16, 4, 2, (2,), 0, 0, 0, 1))  # only N=2


@pytest.mark.parametrize("tb,kept", [(31, True), (32, False), (0, True)])
def test_block_energy_threshold_boundary(tb, kept):
    # Sec. 3.2 keeps a block whose energy is above the threshold (reading C7).
    # In the hand-derived 2x1 example both Y residual blocks are +-2 over 16
    # pixels: energy 32.  At T_blk = 32 both are discarded and every view
    # decodes to the top RKV (Y = 102).
    lf = np.zeros((1, 2, 4, 4, 3), dtype=np.uint8)
    lf[0, 0] = 100
    lf[0, 1] = 104
    enc = oracle.encode(lf, oracle.Params(2, 1, 4, 4, 4, 2, (2,), 0, tb, 0))
    dec = oracle.decode_all(enc.stream)
    if kept:
        assert enc.hist.sum() == 2 and np.all(dec[0, 0] == 100) and np.all(dec[1, 0] == 104)
    else:
        assert enc.hist.sum() == 0 and np.all(dec[:, 0] == 102)
        assert len(enc.stream) == 240 + 8
