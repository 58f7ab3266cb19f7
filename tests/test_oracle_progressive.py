"""Pins of the oracle's progressive decompression (Sec. 3.6: the tree
traversal stopped at a level returns that level's filtered key-view value).

* level 0 is the full traversal (DecompressLFIBlock);
* the top level is the stored key-view block alone;
* coded losslessly (no thresholds, q = 0), the level-k result equals the
  level-k RKV of eq. 2 at the view's ancestor, computed bottom-up from the
  input by the RKV filter (itself pinned against exact rational means);
* a mistake in the stopping rule (one level too many or too few) fails the
  lossless check, since the levels' RKVs differ.
"""
import numpy as np
import pytest

import oracle
from helpers import make_lf

CASES = [
    (9, 9, 24, 16, dict(block=4, levels=3, cluster=(2, 2))),
    (7, 7, 16, 12, dict(block=4, levels=4, cluster=(2, 2, 2))),
    (6, 3, 18, 10, dict(block=2, levels=3, cluster=(2, 2))),
    (5, 4, 24, 16, dict(block=8, levels=2, cluster=(3,))),
]


def params(U, V, W, H, kw, **extra):
    return oracle.Params(grid_u=U, grid_v=V, width=W, height=H, **kw, **extra)


def ancestor_uv(u, v, cluster, k):
    for c in cluster[:k]:
        u, v = u // c, v // c
    return u, v


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-B{c[4]['block']}-L{c[4]['levels']}" for c in CASES])
def test_lossless_levels_equal_the_rkv_tree(case):
    U, V, W, H, kw = case
    rgb = make_lf(U, V, W, H, seed=U + 3 * W)
    p = params(U, V, W, H, kw)
    enc = oracle.encode(rgb, p)
    rkv = oracle.rkv_tree(rgb, p)
    g = oracle.geometry(p)
    B, L = kw["block"], kw["levels"]
    rng = np.random.default_rng(U * W)
    for _ in range(40):
        vi, b = int(rng.integers(U * V)), int(rng.integers(g.nb))
        u, v = vi % U, vi // U
        by, bx = divmod(b, g.nbx)
        for k in range(L):
            got = oracle.decode_block_level(enc.stream, vi, b, k)
            au, av = ancestor_uv(u, v, kw["cluster"], k)
            want = rkv[k][av, au, :, by * B:(by + 1) * B, bx * B:(bx + 1) * B]
            assert np.array_equal(got.astype(np.int32), want), (vi, b, k)


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-B{c[4]['block']}-L{c[4]['levels']}" for c in CASES])
def test_end_levels_equal_full_decode_and_key_view(case):
    U, V, W, H, kw = case
    rgb = make_lf(U, V, W, H, seed=2 * U + W)
    p = params(U, V, W, H, kw, blk_threshold=25, quant_bits=1)
    enc = oracle.encode(rgb, p)
    g = oracle.geometry(p)
    _, root = oracle.tree_tables(p)
    B, L = kw["block"], kw["levels"]
    S = B * B
    hdr_p, hdr_g = oracle.read_header(enc.stream)
    rkv = np.frombuffer(enc.stream, dtype=np.int16, count=g.n_top * g.nb * 3 * S, offset=128)
    rkv = rkv.reshape(g.n_top, g.nb, 3, B, B)
    rng = np.random.default_rng(W)
    for _ in range(40):
        vi, b = int(rng.integers(U * V)), int(rng.integers(g.nb))
        assert np.array_equal(oracle.decode_block_level(enc.stream, vi, b, 0), oracle.decode_block(enc.stream, vi, b))
        assert np.array_equal(oracle.decode_block_level(enc.stream, vi, b, L - 1), rkv[root[vi], b])


def test_bad_level_is_rejected():
    rgb = make_lf(4, 4, 8, 8, seed=1)
    enc = oracle.encode(rgb, params(4, 4, 8, 8, dict(block=4, levels=2, cluster=(2,))))
    with pytest.raises(oracle.OracleError):
        oracle.decode_block_level(enc.stream, 0, 0, 2)
    with pytest.raises(oracle.OracleError):
        oracle.decode_block_level(enc.stream, 0, 0, -1)
