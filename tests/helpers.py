"""Shared helpers of the GPU parity tests."""
import sys

import numpy as np

import oracle
from paper_1805_06019_amd import lfc, synth


def say(*a):
    """Names the case before GPU work starts (flushed, so a crash still shows it)."""
    print(*a, flush=True)
    sys.stdout.flush()


def make_lf(U, V, W, H, seed, layers=3, disp=1.5, sigma=2.0, vignetting=False):
    return synth.light_field(synth.LFSpec(U, V, W, H, layers, disp, sigma, seed, vignetting))


def oracle_encode(rgb, **kw):
    V, U, H, W, _ = rgb.shape
    p = oracle.Params(grid_u=U, grid_v=V, width=W, height=H, **kw)
    return oracle.encode(rgb, p)


def blocks_of(planes, B):
    """[nv][3][hp][wp] -> [nv][nb][3][B][B] (block index row-major)."""
    nv, _, hp, wp = planes.shape
    x = planes.reshape(nv, 3, hp // B, B, wp // B, B).transpose(0, 2, 4, 1, 3, 5)
    return np.ascontiguousarray(x.reshape(nv, (hp // B) * (wp // B), 3, B, B))


def max_abs(a, b):
    return float(np.max(np.abs(a.astype(np.float64) - b.astype(np.float64)))) if a.size else 0.0


def strip_stage_words(stream, p):
    """LDS words the whole-field kernel needs to stage each strip (64/B
    blocks of one block row and channel): (groups + pad + directory entries +
    directory rows, bitmaps + entries + directory rows) per strip, read from
    the stream's offsets section and the groups' bitmaps."""
    g = oracle.geometry(p)
    B = p.block
    S, nblk = B * B, 64 // B
    nbw = (g.n_srv + 31) // 32
    o = 128 + g.n_top * g.nb * 3 * S * 2
    off = np.frombuffer(stream, dtype=np.uint32, count=g.ng + 1, offset=o).astype(np.int64)
    srv = np.frombuffer(stream, dtype=np.uint32, offset=o + 4 * (g.ng + 1))
    lens = np.diff(off)
    present = np.array([sum(bin(int(x)).count("1") for x in srv[off[i]:off[i] + nbw]) if lens[i] else 0
                        for i in range(g.ng)], dtype=np.int64)
    lens = lens.reshape(g.nby, g.nbx, 3)
    present = present.reshape(g.nby, g.nbx, 3)
    t1, t2 = [], []
    for by in range(g.nby):
        for bx0 in range(0, g.nbx, nblk):
            for c in range(3):
                w = int(lens[by, bx0:bx0 + nblk, c].sum())
                e = int(present[by, bx0:bx0 + nblk, c].sum())
                t1.append(w + 8 + e + nblk * nbw)
                t2.append(2 * nblk * nbw + e)
    return np.array(t1), np.array(t2)
