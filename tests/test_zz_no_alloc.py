"""The render entry point that allocates nothing (lfc_render_views_noalloc)
against lfc_render_views_ex, called through the C ABI: two calls in a row on
the same device (the second smaller, so it reads only what it has just
written into the shared static scratch), both render paths, and the refusal
of a forced decode-then-interpolate render whose decoded views exceed the
scratch.  The outputs must be the same bytes (both entry points run the same
kernels), and within 1e-5 of the oracle's render.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from helpers import make_lf, max_abs, oracle_encode, say
from paper_1805_06019_amd import lfc, synth

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _both(lf, views, wo, ho, cfg, disparity=0.0):
    d_views = torch.from_numpy(views).cuda()
    ref = lfc.lfc_render_views(lf, d_views, wo, ho, cfg=cfg, disparity=disparity)
    out = torch.full((views.shape[0], 3, ho, wo), -1.0, dtype=torch.float32, device="cuda")
    got = lfc.lfc_render_views_noalloc(lf, d_views, wo, ho, out, cfg=cfg, disparity=disparity)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


GEOMS = [
    # U, V, W, H, encoding
    (8, 8, 64, 64, dict(block=4, levels=2, cluster=(2,), blk_threshold=2)),
    (5, 4, 72, 24, dict(block=8, levels=2, cluster=(3,), blk_threshold=60, quant_bits=3)),
    (6, 3, 130, 10, dict(block=2, levels=3, cluster=(2, 2), blk_threshold=3)),
]


@pytest.mark.parametrize("path", ["decoded", "auto", "tiles"])
@pytest.mark.parametrize("geom", GEOMS, ids=[f"{g[0]}x{g[1]}x{g[2]}x{g[3]}-B{g[4]['block']}" for g in GEOMS])
def test_noalloc_matches_render_views_ex(gpu, geom, path):
    U, V, W, H, kw = geom
    rgb = make_lf(U, V, W, H, seed=U * 7 + W)
    enc = oracle_encode(rgb, **kw)
    lf = lfc.lfc_open(enc.stream)
    cfg = {"decoded": (lfc.RENDER_DECODED, 0, 0), "tiles": (lfc.RENDER_TILES, 0, 0), "auto": None}[path]
    # two calls in a row, the second with fewer views and a smaller output
    for n, wo, ho, seed in ((24, 96, 80, 1), (5, 40, 30, 2)):
        say("noalloc", (U, V, W, H), path, n, wo, ho)
        views = synth.novel_views(n, U, V, seed=seed, pan=1.0)
        got, ref = _both(lf, views, wo, ho, cfg)
        assert np.array_equal(got, ref)
        assert max_abs(got, oracle.render(enc.r0, U, V, W, H, views, wo, ho)) <= TOL
    # refocused, decoded path
    views = synth.novel_views(7, U, V, seed=3, pan=1.0)
    got, ref = _both(lf, views, 50, 40, cfg, disparity=0.75)
    assert np.array_equal(got, ref)
    lfc.lfc_check(lf)
    lf.close()


def test_noalloc_refuses_oversized_decode_and_falls_back_automatically(gpu):
    # 9x9 views of 512x256: 63.7 MB of decoded int16 views, twice the scratch
    U, V, W, H = 9, 9, 512, 256
    rgb = make_lf(U, V, W, H, seed=11)
    p = lfc.Params(grid_u=U, grid_v=V, width=W, height=H, block=4, levels=2, cluster=(3,), blk_threshold=40,
                   quant_bits=2)
    lf = lfc.lfc_open(lfc.lfc_encode(rgb, p))
    assert U * V * 3 * W * H * 2 > lfc.NOALLOC_SCRATCH_BYTES
    views = synth.novel_views(64, U, V, seed=5, pan=1.0)
    d_views = torch.from_numpy(views).cuda()
    out = torch.zeros((64, 3, 64, 64), dtype=torch.float32, device="cuda")
    say("noalloc refusal", (U, V, W, H))
    with pytest.raises(lfc.LFCError) as ei:
        lfc.lfc_render_views_noalloc(lf, d_views, 64, 64, out, cfg=(lfc.RENDER_DECODED, 0, 0))
    assert ei.value.status == -5 and "scratch" in str(ei.value)
    assert float(out.abs().max()) == 0.0          # nothing was launched
    # automatic: the same bytes as lfc_render_views_ex's tile path
    got = lfc.lfc_render_views_noalloc(lf, d_views, 64, 64, out).cpu().numpy()
    ref = lfc.lfc_render_views(lf, d_views, 64, 64, cfg=(lfc.RENDER_TILES, 0, 0)).cpu().numpy()
    assert np.array_equal(got, ref)
    lf.close()


def test_noalloc_argument_errors(gpu):
    # a too-small output is refused before any launch (an exact-size raw
    # allocation: a torch tensor sits inside a larger caching-allocator
    # segment, and the library sees only the allocation)
    rgb = make_lf(4, 4, 32, 24, seed=2)
    enc = oracle_encode(rgb, block=4, levels=2, cluster=(2,))
    lf = lfc.lfc_open(enc.stream)
    views = torch.from_numpy(synth.novel_views(2, 4, 4, seed=1)).cuda()
    L = lfc.load()
    hip = C.CDLL("libamdhip64.so")
    small = C.c_void_p()
    assert hip.hipMalloc(C.byref(small), C.c_size_t(3 * 8 * 8 * 4)) == 0
    try:
        s = torch.cuda.current_stream().cuda_stream
        assert L.lfc_render_views_noalloc(lf.handle, views.data_ptr(), 2, 8, 8, small.value, None, s) == -1
        assert b"too small" in L.lfc_last_error()
        assert L.lfc_render_views_noalloc(None, views.data_ptr(), 1, 8, 8, small.value, None, s) == -1
        assert L.lfc_render_views_noalloc(lf.handle, views.data_ptr(), 1, 8, 8, small.value, None, s) == 0
        torch.cuda.synchronize()
    finally:
        hip.hipFree(small)
    lf.close()
