"""GPU parity of the fused decode + quadrilinear render (Sec. 3.6) against the
oracle's renderer run on the oracle's decoded light field.

The bar is a maximum absolute error of 1e-5 on RGB/255 outputs: the GPU may
contract multiply-adds, the oracle evaluates every lerp in source order.
Both renderers are covered (footprint decode per output tile, and whole-field
decode followed by per-pixel interpolation) and must agree bit for bit.
Covers magnification and minification (down to one output pixel), ragged tiles, block sizes 2/4/8, a
single-row camera grid, a single view, cameras outside the grid, and the
batched render workload (64 novel 512x512 views per launch on the 8x8x64x64
light field and on the 9x9 lenslet-like 625x434 light field).
"""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from helpers import make_lf, max_abs, oracle_encode, say
from paper_1805_06019_amd import lfc, synth
from paper_1805_06019_amd.workloads import WORKLOADS

pytestmark = pytest.mark.gpu
TOL = 1e-5


PATHS = {"tiles": (lfc.RENDER_TILES, 0, 0), "decoded": (lfc.RENDER_DECODED, 0, 0), "auto": None}


def render_both(enc, U, V, W, H, views, wo, ho, path="auto"):
    lf = lfc.lfc_open(enc.stream)
    got = lfc.lfc_render_views(lf, torch.from_numpy(views).cuda(), wo, ho, cfg=PATHS[path]).cpu().numpy()
    ref = oracle.render(enc.r0, U, V, W, H, views, wo, ho)
    return got, ref


CASES = [
    # U, V, W, H, encoding, out_w, out_h, pan
    (8, 8, 64, 64, dict(block=4, levels=2, cluster=(2,), blk_threshold=2), 512, 512, 1.0),
    (8, 8, 64, 64, dict(block=4, levels=2, cluster=(2,), blk_threshold=2), 37, 29, 3.0),
    (5, 4, 72, 24, dict(block=8, levels=2, cluster=(3,), blk_threshold=60, quant_bits=3), 100, 70, 2.0),
    (6, 3, 130, 10, dict(block=2, levels=3, cluster=(2, 2), blk_threshold=3), 65, 33, 1.0),
    (9, 9, 70, 43, dict(block=4, levels=3, cluster=(2, 2), blk_threshold=20, quant_bits=2), 256, 160, 1.0),
    (9, 1, 40, 30, dict(block=4, levels=2, cluster=(3,)), 41, 31, 0.5),
    (1, 1, 24, 20, dict(block=4, levels=1, cluster=()), 48, 40, 0.5),
    (4, 4, 200, 120, dict(block=4, levels=2, cluster=(2,), blk_threshold=10), 50, 30, 4.0),
    # odd width (padded to 48): the staged source rows reach into the padding
    (5, 5, 45, 27, dict(block=4, levels=2, cluster=(2,), blk_threshold=5), 60, 40, 1.0),
    # strong minification: a whole view into one or a few output pixels
    (4, 4, 200, 120, dict(block=4, levels=2, cluster=(2,), blk_threshold=10), 1, 1, 4.0),
    (6, 3, 130, 10, dict(block=2, levels=3, cluster=(2, 2), blk_threshold=3), 3, 2, 1.0),
]


@pytest.mark.parametrize("path", ["tiles", "decoded"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}x{c[3]}-to-{c[5]}x{c[6]}" for c in CASES])
def test_render_matches_oracle(gpu, case, path):
    # both renderers: footprint decode per output tile, and whole-field decode
    # followed by per-pixel interpolation (chosen by batch size unless forced)
    U, V, W, H, kw, wo, ho, pan = case
    say("render", case, path)
    rgb = make_lf(U, V, W, H, seed=U * 19 + W)
    enc = oracle_encode(rgb, **kw)
    views = synth.novel_views(6, U, V, seed=W + wo, pan=pan)
    views[0] = (0, 0, 0, 0)                       # a corner camera
    views[1] = (U - 1, V - 1, 0.25, -0.5)         # the far corner
    views[2] = (-3.0, V + 2.0, pan, pan)          # outside the grid: clamped
    got, ref = render_both(enc, U, V, W, H, views, wo, ho, path)
    assert max_abs(got, ref) <= TOL


def test_integer_cameras_reproduce_decoded_views(gpu):
    U, V, W, H = 4, 4, 32, 24
    rgb = make_lf(U, V, W, H, seed=8)
    enc = oracle_encode(rgb, block=4, levels=2, cluster=(2,))   # lossless
    views = np.array([[u, v, 0, 0] for v in range(V) for u in range(U)], dtype=np.float32)
    lf = lfc.lfc_open(enc.stream)
    got = lfc.lfc_render_views(lf, torch.from_numpy(views).cuda(), W, H).cpu().numpy()
    expect = rgb.reshape(U * V, H, W, 3).transpose(0, 3, 1, 2).astype(np.float32) / 255.0
    assert max_abs(got, expect) <= TOL


def test_render_argument_errors(gpu):
    rgb = make_lf(2, 2, 8, 8, seed=1)
    enc = oracle_encode(rgb, block=4, levels=2, cluster=(2,))
    lf = lfc.lfc_open(enc.stream)
    lib = lfc.load()
    s = torch.cuda.current_stream().cuda_stream
    views = torch.zeros((2, 4), dtype=torch.float32, device="cuda")
    out = torch.zeros((2, 3, 8, 8), dtype=torch.float32, device="cuda")
    assert lib.lfc_render_views(lf.handle, views.data_ptr(), 2, 0, 8, out.data_ptr(), s) == -1
    assert lib.lfc_render_views(lf.handle, views.data_ptr(), -1, 8, 8, out.data_ptr(), s) == -1
    assert lib.lfc_render_views(lf.handle, views.data_ptr(), 0, 8, 8, out.data_ptr(), s) == 0
    # an output too small for 2 x 3 x 64 x 64 floats: exact-size raw allocation
    hip = C.CDLL("libamdhip64.so")
    small = C.c_void_p()
    assert hip.hipMalloc(C.byref(small), C.c_size_t(2 * 3 * 8 * 8 * 4)) == 0
    try:
        assert lib.lfc_render_views(lf.handle, views.data_ptr(), 2, 64, 64, small.value, s) == -1
        assert lib.lfc_render_views(lf.handle, views.data_ptr(), 2, 8, 8, small.value, s) == 0
    finally:
        torch.cuda.synchronize()
        hip.hipFree(small)
    torch.cuda.synchronize()


def _workload_enc(name):
    w = WORKLOADS[name]
    rgb = synth.light_field(w.spec)
    p = w.params()
    return w, oracle.encode(rgb, oracle.Params(p.grid_u, p.grid_v, p.width, p.height, p.block, p.levels,
                                               p.cluster, p.pix_threshold, p.blk_threshold, p.quant_bits))


@pytest.mark.parametrize("name", ["tiny", "lenslet40"])
def test_batched_render_workload(gpu, name):
    say("batched render", name)
    w, enc = _workload_enc(name)
    s = w.spec
    views = synth.novel_views(64, s.grid_u, s.grid_v, seed=302)
    got, ref = render_both(enc, s.grid_u, s.grid_v, s.width, s.height, views, 512, 512)
    assert max_abs(got, ref) <= TOL


@pytest.mark.parametrize("case", CASES[:5], ids=[f"{c[0]}x{c[1]}x{c[2]}x{c[3]}-to-{c[5]}x{c[6]}" for c in CASES[:5]])
def test_render_paths_are_bit_identical(gpu, case):
    U, V, W, H, kw, wo, ho, pan = case
    rgb = make_lf(U, V, W, H, seed=U * 19 + W)
    enc = oracle_encode(rgb, **kw)
    lf = lfc.lfc_open(enc.stream)
    views = torch.from_numpy(synth.novel_views(9, U, V, seed=W + 7, pan=pan)).cuda()
    outs = []
    for path in ("tiles", "decoded"):
        outs.append(lfc.lfc_render_views(lf, views, wo, ho, cfg=PATHS[path]))
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("path", ["tiles", "decoded"])
@pytest.mark.parametrize("d", [-2.0, 0.7, 3.0])
@pytest.mark.parametrize("case", [CASES[0], CASES[2], CASES[3], CASES[4], CASES[5], CASES[8]],
                         ids=["8x8-512", "B8", "B2", "9x9", "row", "minified"])
def test_refocused_render_matches_oracle(gpu, case, d, path):
    # reading C20: each source view sampled at its own image-plane shift
    U, V, W, H, kw, wo, ho, pan = case
    say("refocus", case[:4], d, path)
    rgb = make_lf(U, V, W, H, seed=U * 19 + W)
    enc = oracle_encode(rgb, **kw)
    lf = lfc.lfc_open(enc.stream)
    views = synth.novel_views(5, U, V, seed=U + W, pan=pan)
    mode = lfc.RENDER_TILES if path == "tiles" else lfc.RENDER_DECODED
    got = lfc.lfc_render_views(lf, torch.from_numpy(views).cuda(), wo, ho, cfg=(mode, 0, 0, d)).cpu().numpy()
    ref = oracle.render(enc.r0, U, V, W, H, views, wo, ho, disparity=d)
    assert max_abs(got, ref) <= TOL
    lf.close()


def test_refocus_on_a_plane_is_sharp_on_the_gpu(gpu):
    # views of one plane moving by 2 pixels per camera step, coded losslessly:
    # focused at d = -2, a camera between grid positions sees the plane's pixels
    U, V, W, H, delta = 4, 4, 64, 40, 2
    r = np.random.default_rng(5)
    base = r.integers(0, 256, (H + delta * (V - 1), W + delta * (U - 1), 3), dtype=np.uint8)
    rgb = np.zeros((V, U, H, W, 3), dtype=np.uint8)
    for j in range(V):
        for i in range(U):
            rgb[j, i] = base[delta * j: delta * j + H, delta * i: delta * i + W]
    enc = oracle_encode(rgb, block=4, levels=2, cluster=(2,))
    lf = lfc.lfc_open(enc.stream)
    u, v = 1.5, 0.5
    views = torch.tensor([[u, v, 0.0, 0.0]], dtype=torch.float32, device="cuda")
    want = base[int(delta * v) + 1: int(delta * v) + H - 1, int(delta * u) + 1: int(delta * u) + W - 1]
    want = want.transpose(2, 0, 1).astype(np.float32) / 255.0
    for mode in (lfc.RENDER_TILES, lfc.RENDER_DECODED):
        got = lfc.lfc_render_views(lf, views, W, H, cfg=(mode, 0, 0, -float(delta)))[0].cpu().numpy()
        assert np.array_equal(got[:, 1:H - 1, 1:W - 1], want), mode
    plan = lfc.RenderPlan(lf, views, W, H, disparity=-float(delta))
    assert np.array_equal(plan.launch()[0].cpu().numpy()[:, 1:H - 1, 1:W - 1], want)
    plan.close()
    with pytest.raises(lfc.LFCError):
        lfc.lfc_render_views(lf, views, W, H, disparity=float("nan"))
    lf.close()


def test_refocused_64_view_batch_on_lenslet40(gpu):
    # the full-size batch (64 novel 512x512 views of the 9x9 lenslet-like field),
    # refocused, in the launch shape the automatic choice takes (decode then
    # interpolate) and in tiles (the same bytes: both compute each sample
    # position with the same roundings); the oracle renders 4 of the views
    say("refocused batch lenslet40")
    w, enc = _workload_enc("lenslet40")
    s = w.spec
    lf = lfc.lfc_open(enc.stream)
    views = synth.novel_views(64, s.grid_u, s.grid_v, seed=303)
    tv = torch.from_numpy(views).cuda()
    auto = lfc.lfc_render_views(lf, tv, 512, 512, disparity=0.8)
    tiles = lfc.lfc_render_views(lf, tv, 512, 512, cfg=(lfc.RENDER_TILES, 0, 0, 0.8))
    assert torch.equal(auto, tiles)
    pick = [0, 17, 40, 63]
    ref = oracle.render(enc.r0, s.grid_u, s.grid_v, s.width, s.height, views[pick], 512, 512, disparity=0.8)
    assert max_abs(auto[pick].cpu().numpy(), ref) <= TOL
    lf.close()
