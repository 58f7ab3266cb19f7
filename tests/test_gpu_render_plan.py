"""GPU tests of the render's launch shapes, the measured tuner and render
plans captured in HIP graphs.

Every launch shape (decode-then-interpolate, or per-tile footprint decode
with any tile size) computes each output pixel from the same decoded samples
with the same arithmetic, so all of them must give the same bytes as the
automatic choice, which the oracle-parity tests cover to 1e-5 (one case is
re-checked against the oracle here).  A graph replay must equal an eager
render of the views the buffer holds at replay time, on every replay, with
other GPU work and synchronisations between the replays.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import make_lf, max_abs, oracle_encode, say
from paper_1805_06019_amd import lfc, synth

pytestmark = pytest.mark.gpu

FIELDS = [
    # U, V, W, H, encoding, out_w, out_h, views
    (9, 9, 70, 43, dict(block=4, levels=3, cluster=(2, 2), blk_threshold=20, quant_bits=2), 256, 160, 5),
    (6, 3, 130, 10, dict(block=2, levels=3, cluster=(2, 2), blk_threshold=3), 65, 33, 3),
    (5, 4, 72, 24, dict(block=8, levels=2, cluster=(3,), blk_threshold=60, quant_bits=3), 100, 70, 4),
    (8, 8, 64, 64, dict(block=4, levels=2, cluster=(2,), blk_threshold=2), 512, 512, 16),
]
SHAPES = [(lfc.RENDER_DECODED, 0, 0), (lfc.RENDER_TILES, 0, 0), (lfc.RENDER_TILES, 32, 8),
          (lfc.RENDER_TILES, 64, 16), (lfc.RENDER_TILES, 128, 8), (lfc.RENDER_TILES, 17, 5),
          (lfc.RENDER_TILES, 1, 1), (lfc.RENDER_TILES, 256, 2)]


def field(case, seed):
    U, V, W, H, kw, wo, ho, n = case
    enc = oracle_encode(make_lf(U, V, W, H, seed=seed), **kw)
    views = synth.novel_views(n, U, V, seed=seed + 1)
    return enc, lfc.lfc_open(enc.stream), torch.from_numpy(views).cuda(), views


@pytest.mark.parametrize("case", FIELDS, ids=[f"{c[0]}x{c[1]}x{c[2]}x{c[3]}-B{c[4]['block']}" for c in FIELDS])
def test_every_launch_shape_gives_the_same_bytes(gpu, case):
    U, V, W, H, kw, wo, ho, n = case
    enc, lf, views, vnp = field(case, seed=U * 31 + W)
    ref = lfc.lfc_render_views(lf, views, wo, ho)
    for cfg in SHAPES:
        say("shape", case[:4], cfg)
        try:
            got = lfc.lfc_render_views(lf, views, wo, ho, cfg=cfg)
        except lfc.LFCError as e:
            # only an explicit tile whose footprint exceeds the LDS budget may be refused
            assert e.status == -6 and cfg[1] > 0, (cfg, e)
            continue
        assert torch.equal(got, ref), cfg
    if case is FIELDS[0]:
        o = oracle.render(enc.r0, U, V, W, H, vnp, wo, ho)
        assert max_abs(ref.cpu().numpy(), o) <= 1e-5
    lf.close()


def test_launch_shape_errors(gpu):
    case = FIELDS[0]
    _, lf, views, _ = field(case, seed=3)
    for cfg in [(3, 0, 0), (-1, 0, 0), (lfc.RENDER_TILES, 0, 8), (lfc.RENDER_TILES, 2000, 8),
                (lfc.RENDER_TILES, 8, -1)]:
        with pytest.raises(lfc.LFCError) as ei:
            lfc.lfc_render_views(lf, views, 256, 160, cfg=cfg)
        assert ei.value.status == -1, cfg
    # one tile over the whole 256 x 160 output: its footprint (about 21 x 14
    # blocks in 4 views) exceeds 64 KB of LDS
    with pytest.raises(lfc.LFCError) as ei:
        lfc.lfc_render_views(lf, views, 256, 160, cfg=(lfc.RENDER_TILES, 1024, 1024))
    assert ei.value.status == -6
    lf.close()


def test_tuner_times_every_shape_and_leaves_the_result(gpu):
    case = FIELDS[3]
    U, V, W, H, kw, wo, ho, n = case
    _, lf, views, _ = field(case, seed=41)
    ref = lfc.lfc_render_views(lf, views, wo, ho)
    out = torch.zeros_like(ref)
    best, tried = lfc.lfc_render_tune(lf, views, wo, ho, out=out, reps=3)
    say("tuned", best, tried)
    assert len(tried) >= 2 and best in [c for c, _ in tried]
    assert all(ms > 0 for _, ms in tried)
    assert min(tried, key=lambda t: t[1])[0] == best
    assert (lfc.RENDER_DECODED, 0, 0) in [c for c, _ in tried]
    assert torch.equal(out, ref)
    assert torch.equal(lfc.lfc_render_views(lf, views, wo, ho, cfg=best), ref)
    with pytest.raises(lfc.LFCError):
        lfc.lfc_render_tune(lf, views, wo, ho, reps=0)
    lf.close()


@pytest.mark.parametrize("cfg", [None, (lfc.RENDER_DECODED, 0, 0), (lfc.RENDER_TILES, 32, 8)])
def test_graph_plan_replays_match_eager_renders(gpu, cfg):
    case = FIELDS[0]
    U, V, W, H, kw, wo, ho, n = case
    _, lf, views, _ = field(case, seed=57)
    buf = views.clone()
    plan = lfc.RenderPlan(lf, buf, wo, ho, cfg=cfg, graph=True)
    eager_plan = lfc.RenderPlan(lf, buf, wo, ho, cfg=cfg, graph=False)
    shape, graphed = plan.info()
    say("plan", cfg, shape, graphed)
    assert graphed and not eager_plan.info()[1] and shape == eager_plan.info()[0]
    if cfg is not None and cfg[1]:
        assert shape == cfg
    x = torch.randn(512, 512, device="cuda")
    for rep in range(4):
        nv = torch.from_numpy(synth.novel_views(n, U, V, seed=100 + rep)).cuda()
        buf.copy_(nv)
        got = plan.launch().clone()
        y = (x @ x).sum()          # other work on the stream between replays
        torch.cuda.synchronize()
        ref = lfc.lfc_render_views(lf, nv, wo, ho, cfg=cfg)
        assert torch.equal(got, ref), rep
        assert torch.equal(eager_plan.launch(), ref), rep
        assert torch.isfinite(y)
    plan.close()
    eager_plan.close()
    lf.close()


def test_graph_plan_on_a_side_stream(gpu):
    case = FIELDS[1]
    U, V, W, H, kw, wo, ho, n = case
    _, lf, views, _ = field(case, seed=77)
    plan = lfc.RenderPlan(lf, views, wo, ho, graph=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.launch(cuda_stream=side)
    side.synchronize()
    assert torch.equal(plan.out, lfc.lfc_render_views(lf, views, wo, ho))
    plan.close()
    with pytest.raises(lfc.LFCError):
        lfc.RenderPlan(lf, views[:0], wo, ho)
    lf.close()
