"""GPU parity of the decode path (Alg. 2 batched, Sec. 3.5-3.6) against the oracle.

Bit-exact: every decoded int16 sample equals the oracle's closed-loop
reconstruction R^0, which its own decoders reproduce (pinned in
test_oracle_codec.py).  Covers the whole-field kernel (images layout), the
random-access kernel (blocks layout, all blocks or a request list), ragged
images, block sizes 2/4/8, tree heights 1-6, every range code of each kind
(plain bits, trits, quints) that 8-bit views reach, empty and out-of-range requests,
the staging tiers of the whole-field kernel, progressive decompression at
every tree level (Sec. 3.6), and the full 17x17x512x512 workload in the
launch configuration the benchmark times.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from helpers import blocks_of, make_lf, oracle_encode, say
from paper_1805_06019_amd import lfc, synth
from paper_1805_06019_amd.workloads import WORKLOADS

pytestmark = pytest.mark.gpu

GEOMS = [
    # U, V, W, H, encoding parameters
    (8, 8, 64, 64, dict(block=4, levels=2, cluster=(2,), blk_threshold=2)),
    (1, 1, 12, 10, dict(block=4, levels=1, cluster=())),
    (3, 5, 13, 9, dict(block=4, levels=2, cluster=(2,))),
    (17, 17, 20, 12, dict(block=4, levels=3, cluster=(2, 3), blk_threshold=30, quant_bits=1)),
    (9, 9, 70, 43, dict(block=4, levels=3, cluster=(2, 2), pix_threshold=2, blk_threshold=20, quant_bits=2)),
    (5, 4, 72, 24, dict(block=8, levels=2, cluster=(3,), blk_threshold=60, quant_bits=3)),
    (6, 3, 130, 10, dict(block=2, levels=3, cluster=(2, 2), pix_threshold=1, blk_threshold=3)),
    (7, 7, 33, 17, dict(block=4, levels=4, cluster=(2, 2, 2), quant_bits=4, blk_threshold=10)),
    (4, 4, 150, 8, dict(block=4, levels=2, cluster=(2,), range_mask=0x3F80000 | 0x7F000 | (0xF << 8))),
    (2, 3, 64, 64, dict(block=4, levels=6, cluster=(2, 2, 2, 2, 2))),
]


def gpu_open(stream):
    return lfc.lfc_open(stream)


def oracle_rgb_words(r0):
    """The oracle's reconstruction [nv][3][hp][wp] (Y, Co, Cg) as the colour
    decode's pixel words: inverse YCoCg-R clamped to 8 bits, R | G << 8 | B << 16."""
    rgb = oracle.ycocg_inverse(np.ascontiguousarray(np.transpose(r0, (0, 2, 3, 1)))).astype(np.uint32)
    return (rgb[..., 0] | (rgb[..., 1] << 8) | (rgb[..., 2] << 16)).view(np.int32)


@pytest.mark.parametrize("case", GEOMS, ids=[f"{c[0]}x{c[1]}x{c[2]}x{c[3]}-B{c[4]['block']}-L{c[4]['levels']}"
                                             for c in GEOMS])
def test_whole_field_rgb(gpu, case):
    # every view as 8-bit RGB: the colour whole-field kernel (strips of all
    # three channels) against the oracle's reconstruction and colour transform
    U, V, W, H, kw = case
    say("rgb", case)
    rgb = make_lf(U, V, W, H, seed=U * 13 + W)
    enc = oracle_encode(rgb, **kw)
    lf = gpu_open(enc.stream)
    got = lfc.lfc_decode_rgb(lf).cpu().numpy()
    assert np.array_equal(got, oracle_rgb_words(enc.r0))
    # the unpadded part is the light field's own colour image of the reconstruction
    lf.close()


@pytest.mark.parametrize("case", GEOMS, ids=[f"{c[0]}x{c[1]}x{c[2]}x{c[3]}-B{c[4]['block']}-L{c[4]['levels']}"
                                             for c in GEOMS])
def test_whole_field_images_layout(gpu, case):
    U, V, W, H, kw = case
    say("images", case)
    rgb = make_lf(U, V, W, H, seed=U * 13 + W)
    enc = oracle_encode(rgb, **kw)
    lf = gpu_open(enc.stream)
    out = lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_IMAGES)
    got = out.cpu().numpy()
    assert np.array_equal(got, enc.r0)
    lfc.lfc_check(lf)
    # repeatable: a second run is bit-identical
    out2 = lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_IMAGES)
    assert torch.equal(out, out2)


# Range codes restricted to one kind (Sec. 3.3: plain bits, trits, quints),
# on light fields whose residuals reach the largest codes of the kind: views
# of uniform noise of a given amplitude (and the smooth synthetic field for
# the small codes), with the quantiser shift q.  Per kind: the noise
# amplitudes and shifts used, and the code every block size must reach.
KIND_CASES = {
    "plain": ((1 << 12) - 1, [(64, 0), (256, 0), (0, 0)], 8),
    "trit": (0x7F000, [(64, 0), (128, 1), (256, 2), (0, 0)], 18),
    "quint": (0x3F80000, [(64, 0), (128, 0), (256, 1), (0, 0)], 25),
}


@pytest.mark.parametrize("B", [2, 4, 8])
@pytest.mark.parametrize("kind", list(KIND_CASES))
def test_every_range_code_of_a_kind(gpu, kind, B):
    # the whole-field kernel, the colour kernel and random access against the
    # oracle, block by block, with every code of the kind that 8-bit views
    # reach: trits and quints up to m = 6, plain bits up to m = 10 (over 32
    # bits per row at B = 4)
    mask, configs, top = KIND_CASES[kind]
    rs = np.random.default_rng(1000 + B)
    seen = set()
    for amp, q in configs:
        say("kind", kind, "B", B, "noise", amp, "q", q)
        if amp:
            rgb = (rs.integers(0, amp, size=(3, 3, 40, 48, 3)) + (128 - amp // 2)).clip(0, 255).astype(np.uint8)
        else:
            rgb = make_lf(3, 3, 48, 40, seed=7, sigma=2.0)
        enc = oracle_encode(rgb, block=B, levels=2, cluster=(2,), range_mask=mask, quant_bits=q)
        seen |= {c for c in range(26) if enc.hist[c]}
        lf = gpu_open(enc.stream)
        assert np.array_equal(lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_IMAGES).cpu().numpy(), enc.r0)
        assert np.array_equal(lfc.lfc_decode_rgb(lf).cpu().numpy(), oracle_rgb_words(enc.r0))
        allb = lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_BLOCKS).cpu().numpy()
        assert np.array_equal(allb, blocks_of(enc.r0, B).reshape(-1, 3, B, B))
        lfc.lfc_check(lf)
        lf.close()
    lo, hi = {"plain": (0, 11), "trit": (12, 18), "quint": (19, 25)}[kind]
    assert seen and min(seen) >= lo and max(seen) <= hi
    assert top in seen, (kind, B, sorted(seen))


@pytest.mark.parametrize("tiers", ["global", "no-payload", "mixed", "as-needed"])
@pytest.mark.parametrize("case", [GEOMS[0], GEOMS[3], GEOMS[5], GEOMS[6]],
                         ids=["8x8x64x64-B4-L2", "17x17x20x12-B4-L3", "5x4x72x24-B8-L2", "6x3x130x10-B2-L3"])
def test_whole_field_staging_tiers(gpu, case, tiers):
    # stage_cap_words bounds the LDS the whole-field kernel may use to
    # stage a strip: 0 reads everything from global memory; a cap that holds
    # the schedule but not the payload of most strips stages the schedule
    # only; the median strip's full need mixes the tiers in one launch; -1
    # stages what each strip needs within the workgroup's LDS budget
    U, V, W, H, kw = case
    rgb = make_lf(U, V, W, H, seed=U * 13 + W)
    enc = oracle_encode(rgb, **kw)
    lf = gpu_open(enc.stream)
    need = lfc.lfc_stage_needs(lf).astype(np.int64)
    t1, t2 = need[:, 0] + 8, need[:, 1]
    if tiers == "global":
        cap = 0
    elif tiers == "no-payload":
        # the cap that puts the most strips in the middle tier
        cap = max((int(c) for c in t2), key=lambda c: int(np.sum((t2 <= c) & (t1 > c))))
        assert np.sum((t2 <= cap) & (t1 > cap)) > 0
    elif tiers == "mixed":
        cap = int(np.median(t1))
    else:
        cap = -1
    say("images staging", case, tiers, cap)
    got = lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_IMAGES, stage_cap_words=cap).cpu().numpy()
    assert np.array_equal(got, enc.r0)


@pytest.mark.parametrize("case", GEOMS[:8], ids=[f"{c[0]}x{c[1]}x{c[2]}x{c[3]}-B{c[4]['block']}-L{c[4]['levels']}"
                                                 for c in GEOMS[:8]])
def test_random_access_blocks_layout(gpu, case):
    U, V, W, H, kw = case
    say("blocks", case)
    rgb = make_lf(U, V, W, H, seed=U * 17 + H)
    enc = oracle_encode(rgb, **kw)
    g = oracle.geometry(oracle.Params(U, V, W, H, kw["block"], kw["levels"], kw["cluster"]))
    expect = blocks_of(enc.r0, kw["block"])
    lf = gpu_open(enc.stream)
    # every block, canonical order
    allb = lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_BLOCKS).cpu().numpy()
    assert np.array_equal(allb, expect.reshape(-1, 3, kw["block"], kw["block"]))
    # a random request list that includes the first and the last (padded) block
    req = synth.block_requests(3001, U * V, g.nb, seed=7)
    req[0] = (0, 0)
    req[1] = (U * V - 1, g.nb - 1)
    req_d = torch.from_numpy(req).cuda()
    got = lfc.lfc_decode_blocks(lf, req_d, lfc.LAYOUT_BLOCKS).cpu().numpy()
    assert np.array_equal(got, expect[req[:, 0], req[:, 1]])
    # the literal Alg. 2 decoder on a sample
    for k in range(20):
        vi, b = int(req[k, 0]), int(req[k, 1])
        assert np.array_equal(got[k], oracle.decode_block(enc.stream, vi, b))
    lfc.lfc_check(lf)


def test_out_of_range_requests_raise_flag(gpu):
    rgb = make_lf(4, 4, 16, 16, seed=3)
    enc = oracle_encode(rgb, block=4, levels=2, cluster=(2,), blk_threshold=5)
    lf = gpu_open(enc.stream)
    nb = 16
    req = np.array([[0, 0], [-1, 3], [5, nb], [16, 0], [15, nb - 1], [2, -7]], dtype=np.int32)
    got = lfc.lfc_decode_blocks(lf, torch.from_numpy(req).cuda(), lfc.LAYOUT_BLOCKS).cpu().numpy()
    expect = blocks_of(enc.r0, 4)
    assert np.array_equal(got[0], expect[0, 0]) and np.array_equal(got[4], expect[15, nb - 1])
    assert not got[[1, 2, 3, 5]].any()
    with pytest.raises(lfc.LFCError) as e:
        lfc.lfc_check(lf)
    assert e.value.status == -1
    lfc.lfc_check(lf)  # the flag was cleared


def test_empty_request_list_and_argument_errors(gpu):
    rgb = make_lf(4, 4, 16, 16, seed=4)
    enc = oracle_encode(rgb, block=4, levels=2, cluster=(2,))
    lf = gpu_open(enc.stream)
    empty = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    out = lfc.lfc_decode_blocks(lf, empty, lfc.LAYOUT_BLOCKS)
    assert out.shape == (0, 3, 4, 4)
    lib = lfc.load()
    s = torch.cuda.current_stream().cuda_stream
    # output too small for the whole field: an exact-size raw allocation (a
    # small torch tensor lives inside a larger caching-allocator segment, and
    # the library can only see the allocation that holds the pointer)
    hip = C.CDLL("libamdhip64.so")
    small = C.c_void_p()
    assert hip.hipMalloc(C.byref(small), C.c_size_t(4096)) == 0
    try:
        assert lib.lfc_decode_blocks(lf.handle, None, 16, lfc.LAYOUT_IMAGES, small.value, s) == -1
        assert lib.lfc_decode_blocks(lf.handle, None, 16 * 16, lfc.LAYOUT_BLOCKS, small.value, s) == -1
        assert lib.lfc_decode_rgb(lf.handle, small.value, s) == -1   # 16 views of 16 x 16 words need 16 KB
    finally:
        hip.hipFree(small)
    # wrong count for the images layout, unknown layout, host pointer as output
    big = torch.zeros(16 * 3 * 16 * 16, dtype=torch.int16, device="cuda")
    assert lib.lfc_decode_blocks(lf.handle, None, 15, lfc.LAYOUT_IMAGES, big.data_ptr(), s) == -1
    assert lib.lfc_decode_blocks(lf.handle, None, 16, 7, big.data_ptr(), s) == -1
    host = np.zeros(16 * 3 * 16 * 16, dtype=np.int16)
    assert lib.lfc_decode_blocks(lf.handle, None, 16, lfc.LAYOUT_IMAGES, host.ctypes.data, s) == -1
    assert lib.lfc_decode_rgb(lf.handle, host.ctypes.data, s) == -1
    assert lib.lfc_decode_rgb(None, big.data_ptr(), s) == -1
    # a corrupt stream never reaches the device
    with pytest.raises(lfc.LFCError) as e:
        lfc.lfc_open(enc.stream[:-4])
    assert e.value.status == -2
    torch.cuda.synchronize()


def test_tiny_workload_whole_field(gpu):
    w = WORKLOADS["tiny"]
    say("tiny workload")
    rgb = synth.light_field(w.spec)
    enc = oracle.encode(rgb, oracle.Params(8, 8, 64, 64, 4, 2, (2,), 0, 2, 0))
    lf = gpu_open(enc.stream)
    got = lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_IMAGES).cpu().numpy()
    assert np.array_equal(got, enc.r0)
    assert np.array_equal(got, oracle.decode_all(enc.stream))


@pytest.fixture(scope="module")
def full_rgb():
    say("full: generating the 17x17x512x512 light field")
    return synth.light_field(WORKLOADS["full40"].spec)


def _oracle_workload(name, rgb):
    w = WORKLOADS[name]
    say(f"{name}: encoding with the oracle")
    p = w.params()
    enc = oracle.encode(rgb, oracle.Params(p.grid_u, p.grid_v, p.width, p.height, p.block, p.levels,
                                           p.cluster, p.pix_threshold, p.blk_threshold, p.quant_bits))
    return w, rgb, enc


@pytest.fixture(scope="module")
def full40(full_rgb):
    return _oracle_workload("full40", full_rgb)


@pytest.fixture(scope="module")
def full50(full_rgb):
    return _oracle_workload("full50", full_rgb)


def test_full_size_whole_field_and_random_access(gpu, full40):
    w, rgb, enc = full40
    say("full40: whole field on the GPU")
    lf = gpu_open(enc.stream)
    out = lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_IMAGES)
    got = out.cpu().numpy()
    assert np.array_equal(got, enc.r0)
    del out
    # the literal Alg. 2 decoder on sampled (view, block) pairs
    nb = lf.info.n_blocks
    req = synth.block_requests(1_000_000, 289, nb, seed=202)
    for vi, b in req[:64]:
        by, bx = divmod(int(b), 128)
        assert np.array_equal(got[vi, :, by * 4:by * 4 + 4, bx * 4:bx * 4 + 4], oracle.decode_block(enc.stream, int(vi), int(b)))
    say("full40: 10^6 random block accesses on the GPU")
    blk = lfc.lfc_decode_blocks(lf, torch.from_numpy(req).cuda(), lfc.LAYOUT_BLOCKS).cpu().numpy()
    expect = blocks_of(enc.r0, 4)
    assert np.array_equal(blk, expect[req[:, 0], req[:, 1]])
    del blk, expect
    say("full40: every view as 8-bit RGB")
    assert np.array_equal(lfc.lfc_decode_rgb(lf).cpu().numpy(), oracle_rgb_words(enc.r0))
    lfc.lfc_check(lf)


def test_full50_whole_field_and_random_access(gpu, full50):
    # the 50 dB coding of the same light field (more stored blocks per strip,
    # more chunks, mostly schedule-only staging), at the tile capacity the
    # tuner keeps, as the benchmark decodes it
    w, rgb, enc = full50
    lf = gpu_open(enc.stream)
    say("full50: tuning the whole-field decode")
    best, tried = lfc.lfc_tune_decode(lf, reps=2)
    say("tried", tried, "kept", best)
    say("full50: whole field on the GPU")
    out = lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_IMAGES)
    got = out.cpu().numpy()
    assert np.array_equal(got, enc.r0)
    del out
    nb = lf.info.n_blocks
    req = synth.block_requests(1_000_000, 289, nb, seed=202)
    for vi, b in req[:64]:
        by, bx = divmod(int(b), 128)
        assert np.array_equal(got[vi, :, by * 4:by * 4 + 4, bx * 4:bx * 4 + 4],
                              oracle.decode_block(enc.stream, int(vi), int(b)))
    del got
    say("full50: 10^6 random block accesses on the GPU")
    blk = lfc.lfc_decode_blocks(lf, torch.from_numpy(req).cuda(), lfc.LAYOUT_BLOCKS).cpu().numpy()
    expect = blocks_of(enc.r0, 4)
    assert np.array_equal(blk, expect[req[:, 0], req[:, 1]])
    lfc.lfc_check(lf)
    lf.close()


@pytest.mark.parametrize("case", GEOMS[:8], ids=[f"{c[0]}x{c[1]}x{c[2]}x{c[3]}-B{c[4]['block']}-L{c[4]['levels']}"
                                                 for c in GEOMS[:8]])
def test_progressive_decode_matches_oracle(gpu, case):
    # Sec. 3.6: the traversal stopped at level k, every level of the tree
    U, V, W, H, kw = case
    say("progressive", case)
    rgb = make_lf(U, V, W, H, seed=U * 13 + W)
    enc = oracle_encode(rgb, **kw)
    lf = gpu_open(enc.stream)
    nv, nb = U * V, lf.info.n_blocks
    req = synth.block_requests(64, nv, nb, seed=U + W)
    dreq = torch.from_numpy(req).cuda()
    full = lfc.lfc_decode_blocks(lf, dreq, lfc.LAYOUT_BLOCKS)
    for k in range(kw["levels"]):
        got = lfc.lfc_decode_progressive(lf, dreq, k).cpu().numpy()
        want = np.stack([oracle.decode_block_level(enc.stream, int(v), int(b), k) for v, b in req])
        assert np.array_equal(got, want), k
        if k == 0:
            assert np.array_equal(got, full.cpu().numpy())
    lfc.lfc_check(lf)


def test_full_size_render_paths_agree(gpu, full40):
    # 64 views of 512^2: the decode-then-interpolate path decodes full40 into
    # 454.6 MB of scratch, more than the Infinity Cache, so that decode streams
    # its output with the non-temporal hint; the tile path decodes footprints
    w, _, enc = full40
    s = w.spec
    lf = gpu_open(enc.stream)
    views = torch.from_numpy(synth.novel_views(64, s.grid_u, s.grid_v, seed=303)).cuda()
    outs = []
    for path in ("decoded", "tiles"):
        say("full40: 64-view render,", path)
        cfg = (lfc.RENDER_DECODED, 0, 0) if path == "decoded" else (lfc.RENDER_TILES, 0, 0)
        outs.append(lfc.lfc_render_views(lf, views, 512, 512, cfg=cfg))
    assert torch.equal(outs[0], outs[1])
    ref = oracle.render(enc.r0, s.grid_u, s.grid_v, s.width, s.height, views[:2].cpu().numpy(), 512, 512)
    assert np.abs(outs[0][:2].cpu().numpy() - ref).max() <= 1e-5


def test_largest_light_field_of_the_workloads(gpu):
    # 17 x 17 views of 1024 x 1024 (the serving mix's largest light fields):
    # 909 M samples, a 1.8 GB decode; whole field, random access and two
    # novel views against the oracle's encoder, reconstruction and renderer
    w = WORKLOADS["serve_large40"]
    s = w.spec
    say("serve_large40: generating")
    rgb = synth.light_field(s)
    say("serve_large40: encoding with the oracle")
    p = w.params()
    enc = oracle.encode(rgb, oracle.Params(p.grid_u, p.grid_v, p.width, p.height, p.block, p.levels,
                                           p.cluster, p.pix_threshold, p.blk_threshold, p.quant_bits))
    del rgb
    lf = gpu_open(enc.stream)
    say("serve_large40: whole field on the GPU")
    out = lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_IMAGES)
    assert np.array_equal(out.cpu().numpy(), enc.r0)
    del out
    say("serve_large40: random access")
    nb = lf.info.n_blocks
    req = synth.block_requests(4096, s.grid_u * s.grid_v, nb, seed=404)
    got = lfc.lfc_decode_blocks(lf, torch.from_numpy(req).cuda(), lfc.LAYOUT_BLOCKS).cpu().numpy()
    nbx = (s.width + 3) // 4
    for (vi, b), blk in zip(req, got):
        by, bx = divmod(int(b), nbx)
        assert np.array_equal(blk, enc.r0[vi, :, by * 4:by * 4 + 4, bx * 4:bx * 4 + 4])
    say("serve_large40: two novel views at 512^2 and two at 1024^2")
    views = synth.novel_views(2, s.grid_u, s.grid_v, seed=405)
    img = lfc.lfc_render_views(lf, torch.from_numpy(views).cuda(), 512, 512).cpu().numpy()
    ref = oracle.render(enc.r0, s.grid_u, s.grid_v, s.width, s.height, views, 512, 512)
    assert np.abs(img - ref).max() <= 1e-5
    views = synth.novel_views(2, s.grid_u, s.grid_v, seed=406)
    for path in (lfc.RENDER_TILES, lfc.RENDER_DECODED):
        img = lfc.lfc_render_views(lf, torch.from_numpy(views).cuda(), 1024, 1024, cfg=(path, 0, 0)).cpu().numpy()
        ref = oracle.render(enc.r0, s.grid_u, s.grid_v, s.width, s.height, views, 1024, 1024)
        assert np.abs(img - ref).max() <= 1e-5, path


def test_progressive_decode_full_size_and_errors(gpu, full40):
    _, _, enc = full40
    lf = gpu_open(enc.stream)
    nv, nb = 289, lf.info.n_blocks
    req = synth.block_requests(100_000, nv, nb, seed=303)
    dreq = torch.from_numpy(req).cuda()
    got = lfc.lfc_decode_progressive(lf, dreq, 1).cpu().numpy()
    for i in np.random.default_rng(5).integers(0, len(req), 100):
        assert np.array_equal(got[i], oracle.decode_block_level(enc.stream, int(req[i, 0]), int(req[i, 1]), 1))
    lib = lfc.load()
    s = torch.cuda.current_stream().cuda_stream
    out = torch.empty((4, 3, 4, 4), dtype=torch.int16, device="cuda")
    assert lib.lfc_decode_progressive(lf.handle, dreq.data_ptr(), 4, 3, out.data_ptr(), s) == -1
    assert lib.lfc_decode_progressive(lf.handle, dreq.data_ptr(), 4, -1, out.data_ptr(), s) == -1
    assert lib.lfc_decode_progressive(lf.handle, dreq.data_ptr(), 0, 2, out.data_ptr(), s) == 0
    lfc.lfc_check(lf)


@pytest.mark.parametrize("case", [GEOMS[0], GEOMS[3], GEOMS[5], GEOMS[6], GEOMS[7], GEOMS[1]],
                         ids=["8x8-B4", "17x17-L3", "B8", "B2", "L4", "L1"])
def test_decode_tuner_keeps_the_output(gpu, case):
    # every tile capacity decodes the same samples; the tuner keeps one of
    # those it timed, and a second tuning replaces the first one's tables
    U, V, W, H, kw = case
    say("tune decode", case)
    rgb = make_lf(U, V, W, H, seed=U * 13 + W)
    enc = oracle_encode(rgb, **kw)
    lf = gpu_open(enc.stream)
    n_strips = lfc.lfc_stage_needs(lf).shape[0]
    for _ in range(2):
        best, tried = lfc.lfc_tune_decode_ex(lf, reps=2)
        say("tried", tried, "kept", best)
        assert best in [(c, st) for c, st, _ in tried] and all(ms > 0 for _, _, ms in tried)
        # every capacity is timed with and without staging
        assert sorted(st for _, st, _ in tried) == [False, True] * (len(tried) // 2) or \
            sum(st for _, st, _ in tried) * 2 == len(tried)
        if kw["levels"] >= 2:
            assert len(tried) >= 4
        assert lfc.lfc_stage_needs(lf).shape[0] == n_strips
        got = lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_IMAGES).cpu().numpy()
        assert np.array_equal(got, enc.r0)
    lfc.lfc_check(lf)
    lf.close()


@pytest.mark.parametrize("case", [GEOMS[0], GEOMS[3], GEOMS[5], GEOMS[6], GEOMS[7]],
                         ids=["8x8-B4", "17x17-L3", "B8", "B2", "L4"])
def test_rgb_tuner_keeps_the_output(gpu, case):
    # the colour kernel's tile capacity: every capacity the tuner times gives
    # the oracle's RGB words, and a decode-then-interpolate render gives the
    # same bytes before and after; a second tuning replaces the first's tables
    U, V, W, H, kw = case
    say("tune rgb", case)
    rgb = make_lf(U, V, W, H, seed=U * 13 + W)
    enc = oracle_encode(rgb, **kw)
    lf = gpu_open(enc.stream)
    want = oracle_rgb_words(enc.r0)
    views = torch.from_numpy(synth.novel_views(6, U, V, seed=U + 5)).cuda()
    before = lfc.lfc_render_views(lf, views, 40, 30, cfg=(lfc.RENDER_DECODED, 0, 0, 0.0))
    for _ in range(2):
        best, tried = lfc.lfc_tune_decode_rgb(lf, reps=2)
        say("tried", tried, "kept", best)
        assert best in [c for c, _ in tried] and all(ms > 0 for _, ms in tried) and len(tried) >= 3
        assert np.array_equal(lfc.lfc_decode_rgb(lf).cpu().numpy(), want)
        after = lfc.lfc_render_views(lf, views, 40, 30, cfg=(lfc.RENDER_DECODED, 0, 0, 0.0))
        assert torch.equal(before, after)
    lf.close()


def test_rgb_tuner_errors(gpu):
    U, V, W, H, kw = GEOMS[1]
    assert kw["levels"] == 1
    lf = gpu_open(oracle_encode(make_lf(U, V, W, H, seed=3), **kw).stream)
    with pytest.raises(lfc.LFCError):
        lfc.lfc_tune_decode_rgb(lf, reps=2)
    lf.close()


def test_decode_tuner_on_full40(gpu, full40):
    w, rgb, enc = full40
    say("full40: tuning the whole-field decode")
    lf = gpu_open(enc.stream)
    best, tried = lfc.lfc_tune_decode(lf, reps=3)
    say("tried", tried, "kept", best)
    got = lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_IMAGES).cpu().numpy()
    assert np.array_equal(got, enc.r0)
    lf.close()
