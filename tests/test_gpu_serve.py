"""GPU tests of batched rendering across light fields and of the serving loop.

A batched request must give exactly the bytes that lfc_render_views gives
for it alone (the same tile code runs, only the launch is shared), and
through it the oracle's renderer to 1e-5.  The server must return every
request's result unchanged whatever it is batched with, including when the
output pool admits only a few results at a time.  Batched random access over
several light fields must equal each light field's own decode.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from helpers import make_lf, max_abs, oracle_encode, say
from paper_1805_06019_amd import lfc, synth

pytestmark = pytest.mark.gpu

FIELDS = [
    # U, V, W, H, encoding
    (8, 8, 64, 64, dict(block=4, levels=2, cluster=(2,), blk_threshold=2)),
    (6, 3, 130, 10, dict(block=2, levels=3, cluster=(2, 2), blk_threshold=3)),
    (5, 4, 72, 24, dict(block=8, levels=2, cluster=(3,), blk_threshold=60, quant_bits=3)),
    (9, 9, 70, 43, dict(block=4, levels=3, cluster=(2, 2), blk_threshold=20, quant_bits=2)),
]


@pytest.fixture(scope="module")
def fields(gpu):
    encs, lfs = [], []
    for U, V, W, H, kw in FIELDS:
        enc = oracle_encode(make_lf(U, V, W, H, seed=U * 7 + W), **kw)
        encs.append(enc)
        lfs.append(lfc.lfc_open(enc.stream))
    yield encs, lfs
    for lf in lfs:
        lf.close()


def mixed_requests(n, seed):
    rng = np.random.default_rng(seed)
    sizes = [(64, 64), (37, 29), (128, 96), (1, 1), (200, 50)]
    reqs = []
    for _ in range(n):
        li = int(rng.integers(len(FIELDS)))
        U, V = FIELDS[li][0], FIELDS[li][1]
        w, h = sizes[int(rng.integers(len(sizes)))]
        view = (rng.uniform(-0.5, U - 0.5), rng.uniform(-0.5, V - 0.5), rng.uniform(-2, 2), rng.uniform(-2, 2))
        reqs.append((li, w, h, view))
    return reqs


def single(lfs, req):
    li, w, h, v = req
    views = torch.tensor([v], dtype=torch.float32, device="cuda")
    return lfc.lfc_render_views(lfs[li], views, w, h)[0]


def test_batch_matches_single_renders_and_oracle(fields):
    encs, lfs = fields
    reqs = mixed_requests(24, seed=5)
    say("batch", len(reqs), "requests over", len(lfs), "light fields")
    b = lfc.Batch()
    outs = b.render(lfs, reqs)
    for r, o in zip(reqs, outs):
        assert torch.equal(o, single(lfs, r)), r
    # a few of them against the oracle's renderer
    for r, o in list(zip(reqs, outs))[:6]:
        li, w, h, v = r
        U, V, W, H, _ = FIELDS[li]
        ref = oracle.render(encs[li].r0, U, V, W, H, np.array([v], dtype=np.float32), w, h)[0]
        assert max_abs(o.cpu().numpy(), ref) <= 1e-5
    # two more calls on the same context, one larger than any before (staging grows)
    more = mixed_requests(300, seed=6)
    outs2 = b.render(lfs, more)
    outs3 = b.render(lfs, reqs)
    for r, o in zip(more[:20], outs2[:20]):
        assert torch.equal(o, single(lfs, r))
    for o, o3 in zip(outs, outs3):
        assert torch.equal(o, o3)
    b.close()


DENSE = [(8, 8, 64, 64, dict(block=4, levels=2, cluster=(2,), blk_threshold=2)),
         (9, 9, 125, 87, dict(block=4, levels=3, cluster=(2, 2), blk_threshold=40, quant_bits=2))]


@pytest.fixture(scope="module")
def dense_pair(gpu):
    # an 8x8 light field of 64x64 views and a 9x9 lenslet-like one, with 64
    # novel 128x96 views that cover most of both
    encs = [oracle_encode(make_lf(U, V, W, H, seed=300 + U, vignetting=U == 9), **kw) for U, V, W, H, kw in DENSE]
    lfs = [lfc.lfc_open(e.stream) for e in encs]
    rng = np.random.default_rng(302)
    reqs = []
    for k in range(64):
        li = k % 2
        U, V = DENSE[li][0], DENSE[li][1]
        reqs.append((li, 128, 96, (rng.uniform(0, U - 1), rng.uniform(0, V - 1), rng.uniform(-1, 1),
                                   rng.uniform(-1, 1))))
    yield encs, lfs, reqs
    for lf in lfs:
        lf.close()


def test_dense_batch_over_two_light_fields(dense_pair):
    # each light field is decoded once by the persistent colour kernel (both
    # in one launch) and interpolated in one launch; every result equals the
    # light field's own render of it, and the oracle's to 1e-5.  Six calls in
    # a row reuse every table slot and its work counters.
    encs, lfs, reqs = dense_pair
    say("dense batch over two light fields")
    b = lfc.Batch()
    outs = b.render(lfs, reqs)
    for li in range(2):
        mine = [(r, o) for r, o in zip(reqs, outs) if r[0] == li]
        views = torch.tensor([r[3] for r, _ in mine], dtype=torch.float32, device="cuda")
        own = lfc.lfc_render_views(lfs[li], views, 128, 96)
        for (r, o), ref in zip(mine, own):
            assert torch.equal(o, ref), r
        U, V, W, H, _ = DENSE[li]
        got = torch.stack([o for _, o in mine[:4]]).cpu().numpy()
        ref = oracle.render(encs[li].r0, U, V, W, H, np.array([r[3] for r, _ in mine[:4]], dtype=np.float32), 128, 96)
        assert max_abs(got, ref) <= 1e-5
    for call in range(6):
        again = b.render(lfs, reqs)
        for o, o2 in zip(outs, again):
            assert torch.equal(o, o2), call
    b.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_plan_replays(fields, dense_pair, graph):
    # a batch plan writes what lfc_batch_render writes for the same requests,
    # at every launch: a sparse batch (every light field by tiles), a mixed
    # one and the dense pair (both decoded by the colour path in one
    # persistent launch, whose counters the graph never clears).  The outputs
    # are filled with NaN before each launch, and eager work and
    # synchronisations run between the launches.
    _, lfs = fields
    rng = np.random.default_rng(77)
    sparse = [(li, 30, 20, (rng.uniform(0, FIELDS[li][0] - 1), rng.uniform(0, FIELDS[li][1] - 1), 0.3, -0.2))
              for li in range(len(FIELDS))]
    cases = [("sparse", lfs, sparse, 0), ("mixed", lfs, mixed_requests(48, 911), None),
             ("dense", dense_pair[1], dense_pair[2], 2)]
    side = torch.zeros(1 << 20, device="cuda")
    for name, lf_list, reqs, n_dec in cases:
        say(f"batch plan {name}, graph={graph}, {len(reqs)} requests")
        b = lfc.Batch()
        ref = [o.clone() for o in b.render(lf_list, reqs)]
        b.close()
        plan = lfc.BatchPlan(lf_list, reqs, graph=graph)
        k, g = plan.info()
        assert g == graph
        if n_dec is not None:
            assert k == n_dec, name
        for rep in range(4):
            for o in plan.outs:
                o.fill_(float("nan"))
            torch.cuda.synchronize()
            plan.launch()
            side.add_(1.0)
            torch.cuda.synchronize()
            for i, (o, r) in enumerate(zip(plan.outs, ref)):
                assert torch.equal(o, r), (name, rep, i, reqs[i])
        plan.close()
    assert float(side[0]) == 4.0 * len(cases)
    with pytest.raises(lfc.LFCError):
        lfc.BatchPlan(lfs, [])
    with pytest.raises(lfc.LFCError):
        lfc.BatchPlan(lfs, [(len(lfs), 8, 8, (0.0, 0.0, 0.0, 0.0))])


def test_batch_argument_errors(fields):
    _, lfs = fields
    lib = lfc.load()
    b = lfc.Batch()
    s = torch.cuda.current_stream().cuda_stream
    out = torch.empty((3, 8, 8), dtype=torch.float32, device="cuda")
    handles = (C.c_void_p * len(lfs))(*[lf.handle for lf in lfs])
    ptrs = (C.c_void_p * 1)(out.data_ptr())
    bad_index = lfc._requests([(len(lfs), 8, 8, (0, 0, 0, 0))])
    assert lib.lfc_batch_render(b.handle, handles, len(lfs), bad_index, 1, ptrs, s) == -1
    bad_size = lfc._requests([(0, 0, 8, (0, 0, 0, 0))])
    assert lib.lfc_batch_render(b.handle, handles, len(lfs), bad_size, 1, ptrs, s) == -1
    null_out = (C.c_void_p * 1)(None)
    ok = lfc._requests([(0, 8, 8, (0, 0, 0, 0))])
    assert lib.lfc_batch_render(b.handle, handles, len(lfs), ok, 1, null_out, s) == -1
    assert lib.lfc_batch_render(b.handle, handles, len(lfs), ok, 0, ptrs, s) == 0
    assert lib.lfc_batch_render(b.handle, handles, len(lfs), ok, 1, ptrs, s) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, single(lfs, (0, 8, 8, (0, 0, 0, 0))))
    b.close()


def test_server_results_match_single_renders(fields):
    _, lfs = fields
    reqs = mixed_requests(60, seed=7)
    say("server", len(reqs), "requests")
    sv = lfc.Server(lfs, max_batch=16, streams=2, out_pool_bytes=64 << 20)
    tickets = [sv.submit(*r) for r in reqs]
    for t, r in zip(tickets, reqs):
        got, lat = sv.fetch(t, r[1], r[2], timeout_ms=60000)
        assert lat >= 0
        assert torch.equal(got, single(lfs, r)), r
    st = sv.stats()
    assert st["submitted"] == st["completed"] == len(reqs)
    assert 1 <= st["max_batch_seen"] <= 16 and st["pool_bytes_in_use"] == 0
    sv.close()


def test_server_results_repeatable(fields):
    # the whole mix several times over, two lanes: every result of every
    # round must be the lone render's bytes (before the batched render kernel
    # read its request record once per workgroup, this mix showed rare
    # residual-sized errors whose mechanism was not established; this test
    # guards the fixed code)
    _, lfs = fields
    reqs = mixed_requests(60, seed=7)
    refs = [single(lfs, r) for r in reqs]
    for rnd in range(6):
        say("round", rnd)
        sv = lfc.Server(lfs, max_batch=16, streams=2, out_pool_bytes=64 << 20)
        tickets = [sv.submit(*r) for r in reqs]
        for t, r, ref in zip(tickets, reqs, refs):
            got, _ = sv.fetch(t, r[1], r[2], timeout_ms=60000)
            assert torch.equal(got, ref), (rnd, r)
        sv.close()


def test_batch_contexts_across_streams(fields):
    # one context, calls alternating between two streams with no waits in
    # between: each call's table must survive until its own launches finish
    _, lfs = fields
    reqs = mixed_requests(200, seed=11)
    refs = [single(lfs, r) for r in reqs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    b = lfc.Batch()
    pending = []
    for k in range(0, len(reqs), 10):
        part = list(range(k, min(k + 10, len(reqs))))
        st = streams[(k // 10) % 2]
        with torch.cuda.stream(st):
            outs = b.render(lfs, [reqs[i] for i in part], cuda_stream=st)
        pending.append((part, outs))
    torch.cuda.synchronize()
    for part, outs in pending:
        for i, o in zip(part, outs):
            assert torch.equal(o, refs[i]), reqs[i]
    b.close()


def test_server_memory_admission(fields):
    # a pool that holds two 64x64 results: the queue waits for releases
    _, lfs = fields
    reqs = [(i % len(lfs), 64, 64, (0.5 * i % 3, 0.25 * i % 2, 0.0, 0.0)) for i in range(12)]
    pool = 2 * 3 * 64 * 64 * 4
    say("server admission, pool", pool)
    sv = lfc.Server(lfs, max_batch=8, streams=2, out_pool_bytes=pool)
    tickets = [sv.submit(*r) for r in reqs]
    for t, r in zip(tickets, reqs):
        got, _ = sv.fetch(t, 64, 64, timeout_ms=60000)
        assert torch.equal(got, single(lfs, r))
    st = sv.stats()
    assert st["completed"] == len(reqs) and st["max_batch_seen"] <= 2 and st["admission_waits"] > 0
    with pytest.raises(lfc.LFCError):
        sv.submit(0, 128, 128, (0, 0, 0, 0))   # larger than the whole pool
    sv.close()


def test_server_device_memory_cap_and_queue_limit(fields):
    # memory admission of the resident light fields: a cap below their device
    # bytes plus the pool refuses the server; a cap that holds them but not
    # the decoded-view buffers serves every request by tiles, the same bytes
    _, lfs = fields
    resident = sum(int(lf.info.device_bytes) for lf in lfs)
    pool = 8 << 20
    with pytest.raises(lfc.LFCError) as e:
        lfc.Server(lfs, max_batch=8, streams=2, out_pool_bytes=pool, device_bytes_cap=resident + pool - 1)
    assert e.value.status == -3
    reqs = mixed_requests(40, seed=11)
    sv = lfc.Server(lfs, max_batch=16, streams=2, out_pool_bytes=pool, device_bytes_cap=resident + pool)
    tickets = [sv.submit(*r) for r in reqs]
    for t, r in zip(tickets, reqs):
        got, _ = sv.fetch(t, r[1], r[2], timeout_ms=60000)
        assert torch.equal(got, single(lfs, r)), r
    sv.close()
    # queue overflow: a pool that holds one 64x64 result and nothing released,
    # so requests pile up; submits beyond max_queue waiting ones are refused
    one = 3 * 64 * 64 * 4
    sv = lfc.Server(lfs, max_batch=1, streams=1, out_pool_bytes=one, max_queue=2)
    accepted, refused = [], 0
    for i in range(8):
        try:
            accepted.append(sv.submit(0, 64, 64, (0.5, 0.5, 0.0, 0.0)))
        except lfc.LFCError as err:
            assert err.status == -3
            refused += 1
    assert refused >= 8 - 3 and len(accepted) <= 3
    for t in accepted:   # each release admits the next waiting one
        got, _ = sv.fetch(t, 64, 64, timeout_ms=60000)
        assert torch.equal(got, single(lfs, (0, 64, 64, (0.5, 0.5, 0.0, 0.0))))
    sv.close()
    with pytest.raises(lfc.LFCError):
        lfc.Server(lfs, max_batch=1, streams=1, out_pool_bytes=one, max_queue=-1)


def test_server_replay_and_plain_mode(fields):
    _, lfs = fields
    reqs = mixed_requests(300, seed=8)
    arrivals = np.cumsum(np.random.default_rng(9).exponential(0.05, len(reqs)))
    for max_batch, streams in ((32, 2), (1, 1)):
        say("replay", max_batch, streams)
        sv = lfc.Server(lfs, max_batch=max_batch, streams=streams, out_pool_bytes=256 << 20)
        lat = sv.replay(reqs, arrivals)
        st = sv.stats()
        assert st["completed"] == len(reqs) and np.all(lat > 0) and np.all(np.isfinite(lat))
        assert st["max_batch_seen"] <= max_batch and st["pool_bytes_in_use"] == 0
        sv.close()


def test_server_workload_sizes(gpu):
    # the serving mix's two output sizes on a 17x17 light field; every result
    # equals the lone render's bytes and the oracle's renderer to 1e-5
    lfspec = synth.LFSpec(17, 17, 128, 128, 3, 2.0, 1.5, 77)
    enc = oracle_encode(synth.light_field(lfspec), block=4, levels=3, cluster=(2, 3), blk_threshold=30, quant_bits=1)
    lf = lfc.lfc_open(enc.stream)
    views = synth.novel_views(6, 17, 17, seed=78)
    reqs = [(0, 512 if i % 2 else 1024, 512 if i % 2 else 1024, tuple(views[i])) for i in range(6)]
    sv = lfc.Server([lf], max_batch=8, streams=2, out_pool_bytes=6 * 3 * 1024 * 1024 * 4)
    tickets = [sv.submit(*r) for r in reqs]
    for t, r in zip(tickets, reqs):
        got, _ = sv.fetch(t, r[1], r[2], timeout_ms=60000)
        assert torch.equal(got, single([lf], r))
        ref = oracle.render(enc.r0, 17, 17, 128, 128, np.array([r[3]], dtype=np.float32), r[1], r[2])[0]
        assert max_abs(got.cpu().numpy(), ref) <= 1e-5, r
    sv.close()
    lf.close()


def test_batch_calls_check_buffer_sizes(fields):
    # outputs and request lists too small for the call are refused before any
    # launch (exact-size raw allocations: a torch tensor sits inside a larger
    # caching-allocator segment, and the library sees only the allocation)
    _, lfs = fields
    lib = lfc.load()
    s = torch.cuda.current_stream().cuda_stream
    hip = C.CDLL("libamdhip64.so")
    small = C.c_void_p()
    assert hip.hipMalloc(C.byref(small), C.c_size_t(3 * 8 * 8 * 4)) == 0
    b = lfc.Batch()
    try:
        handles = (C.c_void_p * len(lfs))(*[lf.handle for lf in lfs])
        ptrs = (C.c_void_p * 1)(small.value)
        fits = lfc._requests([(0, 8, 8, (0, 0, 0, 0))])
        too_big = lfc._requests([(0, 9, 8, (0, 0, 0, 0))])
        assert lib.lfc_batch_render(b.handle, handles, len(lfs), too_big, 1, ptrs, s) == -1
        assert b"too small" in lib.lfc_last_error()
        host = np.zeros(3 * 8 * 8, dtype=np.float32)
        host_ptr = (C.c_void_p * 1)(host.ctypes.data)
        assert lib.lfc_batch_render(b.handle, handles, len(lfs), fits, 1, host_ptr, s) == -1
        assert lib.lfc_batch_render(b.handle, handles, len(lfs), fits, 1, ptrs, s) == 0
        torch.cuda.synchronize()
        # batched random access: 16 requests need 16 x 3 x 16 int16 out, 16 x 3 int32 in
        pick = (C.c_void_p * 2)(lfs[0].handle, lfs[3].handle)
        req = torch.zeros((16, 3), dtype=torch.int32, device="cuda")
        out = torch.zeros((16, 3, 4, 4), dtype=torch.int16, device="cuda")
        assert lib.lfc_batch_decode(b.handle, pick, 2, req.data_ptr(), 16, small.value, s) == -1
        assert lib.lfc_batch_decode(b.handle, pick, 2, small.value, 65, out.data_ptr(), s) == -1
        assert lib.lfc_batch_decode(b.handle, pick, 2, req.data_ptr(), 16, out.data_ptr(), s) == 0
        b.check()
    finally:
        torch.cuda.synchronize()
        b.close()
        hip.hipFree(small)


def test_batch_decode_across_light_fields(fields):
    # random access over two light fields of block size 4 in one launch
    encs, lfs = fields
    pick = [lfs[0], lfs[3]]
    rng = np.random.default_rng(11)
    rows = []
    for _ in range(5000):
        li = int(rng.integers(2))
        lf = pick[li]
        nv = lf.info.params.grid_u * lf.info.params.grid_v
        rows.append((li, int(rng.integers(nv)), int(rng.integers(lf.info.n_blocks))))
    req = torch.tensor(rows, dtype=torch.int32, device="cuda")
    b = lfc.Batch()
    got = b.decode(pick, req)
    b.check()
    for li in (0, 1):
        sel = [i for i, r in enumerate(rows) if r[0] == li]
        single = lfc.lfc_decode_blocks(pick[li], req[sel][:, 1:].contiguous(), lfc.LAYOUT_BLOCKS)
        assert torch.equal(got[sel], single)
    # out-of-range requests give zeros and raise the batch's flag
    bad = torch.tensor([[2, 0, 0], [0, 10_000, 0], [1, 0, -1], [0, 0, 0]], dtype=torch.int32, device="cuda")
    out = b.decode(pick, bad)
    with pytest.raises(lfc.LFCError):
        b.check()
    assert not out[:3].any()
    first = lfc.lfc_decode_blocks(pick[0], torch.zeros((1, 2), dtype=torch.int32, device="cuda"), lfc.LAYOUT_BLOCKS)
    assert torch.equal(out[3], first[0])
    b.check()   # cleared
    with pytest.raises(lfc.LFCError):
        b.decode([lfs[0], lfs[1]], req)   # block sizes 4 and 2
    b.close()
