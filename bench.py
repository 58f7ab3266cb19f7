"""Benchmark of the RLFC decode-and-render path on one MI355X.

One step = one whole-light-field decode (images layout) of the 17x17 x
512x512 RGB workload coded at 40 dB PSNR_YCoCg: every block of every view,
through the key view and the residuals of both tree levels.  The same run
also times, on the same light field, a batched render of 64 novel 512x512
views per launch, single-view renders launched one per request (the plain
kernel; p50/p99 latency), 10^6 random block accesses, the 50 dB coding of
the same light field, the 64-view render of the 9x9 lenslet-like light
field, and the serving loop over 12 resident light fields (Poisson arrivals,
batched server vs one plain launch per request).  Inputs are resident in
device memory before any timed region.

Prints one JSON line.  ``value`` is decoded samples per second of the step.
``roofline`` prices the whole-field kernel's algorithmic bytes per launch
(int16 output, key-view blocks, block offsets, the compressed SRV section
and the rank directory read once) against 8 TB/s of HBM; ``traffic`` is the
kernel's measured HBM bytes per launch from the committed counter runs.  ``cpu_baseline`` is the oracle's
whole-field decoder on the host's cores (bounded sample).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(tile_blocks: int, staged: bool):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on the current kernel source at this decode tile capacity and
    staging; else None."""
    from paper_1805_06019_amd.prof_summary import kernel_source_hash
    path = os.path.join(ROOT, "profiles", f"traffic_decode_lf_full40_t{tile_blocks}{'_staged' if staged else ''}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if (rec.get("kernel_source_hash") != kernel_source_hash() or rec.get("tile_blocks") != tile_blocks
            or bool(rec.get("staged", False)) != staged):
        return None
    return rec.get("bytes_per_launch")


def time_launches(fn, n, torch):
    """Per-launch durations (ms) from events recorded on the launch stream."""
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in ev])


def _cpu_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def _threaded(fn, parts):
    """Runs fn(*part) for every part on its own thread (the oracle's C calls
    release the GIL); returns the wall time."""
    import threading
    ths = [threading.Thread(target=fn, args=p) for p in parts]
    t0 = time.perf_counter()
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    return time.perf_counter() - t0


def cpu_baseline(streams: dict, nv: int, hp: int, wp: int, nb: int, min_cpu_s: float = 8.0):
    """The oracle on the host's cores (16 threads at most: the GPU's share of
    the host), bounded samples of each workload the GPU runs:
    whole-field decode at 40 dB (the headline leg, repeated for about
    min_cpu_s of CPU time), the same single-threaded, the 50 dB whole field,
    per-block decodes (Alg. 2 literally) of the first requests of the 10^6
    random accesses, and 64 novel 512x512 views of the tiny and lenslet-like
    light fields.  Returns the 40 dB decode (for the parity check) and the
    record."""
    import oracle
    from paper_1805_06019_amd import synth
    model, ncpu, usable = _cpu_info()
    threads = max(1, min(16, usable))
    out = np.zeros((nv, 3, hp, wp), dtype=np.int16)
    chunks = np.linspace(0, nb, threads + 1).astype(int)
    parts = [(streams["full40"], int(chunks[i]), int(chunks[i + 1]), out) for i in range(threads)
             if chunks[i] < chunks[i + 1]]
    passes, wall, t_start = 0, 0.0, time.time()
    while True:
        wall += _threaded(oracle.decode_all, parts)
        passes += 1
        if wall * threads >= min_cpu_s or time.time() - t_start > 60:
            break
    samples = passes * nv * 3 * hp * wp
    rec = dict(value=samples / wall / 1e9, unit="Gsamples/s", cores=threads, kind="oracle",
               sample=f"{passes} whole-field decode pass(es) of the 17x17x512x512 40 dB stream, "
                      f"blocks split over {threads} threads, {wall:.2f} s wall",
               cpu_model=model, cpu_count=ncpu, cpu_usable=usable, legs={})
    legs = rec["legs"]
    # one thread, one pass over a quarter of the blocks (into the buffer the
    # threaded passes wrote, so that no page is touched for the first time)
    t0 = time.perf_counter()
    oracle.decode_all(streams["full40"], 0, nb // 4, out)
    dt = time.perf_counter() - t0
    legs["decode_full40_1thread"] = dict(gsamples_per_s=round(nv * 3 * hp * wp / 4 / dt / 1e9, 4), threads=1,
                                         sample="blocks 0..NB/4 of every view, one pass")
    # 50 dB, one threaded pass
    out50 = np.zeros_like(out)
    parts50 = [(streams["full50"], a, b, out50) for _, a, b, _ in parts]
    dt = _threaded(oracle.decode_all, parts50)
    legs["decode_full50"] = dict(gsamples_per_s=round(nv * 3 * hp * wp / dt / 1e9, 4), threads=threads,
                                 sample="one whole-field pass")
    del out50
    # Alg. 2 per block: the first k of the 10^6 uniformly random accesses
    req = synth.block_requests(1_000_000, nv, nb, seed=202)
    k = 32_000 * threads
    blk = np.zeros((k, 3, 4, 4), dtype=np.int16)
    cuts = np.linspace(0, k, threads + 1).astype(int)
    dt = _threaded(lambda a, b: oracle.decode_requests(streams["full40"], req[a:b], blk[a:b]),
                   [(int(cuts[i]), int(cuts[i + 1])) for i in range(threads)])
    legs["random_access_full40"] = dict(ns_per_access=round(dt * 1e9 / k, 1),
                                        gsamples_per_s=round(k * 48 / dt / 1e9, 5), threads=threads,
                                        sample=f"first {k} of the 10^6 accesses (seed 202), all 3 channels")
    # 64 novel 512x512 views (seed 302) from the decoded tiny and lenslet-like fields
    for name, key, U, V, W, H in (("render_tiny", "tiny", 8, 8, 64, 64),
                                  ("render_lenslet40", "lenslet40", 9, 9, 625, 434)):
        dec = oracle.decode_all(streams[key])
        views = synth.novel_views(64, U, V, seed=302)
        img = np.zeros((64, 3, 512, 512), dtype=np.float32)

        def rend(a, b, dec=dec, views=views, img=img, U=U, V=V, W=W, H=H):
            img[a:b] = oracle.render(dec, U, V, W, H, views[a:b], 512, 512)
        cuts = np.linspace(0, 64, threads + 1).astype(int)
        dt = _threaded(rend, [(int(cuts[i]), int(cuts[i + 1])) for i in range(threads) if cuts[i] < cuts[i + 1]])
        legs[name] = dict(views_per_s=round(64 / dt, 2), threads=threads, sample="64 views of 512x512, one pass")
    return out, rec


def serving(lfc, synth, torch, n_req: int = 20000):
    """Serving loop over 12 resident light fields (4 of 8x8x256^2, 4 lenslet-like
    9x9x625x434, 4 of 17x17x1024^2, each coded at about 40 dB): Poisson arrivals
    of novel-view requests, half 512^2 and half 1024^2, uniform over the light
    fields, replayed against the batching server and against one plain launch
    per request; p50/p99 latency from arrival to completion per arrival rate,
    and the saturation throughput of both."""
    from paper_1805_06019_amd.workloads import (WORKLOADS, serve_large_spec, serve_lenslet_spec,
                                                serve_small_spec)
    t0 = time.time()
    kinds = [(serve_small_spec, range(401, 405), WORKLOADS["serve_small40"]),
             (serve_lenslet_spec, range(405, 409), WORKLOADS["serve_lenslet40"]),
             (serve_large_spec, range(409, 413), WORKLOADS["serve_large40"])]
    lfs, grids, psnr = [], [], []
    for mk, seeds, enc in kinds:
        for sd in seeds:
            spec = mk(sd)
            rgb = synth.light_field(spec)
            stream, st = lfc.lfc_encode_ex(rgb, enc.params(grid_u=spec.grid_u, grid_v=spec.grid_v,
                                                           width=spec.width, height=spec.height))
            del rgb
            lfs.append(lfc.lfc_open(stream))
            grids.append((spec.grid_u, spec.grid_v))
            psnr.append(round(st["psnr"], 2))
    log(f"serving: 12 light fields generated, coded and opened in {time.time() - t0:.1f}s")
    rng = np.random.default_rng(402)
    li = rng.integers(0, len(lfs), n_req)
    big = rng.random(n_req) < 0.5
    reqs = []
    for k in range(n_req):
        U, V = grids[li[k]]
        side = 1024 if big[k] else 512
        reqs.append((int(li[k]), side, side, (rng.uniform(0, U - 1), rng.uniform(0, V - 1),
                                              rng.uniform(-1, 1), rng.uniform(-1, 1))))
    pool = 4 << 30
    res = dict(light_fields=len(lfs), psnr_db=psnr, requests=n_req, sizes="50% 512x512, 50% 1024x1024",
               batched=dict(max_batch=64, streams=2), plain=dict(max_batch=1, streams=1), points=[])

    def run(max_batch, streams, arrivals):
        sv = lfc.Server(lfs, max_batch=max_batch, streams=streams, out_pool_bytes=pool)
        t = time.perf_counter()
        lat = sv.replay(reqs, arrivals)
        wall = time.perf_counter() - t
        st = sv.stats()
        sv.close()
        return lat, wall, st

    # saturation: every request queued at once
    zero = np.zeros(n_req)
    sat = {}
    for name, mb, ns in (("batched", 64, 2), ("plain", 1, 1)):
        lat, wall, st = run(mb, ns, zero)
        sat[name] = round(n_req / wall, 1)
        log(f"serving {name} saturation: {n_req / wall:.0f} views/s, {st['batches']} launches")
    res["saturation_views_per_s"] = sat
    res["saturation_speedup"] = round(sat["batched"] / sat["plain"], 2)
    # Poisson arrivals at fractions of the plain kernel's saturation rate, and beyond it
    for frac in (0.5, 0.9, 2.0):
        lam = frac * sat["plain"]
        arrivals = np.cumsum(rng.exponential(1000.0 / lam, n_req))
        point = dict(rate_per_s=round(lam, 1))
        for name, mb, ns in (("batched", 64, 2), ("plain", 1, 1)):
            lat, wall, st = run(mb, ns, arrivals)
            point[name] = dict(p50_ms=round(float(np.percentile(lat, 50)), 3),
                               p99_ms=round(float(np.percentile(lat, 99)), 3),
                               views_per_s=round(n_req / wall, 1), mean_batch=round(n_req / st["batches"], 2))
        res["points"].append(point)
        log(f"serving at {lam:.0f}/s: {point}")
    for lf in lfs:
        lf.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the secondary measurements")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--tile-blocks", type=int, default=0,
                    help="decode tile capacity to use instead of measuring the choice (profiling runs "
                         "take the value a default run chose, so that every traced launch is the timed kernel)")
    ap.add_argument("--no-cold", action="store_true",
                    help="skip the cold-cache launches (profiling runs, so that every traced launch is a warm one)")
    ap.add_argument("--staged", action="store_true",
                    help="with --tile-blocks: stage each strip in LDS (the other choice the tuner measures)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(groups and views shard with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1805_06019_amd import lfc, synth
    from paper_1805_06019_amd.workloads import WORKLOADS

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    lfc.load()
    dev_props = torch.cuda.get_device_properties(0)

    # -- setup: synthetic light field, host encode, upload (untimed) --------
    w40 = WORKLOADS["full40"]
    t0 = time.time()
    rgb = synth.light_field(w40.spec)
    log(f"generated {w40.spec} in {time.time() - t0:.1f}s")
    t0 = time.time()
    stream40, st40 = lfc.lfc_encode_ex(rgb, w40.params())
    host_encode_s = time.time() - t0
    log(f"encoded full40 in {host_encode_s:.1f}s: {len(stream40) / 1e6:.1f} MB, {st40['psnr']:.3f} dB")
    lf = lfc.lfc_open(stream40, tile_blocks=args.tile_blocks)
    info = lf.info
    nv, hp, wp, nb = 289, info.padded_height, info.padded_width, info.n_blocks
    samples = nv * 3 * hp * wp
    out = torch.empty((nv, 3, hp, wp), dtype=torch.int16, device="cuda")
    # setup (untimed): the library's measured choice of the decode tile capacity
    # and of staging strips in LDS
    if args.tile_blocks:
        (tile_blocks, staged), tile_tried = (args.tile_blocks, args.staged), []
        stage_cap = -1 if args.staged else 0
    else:
        (tile_blocks, staged), tile_tried = lfc.lfc_tune_decode_ex(lf, reps=5, out=out)
        stage_cap = None   # the handle keeps the tuner's choice
    log(f"decode tuning: {tile_tried} -> {tile_blocks}, staged {staged}")

    def step():
        lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_IMAGES, out=out, stage_cap_words=stage_cap)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # -- timed region: exactly K steps ---------------------------------------
    t_begin, t_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_begin.record()
    for _ in range(args.steps):
        step()
    t_end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t_begin.elapsed_time(t_end)
    ms_per_step = ms_total / args.steps
    value = samples / (ms_per_step * 1e-3) / 1e9
    lfc.lfc_check(lf)
    log(f"whole-field decode: {ms_per_step:.4f} ms/step, {value:.1f} Gsamples/s (host wall {wall:.3f}s)")

    # per-launch durations of the dominant kernel, on its own stream
    per_launch = time_launches(step, max(args.steps, 20), torch)
    srv_bytes = 4 * (int(np.frombuffer(stream40, dtype=np.uint32, count=1,
                                       offset=int(np.frombuffer(stream40, dtype=np.uint64, count=1, offset=112)[0])
                                       + 4 * info.n_groups)[0]) + 2)
    nbw = (info.n_srv + 31) // 32
    alg_bytes = (samples * 2                       # int16 output written once
                 + info.n_top * nb * 3 * 16 * 2    # key-view blocks
                 + 4 * (info.n_groups + 1)         # block offsets
                 + srv_bytes                       # compressed SRV section
                 + 4 * info.n_groups * nbw         # rank directory: one word per bitmap word
                 + 4 * nv * 4)                     # leaf schedule
    achieved = alg_bytes / (per_launch.mean() * 1e-3) / 1e9
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4), traffic=measured_traffic(tile_blocks, staged),
                    kernel="k_decode_lf<4>", algorithmic_bytes_per_launch=alg_bytes,
                    launch_ms_mean=round(float(per_launch.mean()), 5),
                    launch_ms_p50=round(float(np.median(per_launch)), 5))

    # cold L2/MALL: a 1 GiB write between launches, outside the timed events
    if not args.no_cold:
        flush = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        cold = []
        for _ in range(10):
            flush.fill_(1)
            cold.append(time_launches(step, 1, torch)[0])
        del flush
        roofline["launch_ms_cold_mean"] = round(float(np.mean(cold)), 5)
        roofline["frac_cold"] = round(alg_bytes / (np.mean(cold) * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

    extra = {}
    stream50 = streaml = dec50 = None
    if not args.quick:
        # batched render: 64 novel 512x512 views per launch (fused decode); the
        # colour kernel's tile capacity measured first (untimed setup)
        rgb_tile40, rgb_tried40 = lfc.lfc_tune_decode_rgb(lf, reps=3)
        log(f"colour decode tuning: {rgb_tried40} -> {rgb_tile40}")
        views = torch.from_numpy(synth.novel_views(64, 17, 17, seed=302)).cuda()
        img = torch.empty((64, 3, 512, 512), dtype=torch.float32, device="cuda")
        rfn = lambda: lfc.lfc_render_views(lf, views, 512, 512, out=img)
        for _ in range(3):
            rfn()
        r = time_launches(rfn, 10, torch)
        out_bytes = 64 * 3 * 512 * 512 * 4
        # algorithmic bytes of the launch: the float output written once and
        # the compressed light field (key views, offsets, SRV section) read once
        render_bytes = out_bytes + len(stream40)
        extra["render_full40"] = dict(views_per_launch=64, ms_per_launch=round(float(r.mean()), 4),
                                      views_per_s=round(64 / (r.mean() * 1e-3), 1),
                                      output_write_frac_of_hbm=round(out_bytes / (r.mean() * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                      roofline=dict(bound="hbm", algorithmic_bytes=render_bytes,
                                                    frac=round(render_bytes / (r.mean() * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)),
                                      rgb_tile_blocks=rgb_tile40,
                                      rgb_tile_tuning={str(c): round(ms, 4) for c, ms in rgb_tried40})
        # plain kernel: one launch per 512x512 view request
        one = torch.from_numpy(synth.novel_views(200, 17, 17, seed=303)).cuda()
        img1 = torch.empty((1, 3, 512, 512), dtype=torch.float32, device="cuda")
        for i in range(5):
            lfc.lfc_render_views(lf, one[i:i + 1], 512, 512, out=img1)
        lat = np.array([time_launches(lambda i=i: lfc.lfc_render_views(lf, one[i:i + 1], 512, 512, out=img1),
                                      1, torch)[0] for i in range(200)])
        extra["view_latency_plain"] = dict(requests=200, p50_ms=round(float(np.percentile(lat, 50)), 4),
                                           p99_ms=round(float(np.percentile(lat, 99)), 4),
                                           views_per_s=round(1000.0 / lat.mean(), 1))
        extra["render_full40"]["speedup_vs_plain"] = round(extra["render_full40"]["views_per_s"]
                                                           / extra["view_latency_plain"]["views_per_s"], 2)
        # measured tuning of the launch shape, then the tuned render captured in a HIP graph
        best, tried = lfc.lfc_render_tune(lf, views, 512, 512, out=img, reps=5)
        plan = lfc.RenderPlan(lf, views, 512, 512, out=img, cfg=best, graph=True)
        for _ in range(3):
            plan.launch()
        g = time_launches(plan.launch, 10, torch)
        plan.close()
        extra["render_full40"]["tuned"] = dict(config=list(best), tried={f"{c[0]}:{c[1]}x{c[2]}": round(ms, 4)
                                                                          for c, ms in tried})
        extra["render_full40"]["graph"] = dict(ms_per_launch=round(float(g.mean()), 4),
                                               views_per_s=round(64 / (g.mean() * 1e-3), 1))
        # single-view requests through a graph-captured plan (views rewritten in place)
        buf1 = one[:1].clone()
        best1, _ = lfc.lfc_render_tune(lf, buf1, 512, 512, out=img1, reps=5)
        plan1 = lfc.RenderPlan(lf, buf1, 512, 512, out=img1, cfg=best1, graph=True)
        lat_g = []
        for i in range(200):
            buf1.copy_(one[i:i + 1])
            lat_g.append(time_launches(plan1.launch, 1, torch)[0])
        plan1.close()
        lat_g = np.array(lat_g)
        extra["view_latency_graph"] = dict(requests=200, config=list(best1),
                                           p50_ms=round(float(np.percentile(lat_g, 50)), 4),
                                           p99_ms=round(float(np.percentile(lat_g, 99)), 4),
                                           views_per_s=round(1000.0 / lat_g.mean(), 1))
        del img
        # 10^6 uniformly random (view, block) accesses, all three channels
        req = torch.from_numpy(synth.block_requests(1_000_000, nv, nb, seed=202)).cuda()
        blk = torch.empty((1_000_000, 3, 4, 4), dtype=torch.int16, device="cuda")
        afn = lambda: lfc.lfc_decode_blocks(lf, req, lfc.LAYOUT_BLOCKS, out=blk)
        afn()
        a = time_launches(afn, 10, torch)
        # algorithmic bytes of one access (Alg. 2 for the three channels of one
        # block): per channel the group's two offsets (8 B) and the key-view
        # block (2 B^2), and per residual level the bitmap word, the two
        # directory words and, with the stream's presence rate, a stored
        # block's mean payload; then the int16 output (3 x 2 B^2)
        n_levels = max(0, w40.levels - 1)
        presence = int(st40["present_blocks"]) / max(1, info.n_groups * info.n_srv)
        pay = srv_bytes / max(1, int(st40["present_blocks"]))
        per_access = 3 * (8 + 2 * 16 + n_levels * (4 + 8 + presence * pay)) + 3 * 2 * 16
        ra_bytes = per_access * 1_000_000
        extra["random_access"] = dict(requests=1_000_000, ms=round(float(a.mean()), 4),
                                      ns_per_access=round(float(a.mean()) * 1e6 / 1e6, 3),
                                      gsamples_per_s=round(48e6 / (a.mean() * 1e-3) / 1e9, 2),
                                      roofline=dict(bound="hbm", algorithmic_bytes_per_access=round(per_access, 1),
                                                    achieved_gbs=round(ra_bytes / (a.mean() * 1e-3) / 1e9, 1),
                                                    frac=round(ra_bytes / (a.mean() * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)))
        lfc.lfc_check(lf)
        del blk, req
        # 50 dB coding of the same light field
        w50 = WORKLOADS["full50"]
        stream50, st50 = lfc.lfc_encode_ex(rgb, w50.params())
        lf50 = lfc.lfc_open(stream50)
        out50 = torch.empty_like(out)
        (tile50, staged50), _ = lfc.lfc_tune_decode_ex(lf50, reps=5, out=out50)
        d50 = time_launches(lambda: lfc.lfc_decode_blocks(lf50, None, lfc.LAYOUT_IMAGES, out=out50), 20, torch)
        dec50 = out50.cpu().numpy()   # compared with the oracle's decode with the CPU baseline
        del out50
        extra["full50"] = dict(psnr_db=round(st50["psnr"], 3), bpp=round(8 * len(stream50) / (nv * 512 * 512), 4),
                               ms_per_decode=round(float(d50.mean()), 4), tile_blocks=tile50, staged=staged50,
                               gsamples_per_s=round(samples / (d50.mean() * 1e-3) / 1e9, 1))
        lf50.close()
        # lenslet-like 9x9 x 625x434, 64 views per launch
        wl = WORKLOADS["lenslet40"]
        rgbl = synth.light_field(wl.spec)
        streaml, stl = lfc.lfc_encode_ex(rgbl, wl.params())
        lfl = lfc.lfc_open(streaml)
        rgb_tilel, rgb_triedl = lfc.lfc_tune_decode_rgb(lfl, reps=3)
        log(f"lenslet40 colour decode tuning: {rgb_triedl} -> {rgb_tilel}")
        vl = torch.from_numpy(synth.novel_views(64, 9, 9, seed=302)).cuda()
        imgl = torch.empty((64, 3, 512, 512), dtype=torch.float32, device="cuda")
        lfn = lambda: lfc.lfc_render_views(lfl, vl, 512, 512, out=imgl)
        lfn()
        rl = time_launches(lfn, 10, torch)
        render_bytes_l = 64 * 3 * 512 * 512 * 4 + len(streaml)
        extra["render_lenslet40"] = dict(psnr_db=round(stl["psnr"], 3), views_per_launch=64,
                                         ms_per_launch=round(float(rl.mean()), 4),
                                         views_per_s=round(64 / (rl.mean() * 1e-3), 1),
                                         roofline=dict(bound="hbm", algorithmic_bytes=render_bytes_l,
                                                       frac=round(render_bytes_l / (rl.mean() * 1e-3) / 1e9
                                                                  / HBM_PEAK_GBS, 4)),
                                         rgb_tile_blocks=rgb_tilel,
                                         rgb_tile_tuning={str(c): round(ms, 4) for c, ms in rgb_triedl})
        bestl, _ = lfc.lfc_render_tune(lfl, vl, 512, 512, out=imgl, reps=5)
        planl = lfc.RenderPlan(lfl, vl, 512, 512, out=imgl, cfg=bestl, graph=True)
        planl.launch()
        gl = time_launches(planl.launch, 10, torch)
        planl.close()
        extra["render_lenslet40"]["graph"] = dict(config=list(bestl), ms_per_launch=round(float(gl.mean()), 4),
                                                  views_per_s=round(64 / (gl.mean() * 1e-3), 1))
        lfl.close()
        del imgl
        # the encoder on the GPU (same stream as the host encoder's)
        d_rgb = torch.from_numpy(rgb).cuda()
        lfc.lfc_encode_gpu(d_rgb, w40.params(), want_stream=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gstream, _ = lfc.lfc_encode_gpu(d_rgb, w40.params())
        gpu_encode_s = time.perf_counter() - t0
        extra["encode_full40"] = dict(gpu_s=round(gpu_encode_s, 4), host_s=round(host_encode_s, 3),
                                      host_threads=min(16, os.cpu_count() or 1,
                                                       int(os.environ.get("OMP_NUM_THREADS", "0")) or 16),
                                      same_stream=gstream == stream40)
        del d_rgb, gstream
        # learned encoder control: the per-block network over every control
        # row of the 40 dB field (features from the search mode), and its
        # training step (batch gradient + Adam on 1024 rows)
        from paper_1805_06019_amd import control
        _, stc = lfc.lfc_encode_ctl(rgb, w40.params(), lfc.CTL_SEARCH, 1 << 20, want_features=True, want_stream=False)
        feats = torch.from_numpy(stc["features"]).cuda()
        del stc
        tr = control.Trainer(seed=1)
        lfc.mlp_infer(tr.w, feats)
        mi = time_launches(lambda: lfc.mlp_infer(tr.w, feats), 5, torch)
        rows = feats.shape[0]
        flops = 2.0 * (16 * 64 + 64 * 64 + 64 * 37) * rows
        xb, cb, rb = feats[:1024].contiguous(), torch.zeros(1024, dtype=torch.int8, device="cuda"), \
            torch.zeros(1024, dtype=torch.int8, device="cuda")
        tr.part = torch.empty(8 * (lfc.MLP_PARAMS + 1), dtype=torch.float32, device="cuda")
        tr.step(xb, cb, rb)
        ts = time_launches(lambda: tr.step(xb, cb, rb), 50, torch)
        lfc.mlp_infer(tr.w, feats, precision=lfc.MLP_BF16)
        mb = time_launches(lambda: lfc.mlp_infer(tr.w, feats, precision=lfc.MLP_BF16), 5, torch)
        extra["encoder_control"] = dict(
            infer_rows=int(rows), infer_ms=round(float(mi.mean()), 4),
            infer_rows_per_s=round(rows / (mi.mean() * 1e-3), 1),
            infer_tflops=round(flops / (mi.mean() * 1e-3) / 1e12, 2),
            infer_frac_of_fp32_peak=round(flops / (mi.mean() * 1e-3) / 157.3e12, 4),
            infer_bf16_ms=round(float(mb.mean()), 4),
            infer_bf16_tflops=round(flops / (mb.mean() * 1e-3) / 1e12, 2),
            infer_bf16_frac_of_mfma_peak=round(flops / (mb.mean() * 1e-3) / 2.5e15, 4),
            train_step_ms_1024_rows=round(float(ts.mean()), 4))
        del feats, tr
        if not args.no_serving:
            extra["serving"] = serving(lfc, synth, torch)

    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        streams = dict(full40=stream40)
        streams["full50"] = stream50 if stream50 is not None else lfc.lfc_encode(rgb, WORKLOADS["full50"].params())
        streams["tiny"] = lfc.lfc_encode(synth.light_field(WORKLOADS["tiny"].spec), WORKLOADS["tiny"].params())
        streams["lenslet40"] = streaml if streaml is not None else \
            lfc.lfc_encode(synth.light_field(WORKLOADS["lenslet40"].spec), WORKLOADS["lenslet40"].params())
        ref, cpu = cpu_baseline(streams, nv, hp, wp, nb)
        ok = bool(np.array_equal(ref, out.cpu().numpy()))
        cpu["matches_gpu"] = ok
        if not ok:
            log("WARNING: oracle and GPU whole-field decodes differ")
        if dec50 is not None:
            import oracle
            ok50 = bool(np.array_equal(oracle.decode_all(streams["full50"]), dec50))
            extra["full50"]["matches_oracle"] = ok50
            if not ok50:
                log("WARNING: oracle and GPU 50 dB whole-field decodes differ")

    rec = dict(
        metric="decoded Gsamples/s", value=round(value, 2), unit="Gsamples/s", n_gpus=1,
        steps=args.steps, warmup=args.warmup, ms_per_step=round(ms_per_step, 5), higher_is_better=True,
        scaling="weak", vs_baseline=None, dtype="int16", data="synthetic",
        config=dict(workload="full40: whole-field decode of 17x17 views x 512x512 RGB, 3-level tree "
                             "(17->9->3), 4x4 blocks, q=2, T_blk=67",
                    psnr_db=round(st40["psnr"], 3), bpp=round(8 * len(stream40) / (nv * 512 * 512), 4),
                    samples_per_step=samples, stream_bytes=len(stream40),
                    present_blocks=int(st40["present_blocks"]), tile_blocks=tile_blocks, staged=staged,
                    tile_tuning={f"{c}{'+staged' if st else ''}": round(ms, 4) for c, st, ms in tile_tried}),
        roofline=roofline, cpu_baseline=cpu, device=dict(name=dev_props.name, cus=dev_props.multi_processor_count,
                                                        gcn_arch=getattr(dev_props, "gcnArchName", ""),
                                                        lds_per_block=getattr(dev_props, "shared_memory_per_block", None),
                                                        lds_per_cu=getattr(dev_props, "shared_memory_per_multiprocessor", None)),
        **extra)
    print(json.dumps(rec), flush=True)
    lf.close()


if __name__ == "__main__":
    main()
