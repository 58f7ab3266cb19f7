"""Workloads run alone, for rocprofv3 runs behind the committed profiles.

    python paper_1805_06019_amd/prof_run.py [--reps N] [--calib-copy] WORKLOAD...

WORKLOAD is one of
  render64_full40     64 novel 512 x 512 views of the 17 x 17 field at 40 dB
                      (the automatic path: colour decode of the views the
                      batch reads, then the interpolation), one launch each;
  render64_lenslet40  the same for the 9 x 9 lenslet-like field;
  access_full40       10^6 uniformly random (view, block) accesses of the
                      17 x 17 field, all three channels.
Inputs are the same seeded synthetic light fields and cameras bench.py uses.
Each workload runs twice untimed, then N times timed with events; one line
per workload gives the mean and median per launch.  --calib-copy adds one
256 MiB device-to-device copy (the calibration of FETCH_SIZE / WRITE_SIZE).
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

if __package__ in (None, ""):   # run as a script (e.g. under rocprofv3 from another directory)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def _timed(fn, n, torch):
    s = torch.cuda.current_stream()
    for _ in range(2):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in ev:
        a.record(s)
        fn()
        b.record(s)
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in ev])


def main(argv=None) -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--calib-copy", action="store_true")
    ap.add_argument("workloads", nargs="+",
                    choices=["render64_full40", "render64_lenslet40", "access_full40"])
    args = ap.parse_args(argv)

    import torch
    from paper_1805_06019_amd import lfc, synth
    from paper_1805_06019_amd.workloads import WORKLOADS

    assert torch.cuda.is_available(), "prof_run needs a GPU"
    lfc.load()
    opened = {}

    def field(name):
        if name not in opened:
            w = WORKLOADS[name]
            opened[name] = lfc.lfc_open(lfc.lfc_encode(synth.light_field(w.spec), w.params()))
        return opened[name]

    for wl in args.workloads:
        if wl.startswith("render64_"):
            name = wl[len("render64_"):]
            lf = field(name)
            g = WORKLOADS[name].spec.grid_u
            views = torch.from_numpy(synth.novel_views(64, g, g, seed=302)).cuda()
            img = torch.empty((64, 3, 512, 512), dtype=torch.float32, device="cuda")
            t = _timed(lambda: lfc.lfc_render_views(lf, views, 512, 512, out=img), args.reps, torch)
            del img
        else:
            lf = field("full40")
            i = lf.info
            nv = i.params.grid_u * i.params.grid_v
            req = torch.from_numpy(synth.block_requests(1_000_000, nv, i.n_blocks, seed=202)).cuda()
            blk = torch.empty((1_000_000, 3, 4, 4), dtype=torch.int16, device="cuda")
            t = _timed(lambda: lfc.lfc_decode_blocks(lf, req, lfc.LAYOUT_BLOCKS, out=blk), args.reps, torch)
            del blk, req
        print(f"{wl}: {len(t)} launches, mean {t.mean():.4f} ms, median {np.median(t):.4f} ms", flush=True)
    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    for lf in opened.values():
        lf.close()


if __name__ == "__main__":
    main(sys.argv[1:])
