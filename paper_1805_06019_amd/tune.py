"""Operating-point search for a PSNR target.

For each quantiser step q, bisects the block threshold for the largest value
whose encoding still reaches the target PSNR_YCoCg (eqs. 4-5); PSNR falls
as the threshold grows (the trend of the paper's Figs. 5-6; a violation is
reported).  Among the q, the smallest stream wins, ties to the smaller q.

    python -m paper_1805_06019_amd.tune full 40
"""
from __future__ import annotations

import sys
import time

from . import lfc, synth
from .workloads import FULL_SPEC, LENSLET_SPEC, TINY_SPEC, serve_large_spec, serve_small_spec

BASE = {
    "tiny": (TINY_SPEC, dict(block=4, levels=2, cluster=(2,))),
    "full": (FULL_SPEC, dict(block=4, levels=3, cluster=(2, 3))),
    "lenslet": (LENSLET_SPEC, dict(block=4, levels=3, cluster=(2, 2))),
    "serve_small": (serve_small_spec(401), dict(block=4, levels=2, cluster=(2,))),
    "serve_large": (serve_large_spec(409), dict(block=4, levels=3, cluster=(2, 3))),
}


def search(rgb, spec, base: dict, target: float, qs=(0, 1, 2), hi: int = 4096, log=print):
    npix = spec.grid_u * spec.grid_v * spec.width * spec.height

    def run(q, t):
        p = lfc.Params(spec.grid_u, spec.grid_v, spec.width, spec.height, quant_bits=q,
                       blk_threshold=t, **base)
        _, st = lfc.lfc_encode_ex(rgb, p, want_stream=False)
        return st["psnr"], 8.0 * st["stream_bytes"] / npix

    best = None
    for q in qs:
        ps0, _ = run(q, 0)
        if ps0 < target:
            log(f"q={q}: {ps0:.2f} dB at threshold 0, below target")
            continue
        lo, top = 0, hi
        ps_top, _ = run(q, top)
        if ps_top >= target:
            lo = top
        else:
            while top - lo > 1:
                mid = (lo + top) // 2
                if run(q, mid)[0] >= target:
                    lo = mid
                else:
                    top = mid
        ps, bpp = run(q, lo)
        log(f"q={q}: threshold {lo} -> {ps:.3f} dB, {bpp:.4f} bpp")
        if best is None or bpp < best[2] - 1e-12:
            best = (q, lo, bpp, ps)
    return best


def main(argv):
    name, target = argv[0], float(argv[1])
    spec, base = BASE[name]
    t = time.time()
    rgb = synth.light_field(spec)
    print(f"generated {name} in {time.time() - t:.1f}s", flush=True)
    best = search(rgb, spec, base, target, log=lambda m: print(m, flush=True))
    print(f"best for {name} at {target} dB: quant_bits={best[0]} blk_threshold={best[1]} "
          f"bpp={best[2]:.4f} psnr={best[3]:.3f}")


if __name__ == "__main__":
    main(sys.argv[1:])
