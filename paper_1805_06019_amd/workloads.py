"""Named workloads: synthetic light fields and the parameters they are coded with.

Shapes follow the paper's workloads: two-plane grids of 24-bit RGB views
(Sec. 4), 4 x 4 blocks, trees of height 2-3 (Tables 1-3).  The operating
points of the 40 dB and 50 dB encodings come from ``tune.py`` (the largest
block threshold that still meets the PSNR target, per quantiser step, then
the smallest stream); the command and its output are recorded beside each
entry.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from .synth import LFSpec


@dataclass(frozen=True)
class Workload:
    name: str
    spec: LFSpec
    block: int
    levels: int
    cluster: tuple
    pix_threshold: int = 0
    blk_threshold: int = 0
    quant_bits: int = 0
    note: str = field(default="", compare=False)

    def params(self, **over):
        from .lfc import Params
        kw = dict(grid_u=self.spec.grid_u, grid_v=self.spec.grid_v, width=self.spec.width,
                  height=self.spec.height, block=self.block, levels=self.levels, cluster=self.cluster,
                  pix_threshold=self.pix_threshold, blk_threshold=self.blk_threshold,
                  quant_bits=self.quant_bits)
        kw.update(over)
        return Params(**kw)


TINY_SPEC = LFSpec(8, 8, 64, 64, layers=3, disparity=2.0, noise_sigma=2.0, seed=101)
FULL_SPEC = LFSpec(17, 17, 512, 512, layers=6, disparity=3.0, noise_sigma=1.5, seed=201)
LENSLET_SPEC = LFSpec(9, 9, 625, 434, layers=4, disparity=1.0, noise_sigma=1.0, seed=301, vignetting=True)

# the serving mix: four light fields of each geometry, seeds 401-412
def serve_small_spec(seed: int) -> LFSpec:      # 8x8 views of 256x256, as the tiny workload
    return LFSpec(8, 8, 256, 256, layers=3, disparity=2.0, noise_sigma=2.0, seed=seed)


def serve_lenslet_spec(seed: int) -> LFSpec:    # 9x9 lenslet-like views of 625x434
    return LFSpec(9, 9, 625, 434, layers=4, disparity=1.0, noise_sigma=1.0, seed=seed, vignetting=True)


def serve_large_spec(seed: int) -> LFSpec:      # 17x17 views of 1024x1024, as the full workload
    return LFSpec(17, 17, 1024, 1024, layers=6, disparity=3.0, noise_sigma=1.5, seed=seed)


WORKLOADS = {
    # 8x8 views of 64x64, 2-level tree with a key view per 2x2 group, block threshold 2
    "tiny": Workload("tiny", TINY_SPEC, 4, 2, (2,), blk_threshold=2),
    # 17x17 views of 512x512, 3-level tree (17 -> 9 -> 3 views per side)
    # python -m paper_1805_06019_amd.tune full 40:
    #   q=0: 70 -> 40.036 dB 8.878 bpp; q=1: 69 -> 40.042 dB 7.801 bpp; q=2: 67 -> 40.002 dB 6.696 bpp
    "full40": Workload("full40", FULL_SPEC, 4, 3, (2, 3), blk_threshold=67, quant_bits=2,
                       note="40.002 dB, 6.696 bpp"),
    # python -m paper_1805_06019_amd.tune full 50:
    #   q=0: 22 -> 50.313 dB 15.885 bpp; q=1: 15 -> 50.215 dB 14.529 bpp; q=2: 46.39 dB at 0
    "full50": Workload("full50", FULL_SPEC, 4, 3, (2, 3), blk_threshold=15, quant_bits=1,
                       note="50.215 dB, 14.529 bpp"),
    # 9x9 lenslet-like views of 625x434 (W x H) with vignetting, 3-level tree (9 -> 5 -> 3)
    # python -m paper_1805_06019_amd.tune lenslet 40:
    #   q=0: 106 -> 40.056 dB 9.135 bpp; q=1: 103 -> 40.014 dB 8.633 bpp; q=2: 96 -> 40.085 dB 8.140 bpp
    "lenslet40": Workload("lenslet40", LENSLET_SPEC, 4, 3, (2, 2), blk_threshold=96, quant_bits=2,
                          note="40.085 dB, 8.140 bpp"),
    # serving mix (seeds 401-412); the operating point is tuned on the first seed of each geometry
    # python -m paper_1805_06019_amd.tune serve_small 40:
    #   q=0: 88 -> 40.004 dB 14.682 bpp; q=1: 87 -> 40.020 dB 14.339 bpp; q=2: 86 -> 40.025 dB 13.972 bpp
    "serve_small40": Workload("serve_small40", serve_small_spec(401), 4, 2, (2,), blk_threshold=86, quant_bits=2,
                              note="40.025 dB, 13.972 bpp"),
    "serve_lenslet40": Workload("serve_lenslet40", serve_lenslet_spec(405), 4, 3, (2, 2), blk_threshold=96,
                                quant_bits=2, note="the lenslet40 operating point"),
    # python -m paper_1805_06019_amd.tune serve_large 40:
    #   q=0: 68 -> 40.052 dB 8.700 bpp; q=1: 67 -> 40.058 dB 7.655 bpp; q=2: 65 -> 40.024 dB 6.579 bpp
    "serve_large40": Workload("serve_large40", serve_large_spec(409), 4, 3, (2, 3), blk_threshold=65, quant_bits=2,
                              note="40.024 dB, 6.579 bpp"),
}
