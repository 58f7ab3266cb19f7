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

