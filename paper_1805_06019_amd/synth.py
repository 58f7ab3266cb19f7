"""Seeded synthetic inputs: light fields, block requests and novel views.

This module holds none of the compression method's arithmetic.  It only makes
inputs, and both the library and the test oracle consume what it makes.

Light fields follow the two-plane parameterisation of the paper (a U x V grid
of W x H 24-bit RGB views, Sec. 2.1 and Sec. 4).  The scene is a stack of
fronto-parallel Lambertian layers.  Each layer has its own gradient-noise
texture, a disparity in pixels per view step and an opacity mask.  The layers
are composited back to front.  Gaussian sensor noise is added last.  A
lenslet-like variant adds vignetting.

Random draws use numpy's PCG64 generator.  Block requests use splitmix64
(Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014), computed from a counter.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class LFSpec:
    grid_u: int
    grid_v: int
    width: int
    height: int
    layers: int
    disparity: float      # layer disparities drawn from U[-disparity, disparity] px per view step
    noise_sigma: float
    seed: int
    vignetting: bool = False


def _fade(t: np.ndarray) -> np.ndarray:
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def gradient_noise(h: int, w: int, cell: int, rng: np.random.Generator, octaves: int = 4,
                   lacunarity: int = 2, gain: float = 0.5) -> np.ndarray:
    """Perlin-style 2-D gradient noise (quintic fade), float32 in about [-1, 1]."""
    total = np.zeros((h, w), dtype=np.float64)
    amp, norm, c = 1.0, 0.0, float(cell)
    for _ in range(octaves):
        gh, gw = int(np.ceil(h / c)) + 2, int(np.ceil(w / c)) + 2
        ang = rng.uniform(0.0, 2.0 * np.pi, size=(gh, gw))
        gx, gy = np.cos(ang), np.sin(ang)
        ys = (np.arange(h) + 0.5) / c
        xs = (np.arange(w) + 0.5) / c
        y0 = np.floor(ys).astype(np.int64)
        x0 = np.floor(xs).astype(np.int64)
        fy = (ys - y0)[:, None]
        fx = (xs - x0)[None, :]

        def corner(dy, dx):
            yy, xx = y0 + dy, x0 + dx
            return gx[yy][:, xx] * (fx - dx) + gy[yy][:, xx] * (fy - dy)

        u, v = _fade(fx), _fade(fy)
        top = corner(0, 0) * (1 - u) + corner(0, 1) * u
        bot = corner(1, 0) * (1 - u) + corner(1, 1) * u
        total += amp * (top * (1 - v) + bot * v)
        norm += amp
        amp *= gain
        c = max(c / lacunarity, 1.0)
    return (total / norm * 1.6).astype(np.float32)


def _layer_order(d: np.ndarray) -> list:
    # layer 0 is the opaque background; the rest go back to front by disparity
    return [0] + sorted(range(1, len(d)), key=lambda k: d[k])


def light_field(spec: LFSpec, threads: int | None = None) -> np.ndarray:
    """Returns uint8 [V][U][H][W][3]; view index vi = v * U + u."""
    U, V, W, H = spec.grid_u, spec.grid_v, spec.width, spec.height
    rng = np.random.default_rng(spec.seed)
    cu, cv = (U - 1) / 2.0, (V - 1) / 2.0
    margin = int(np.ceil(spec.disparity * max(cu, cv, 0.0))) + 2
    th, tw = H + 2 * margin, W + 2 * margin
    cell = 16 if max(W, H) <= 256 else 32
    tex, masks, disp = [], [], []
    for k in range(spec.layers):
        base = rng.uniform(40.0, 215.0, size=3)
        chans = [np.clip(base[c] + 60.0 * gradient_noise(th, tw, cell, rng), 0.0, 255.0)
                 for c in range(3)]
        tex.append(np.stack(chans).astype(np.float32))
        disp.append(0.0 if spec.layers == 1 else rng.uniform(-spec.disparity, spec.disparity))
        if k == 0:
            masks.append(np.ones((th, tw), dtype=bool))
        else:
            low = gradient_noise(th, tw, cell * 4, rng, octaves=2)
            masks.append(low > np.quantile(low, 0.65))
    disp = np.array(disp)
    order = _layer_order(disp)
    out = np.empty((V, U, H, W, 3), dtype=np.uint8)
    if spec.vignetting:
        yy, xx = np.mgrid[0:H, 0:W].astype(np.float32)
        rr = ((xx - (W - 1) / 2) ** 2 + (yy - (H - 1) / 2) ** 2) / (((W - 1) / 2) ** 2 + ((H - 1) / 2) ** 2 + 1e-9)
        pix_gain = (1.0 - 0.25 * rr).astype(np.float32)
        corner = np.hypot(cu, cv) + 1e-9

    def one_view(vi: int) -> None:
        u, v = vi % U, vi // U
        img = None
        for k in order:
            sx = margin - disp[k] * (u - cu)
            sy = margin - disp[k] * (v - cv)
            ix, iy = int(np.floor(sx)), int(np.floor(sy))
            fx, fy = np.float32(sx - ix), np.float32(sy - iy)
            t = tex[k]
            a = t[:, iy:iy + H, ix:ix + W] * (1 - fx) + t[:, iy:iy + H, ix + 1:ix + 1 + W] * fx
            b = t[:, iy + 1:iy + 1 + H, ix:ix + W] * (1 - fx) + t[:, iy + 1:iy + 1 + H, ix + 1:ix + 1 + W] * fx
            layer = a * (1 - fy) + b * fy
            if img is None:
                img = layer
            else:
                mx, my = int(np.rint(sx)), int(np.rint(sy))
                m = masks[k][my:my + H, mx:mx + W]
                img = np.where(m[None], layer, img)
        if spec.vignetting:
            rho = np.hypot(u - cu, v - cv) / corner
            img = img * (np.float32(np.clip(1.0 - 0.5 * rho * rho, 0.0, 1.0)) * pix_gain[None])
        nrng = np.random.default_rng([spec.seed, 7919, vi])
        img = img + nrng.standard_normal(img.shape, dtype=np.float32) * np.float32(spec.noise_sigma)
        out[v, u] = np.clip(np.rint(img), 0, 255).astype(np.uint8).transpose(1, 2, 0)

    n = U * V
    workers = threads or min(16, os.cpu_count() or 1)
    if workers <= 1 or n == 1:
        for vi in range(n):
            one_view(vi)
    else:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one_view, range(n)))
    return out


_MASK64 = (1 << 64) - 1


def splitmix64(seed: int, n: int) -> np.ndarray:
    """n outputs of splitmix64 from counter i = 1..n with the given seed."""
    with np.errstate(over="ignore"):
        z = (np.uint64(seed & _MASK64)
             + np.arange(1, n + 1, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def block_requests(n: int, n_views: int, n_blocks: int, seed: int) -> np.ndarray:
    """n uniformly random (view, block) pairs, int32 [n][2]."""
    z = splitmix64(seed, n)
    vi = ((z >> np.uint64(32)) % np.uint64(n_views)).astype(np.int32)
    b = ((z & np.uint64(0xFFFFFFFF)) % np.uint64(n_blocks)).astype(np.int32)
    return np.stack([vi, b], axis=1)


def novel_views(n: int, grid_u: int, grid_v: int, seed: int, pan: float = 1.0) -> np.ndarray:
    """n random cameras (u, v, s, t) inside the grid, float32 [n][4]."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, grid_u - 1, n)
    v = rng.uniform(0.0, grid_v - 1, n)
    s = rng.uniform(-pan, pan, n)
    t = rng.uniform(-pan, pan, n)
    return np.stack([u, v, s, t], axis=1).astype(np.float32)
