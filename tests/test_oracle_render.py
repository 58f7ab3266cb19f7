"""Pins of the oracle's renderer (Sec. 3.6: quadrilinear interpolation of
(u, v, s, t) rays over decoded samples; reading C16).

* integer camera positions with an identity st mapping reproduce the decoded
  view exactly (after inverse YCoCg-R, divided by 255);
* a constant light field renders a constant image (weights sum to one);
* a light field that is multilinear in (u, v, x, y) is reproduced exactly at
  fractional positions, since quadrilinear interpolation is exact on such
  functions.
"""
import numpy as np
import pytest

import oracle
from paper_1805_06019_amd import synth


def encode_decode(lf, U, V, W, H, B=4, L=2, cl=(2,)):
    enc = oracle.encode(lf, oracle.Params(U, V, W, H, B, L, cl))
    return oracle.decode_all(enc.stream)


def test_integer_views_reproduce_decoded_images():
    U, V, W, H = 4, 3, 12, 10
    lf = synth.light_field(synth.LFSpec(U, V, W, H, 3, 1.0, 2.0, 17), threads=1)
    dec = encode_decode(lf, U, V, W, H)
    views = np.array([[u, v, 0, 0] for v in range(V) for u in range(U)], dtype=np.float32)
    out = oracle.render(dec, U, V, W, H, views, W, H)
    expect = lf.reshape(V * U, H, W, 3).transpose(0, 3, 1, 2).astype(np.float32) / 255.0
    assert np.array_equal(out, expect)


def test_constant_light_field_renders_constant():
    U, V, W, H = 5, 4, 8, 8
    lf = np.zeros((V, U, H, W, 3), dtype=np.uint8)
    lf[...] = (200, 30, 90)
    dec = encode_decode(lf, U, V, W, H)
    views = synth.novel_views(16, U, V, seed=3, pan=3.0)
    out = oracle.render(dec, U, V, W, H, views, 13, 7)
    for c, val in enumerate((200, 30, 90)):
        assert np.all(np.abs(out[:, c] - val / 255.0) <= 1e-6)


@pytest.mark.parametrize("wo,ho", [(16, 12), (7, 5), (40, 31)])
def test_multilinear_field_is_exact(wo, ho):
    U, V, W, H = 4, 4, 16, 12
    a, bu, bv, bx, by = 20.0, 9.0, 7.0, 4.0, 5.0
    lf = np.zeros((V, U, H, W, 3), dtype=np.uint8)
    for v in range(V):
        for u in range(U):
            yy, xx = np.mgrid[0:H, 0:W]
            val = a + bu * u + bv * v + bx * xx + by * yy + u * xx
            lf[v, u] = np.stack([val, val * 0.5, 255 - val], axis=-1).astype(np.uint8)
    dec = encode_decode(lf, U, V, W, H)
    views = synth.novel_views(8, U, V, seed=4, pan=0.7)
    out = oracle.render(dec, U, V, W, H, views, wo, ho)
    for k, (u, v, s, t) in enumerate(views.astype(np.float64)):
        X = np.arange(wo)
        Y = np.arange(ho)
        sx = np.clip(s + (X + 0.5) * W / wo - 0.5, 0, W - 1)[None, :]
        ty = np.clip(t + (Y + 0.5) * H / ho - 0.5, 0, H - 1)[:, None]
        val = a + bu * u + bv * v + bx * sx + by * ty + u * sx
        assert np.all(np.abs(out[k, 0] * 255.0 - val) <= 2e-3)
        # (the middle channel was halved and floored, so it is not multilinear)
        assert np.all(np.abs(out[k, 2] * 255.0 - (255 - val)) <= 2e-3)


# -- refocusing (reading C20) -------------------------------------------------

def lambertian_plane(U, V, W, H, delta, seed):
    """Views of one textured plane whose image moves by delta pixels per
    camera step: view (i, j) at pixel (x, y) shows base[y + delta j, x + delta i]."""
    r = np.random.default_rng(seed)
    base = r.integers(0, 256, (H + delta * (V - 1), W + delta * (U - 1), 3), dtype=np.uint8)
    lf = np.zeros((V, U, H, W, 3), dtype=np.uint8)
    for j in range(V):
        for i in range(U):
            lf[j, i] = base[delta * j: delta * j + H, delta * i: delta * i + W]
    return lf, base


def test_refocus_on_a_plane_reproduces_it_sharply():
    # focused at d = -delta, the four source views agree on every ray: a
    # camera half-way between grid positions (u = 1.5, v = 2.5 with delta = 2)
    # sees base[y + delta v, x + delta u], an integer pixel of the plane
    U, V, W, H, delta = 4, 4, 24, 20, 2
    lf, base = lambertian_plane(U, V, W, H, delta, 5)
    dec = encode_decode(lf, U, V, W, H)
    u, v = 1.5, 2.5
    out = oracle.render(dec, U, V, W, H, np.array([[u, v, 0, 0]], dtype=np.float32), W, H,
                        disparity=-float(delta))[0]
    ox, oy = int(delta * u), int(delta * v)
    # interior pixels, where every source view's sample lies inside its image
    want = base[oy + 1: oy + H - 1, ox + 1: ox + W - 1].transpose(2, 0, 1).astype(np.float32) / 255.0
    assert np.array_equal(out[:, 1:H - 1, 1:W - 1], want)
    # without refocusing the same camera blends four different pixels
    plain = oracle.render(dec, U, V, W, H, np.array([[u, v, 0, 0]], dtype=np.float32), W, H)[0]
    assert not np.array_equal(plain[:, 1:H - 1, 1:W - 1], want)


def test_refocus_leaves_grid_cameras_and_zero_disparity_unchanged():
    U, V, W, H = 4, 3, 16, 12
    lf = synth.light_field(synth.LFSpec(U, V, W, H, 3, 1.0, 2.0, 19), threads=1)
    dec = encode_decode(lf, U, V, W, H)
    # a camera on the grid weights one source view by 1 and its own shift is 0;
    # below the last row and column the other weights are exactly 0 (lerp at
    # fraction 0), on them the lerp at fraction 1 rounds
    grid = np.array([[u, v, 0.25, -0.5] for v in range(V) for u in range(U)], dtype=np.float32)
    inner = (grid[:, 0] < U - 1) & (grid[:, 1] < V - 1)
    for d in (-3.0, 0.7, 5.0):
        got = oracle.render(dec, U, V, W, H, grid, 20, 9, disparity=d)
        ref = oracle.render(dec, U, V, W, H, grid, 20, 9)
        assert np.array_equal(got[inner], ref[inner])
        assert np.abs(got - ref).max() <= 1e-6
    # a camera off the grid is the camera clamped to the grid, shift included
    off = np.array([[-1.5, 0.5, 0.3, 0.0], [U + 0.7, V - 1.2, -0.4, 1.0]], dtype=np.float32)
    on = off.copy()
    on[:, 0] = np.clip(on[:, 0], 0, U - 1)
    on[:, 1] = np.clip(on[:, 1], 0, V - 1)
    assert np.array_equal(oracle.render(dec, U, V, W, H, off, 20, 9, disparity=2.5),
                          oracle.render(dec, U, V, W, H, on, 20, 9, disparity=2.5))
    views = synth.novel_views(6, U, V, seed=4, pan=2.0)
    a = oracle.render(dec, U, V, W, H, views, 20, 9)
    b = oracle.render(dec, U, V, W, H, views, 20, 9, disparity=1e-30)   # the general path, vanishing shift
    assert np.array_equal(a, b)
