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
