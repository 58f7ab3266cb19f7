"""GPU encoder (CompressLFI, Alg. 1, on the GPU): the stream and the
statistics must equal the host encoder's byte for byte, which the host
encoder in turn shares with the oracle (tests/test_host_library.py), on
geometries covering block sizes 2/4/8, one to six levels, pixel and block
thresholds, quantiser steps, restricted range masks and ragged images; and
at full size.  A range mask that cannot hold a residual is an error.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import make_lf, say
from paper_1805_06019_amd import lfc, synth
from paper_1805_06019_amd.workloads import WORKLOADS

pytestmark = pytest.mark.gpu

CASES = [
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


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}x{c[3]}-B{c[4]['block']}-L{c[4]['levels']}"
                                             for c in CASES])
def test_gpu_encoder_equals_host_encoder(gpu, case):
    U, V, W, H, kw = case
    say("gpu encode", case)
    rgb = make_lf(U, V, W, H, seed=U * 17 + W)
    p = lfc.Params(U, V, W, H, **kw)
    host, hst = lfc.lfc_encode_ex(rgb, p)
    dev, dst = lfc.lfc_encode_gpu(rgb, p)
    assert dev == host
    assert dst == hst
    assert dev == oracle.encode(rgb, oracle.Params(U, V, W, H, **kw)).stream
    none, st2 = lfc.lfc_encode_gpu(rgb, p, want_stream=False)
    assert none is None and st2 == hst


def test_gpu_encoder_full_size(gpu):
    w = WORKLOADS["full40"]
    say("gpu encode full40")
    rgb = synth.light_field(w.spec)
    host, hst = lfc.lfc_encode_ex(rgb, w.params())
    d = torch.from_numpy(rgb).cuda()
    dev, dst = lfc.lfc_encode_gpu(d, w.params())
    assert dev == host and dst == hst


def test_gpu_encoder_errors(gpu):
    U, V, W, H = 4, 4, 16, 16
    rgb = make_lf(U, V, W, H, seed=3)
    # only a 2-value range allowed: residuals beyond it cannot be coded
    p = lfc.Params(U, V, W, H, block=4, levels=2, cluster=(2,), range_mask=1)
    with pytest.raises(lfc.LFCError) as e1:
        lfc.lfc_encode_ex(rgb, p)
    with pytest.raises(lfc.LFCError) as e2:
        lfc.lfc_encode_gpu(rgb, p)
    assert e1.value.status == e2.value.status == -5
    with pytest.raises(lfc.LFCError):
        lfc.lfc_encode_gpu(rgb, lfc.Params(U, V, W, H, block=3, levels=2, cluster=(2,)))
    with pytest.raises(ValueError):
        lfc.lfc_encode_gpu(rgb[:, :2], lfc.Params(U, V, W, H, block=4, levels=2, cluster=(2,)))
