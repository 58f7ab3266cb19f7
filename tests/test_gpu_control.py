"""GPU tests of the learned encoder control: the network's inference,
gradient and Adam kernels against the oracle (oracle/mlp.py), and the
encoder's network mode.

Tolerances follow the arithmetic: the kernels accumulate in float32 in an
order of their own, the oracle in float64, on the same bfloat16 weights.
Logits and gradients agree to 1e-4 relative to their scale; an argmax is
taken as a decision of float32 arithmetic, so the kernel's class must be
the oracle's wherever the oracle's top two logits differ by more than 1e-3,
and elsewhere must be within 1e-3 of the top.  The encoder's network mode
must give exactly the stream the oracle encodes from the classes and ranges
the library reports using, and that stream must decode bit-exactly on the
GPU; with a confidence floor above 1 every row falls back to the search.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as omlp
from helpers import say
from paper_1805_06019_amd import control, lfc, synth

pytestmark = pytest.mark.gpu


def rand_net(seed, scale=1.0):
    w = control.init_weights(seed) * scale
    w[1024:1088] = np.random.default_rng(seed).normal(0, 0.1, 64)     # nonzero biases too
    bits = control.to_bf16_bits(w)
    return torch.from_numpy(bits.view(np.int16)).cuda(), omlp.from_bf16_bits(bits).astype(np.float64)


def rand_rows(n, seed):
    r = np.random.default_rng(seed)
    x = r.uniform(0, 1, (n, 16)).astype(np.float32)
    return x, r.integers(0, 10, n).astype(np.int8), r.integers(0, 27, n).astype(np.int8)


@pytest.mark.parametrize("n", [1, 63, 256, 1000, 70_001])
def test_inference_matches_oracle(gpu, n):
    say("mlp infer", n)
    wt, w = rand_net(3)
    x, _, _ = rand_rows(n, 4)
    cls, rng, conf, z = lfc.mlp_infer(wt, torch.from_numpy(x).cuda(), logits=True)
    z = z.cpu().numpy()
    z64, _, _ = omlp.forward(w, x)
    scale = max(1.0, float(np.abs(z64).max()))
    assert np.abs(z - z64).max() <= 1e-4 * scale
    ct, cr, conf_o, z32 = omlp.predict(w, x)
    for got, head in ((cls.cpu().numpy(), z32[:, :10]), (rng.cpu().numpy(), z32[:, 10:])):
        top2 = np.sort(head, axis=1)[:, -2:]
        clear = top2[:, 1] - top2[:, 0] > 1e-3
        assert (got[clear] == np.argmax(head, axis=1)[clear]).all()
        assert (head[np.arange(n), got.astype(np.int64)] >= head.max(axis=1) - 1e-3).all()
    assert np.abs(conf.cpu().numpy() - conf_o).max() <= 1e-4


@pytest.mark.parametrize("n", [1, 127, 128, 129, 1000])
def test_gradient_matches_oracle(gpu, n):
    say("mlp grad", n)
    wt, w = rand_net(5)
    x, c, r = rand_rows(n, 6)
    grad, loss = lfc.mlp_grad(wt, torch.from_numpy(x).cuda(), torch.from_numpy(c).cuda(), torch.from_numpy(r).cuda())
    l64, g64 = omlp.loss_and_grad(w, x.astype(np.float64), c.astype(np.int64), r.astype(np.int64))
    g = grad.cpu().numpy().astype(np.float64)
    assert abs(float(loss.cpu()[0]) - l64) <= 1e-4 * max(1.0, abs(l64))
    assert np.abs(g - g64).max() <= 1e-4 * max(1e-3, np.abs(g64).max())
    assert np.linalg.norm(g - g64) <= 1e-4 * np.linalg.norm(g64)


def test_bad_labels_give_nan_loss(gpu):
    wt, _ = rand_net(5)
    x, c, r = rand_rows(10, 6)
    c[3] = 10
    _, loss = lfc.mlp_grad(wt, torch.from_numpy(x).cuda(), torch.from_numpy(c).cuda(), torch.from_numpy(r).cuda())
    assert np.isnan(float(loss.cpu()[0]))


def test_adam_matches_oracle_and_rounds_to_bf16(gpu):
    r = np.random.default_rng(7)
    master = r.normal(size=lfc.MLP_PARAMS).astype(np.float32)
    m = (r.normal(size=lfc.MLP_PARAMS) * 0.01).astype(np.float32)
    v = (r.uniform(size=lfc.MLP_PARAMS) * 1e-4).astype(np.float32)
    g = r.normal(size=lfc.MLP_PARAMS).astype(np.float32)
    tm, tmm, tv, tg = (torch.from_numpy(a.copy()).cuda() for a in (master, m, v, g))
    tw = torch.zeros(lfc.MLP_PARAMS, dtype=torch.int16, device="cuda")
    lfc.mlp_adam(tm, tw, tmm, tv, tg, 5, 1e-3)
    # the kernel takes its hyperparameters as float32: the oracle gets the same values
    f32 = lambda x: float(np.float32(x))
    om, omm, ov, _ = omlp.adam(master.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                               g.astype(np.float64), 5, f32(1e-3), f32(0.9), f32(0.999), f32(1e-8))
    got = tm.cpu().numpy()
    assert np.abs(got - om).max() <= 1e-6
    assert np.abs(tmm.cpu().numpy() - omm).max() <= 1e-6 * np.abs(omm).max()
    assert np.abs(tv.cpu().numpy() - ov).max() <= 1e-6 * np.abs(ov).max()
    # the bf16 copy is the kernel's own master rounded to nearest even
    assert np.array_equal(tw.cpu().numpy().view(np.uint16), omlp.bf16_bits(got))


def test_training_lowers_the_loss_on_a_learnable_task(gpu):
    # labels are a fixed function of the features: the threshold class from
    # feature 2 and the range class from feature 3
    r = np.random.default_rng(8)
    x = r.uniform(0, 1, (40_000, 16)).astype(np.float32)
    c = np.minimum((x[:, 2] * 10).astype(np.int8), 9)
    g = np.minimum((x[:, 3] * 27).astype(np.int8), 26)
    tr = control.Trainer(seed=9, lr=3e-3)
    curve, _ = tr.fit(x, c, g, epochs=6, batch=512, log=lambda *a: None)
    say("curve", curve)
    assert curve[-1] < 0.5 * curve[0]
    acc_c, acc_r = control.accuracy(tr.w, x[:5000], c[:5000], g[:5000])
    assert acc_c > 0.8 and acc_r > 0.3     # chance: 0.1 and 0.037


def small_field():
    U, V, W, H = 6, 6, 48, 40
    rgb = synth.light_field(synth.LFSpec(U, V, W, H, 3, 1.5, 2.0, 61), threads=1)
    kw = dict(block=4, levels=3, cluster=(2, 3), quant_bits=1)
    return rgb, oracle.Params(U, V, W, H, **kw), lfc.Params(U, V, W, H, **kw)


def test_network_mode_stream_is_the_oracles_replay_and_decodes_bit_exactly(gpu):
    rgb, p, P = small_field()
    lam = 1 << 18
    # a network trained briefly on this field's own search labels
    _, st = lfc.lfc_encode_ctl(rgb, P, lfc.CTL_SEARCH, lam, want_features=True, want_stream=False)
    tr = control.Trainer(seed=10)
    tr.fit(st["features"], st["classes"], st["ranges"], epochs=20, batch=256, log=lambda *a: None)
    data, st2 = lfc.lfc_encode_ctl(rgb, P, lfc.CTL_MLP, lam, mlp=tr.w, want_features=True, want_search=True)
    say("network mode: fallbacks", st2["fallbacks"], "agreement", float((st2["classes"] == st2["search_classes"]).mean()))
    # the top residual level codes against the lossless key views in both modes: same features
    g = oracle.geometry(p)
    top = g.lu[1] * g.lv[1] * g.nb * 3
    assert np.array_equal(st2["features"][:top], st["features"][:top])
    enc, _, _, _ = oracle.encode_ctl(rgb, p, oracle.CTL_TABLE, classes=st2["classes"], ranges=st2["ranges"])
    assert data == enc.stream
    lf = lfc.lfc_open(data)
    got = lfc.lfc_decode_blocks(lf, None, lfc.LAYOUT_IMAGES).cpu().numpy()
    assert np.array_equal(got, enc.r0)
    assert np.array_equal(got, oracle.decode_all(data))
    lf.close()
    # the classes the network chose are the kernel's argmax on these features
    feats = torch.from_numpy(st2["features"]).cuda()
    pc, pr, _ = lfc.mlp_infer(tr.w, feats)
    same = st2["classes"] == pc.cpu().numpy()
    assert same.mean() > 0.99     # the rest are int16 fallbacks or masked ranges
    # a confidence floor above 1 sends every row to the search
    data3, st3 = lfc.lfc_encode_ctl(rgb, P, lfc.CTL_MLP, lam, mlp=tr.w, min_confidence=1.01)
    ref, _ = lfc.lfc_encode_ctl(rgb, P, lfc.CTL_SEARCH, lam)
    assert data3 == ref and st3["fallbacks"] == lfc.lfc_control_rows(P)


@pytest.mark.parametrize("n", [1, 31, 33, 1000, 100_003])
def test_bf16_matrix_core_inference_matches_oracle(gpu, n):
    # the oracle rounds the inputs and both hidden layers to bf16 as the
    # kernel does and sums in float64; the kernel's float32 sums can put a
    # hidden value on the other side of a bf16 rounding boundary (one bf16
    # step, 2^-8 relative), so most logits agree to 1e-3 of their scale and
    # all to 2e-2; decisions agree wherever the oracle's margin is clear
    say("mlp infer bf16", n)
    wt, w = rand_net(13)
    x, _, _ = rand_rows(n, 14)
    cls, rng, conf, z = lfc.mlp_infer(wt, torch.from_numpy(x).cuda(), logits=True, precision=lfc.MLP_BF16)
    z = z.cpu().numpy().astype(np.float64)
    ref = omlp.forward_bf16(w, x)
    scale = max(1.0, float(np.abs(ref).max()))
    err = np.abs(z - ref)
    assert err.max() <= 2e-2 * scale and np.quantile(err, 0.99) <= 1e-3 * scale
    for got, head in ((cls.cpu().numpy(), ref[:, :10]), (rng.cpu().numpy(), ref[:, 10:])):
        top2 = np.sort(head, axis=1)[:, -2:]
        clear = top2[:, 1] - top2[:, 0] > 0.05 * scale
        assert (got[clear] == np.argmax(head, axis=1)[clear]).all()
    e = np.exp(ref[:, :10] - ref[:, :10].max(axis=1, keepdims=True))
    assert np.abs(conf.cpu().numpy() - 1 / e.sum(axis=1)).max() <= 2e-2
    # the fp32 path agrees on clear decisions too
    c32, _, _ = lfc.mlp_infer(wt, torch.from_numpy(x).cuda())
    top2 = np.sort(ref[:, :10], axis=1)[:, -2:]
    clear = top2[:, 1] - top2[:, 0] > 0.05 * scale
    assert (c32.cpu().numpy()[clear] == cls.cpu().numpy()[clear]).all()
    with pytest.raises(lfc.LFCError):
        lfc.mlp_infer(wt, torch.from_numpy(x).cuda(), precision=7)
