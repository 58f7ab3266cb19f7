"""Pins of the oracle's per-block encoder control and of its network, and
the library's host encoder checked against the oracle.

The per-block search minimises w_c * SSE * 2^16 + lambda * rate over the
threshold classes.  Pins from the definition, none of them a restatement of
the cost: at lambda = 0 the least-distortion class is the unthresholded one
(rounding quantiser: zeroing a residual never reduces the error), so the
stream equals the paper's global encoder with both thresholds 0; at the
largest lambda every block is dropped; on a two-level tree (parents are
the lossless key views, so the blocks' choices are independent) the total
rate falls and the weighted distortion rises as lambda grows, and the
search's total cost is at most that of any single global pixel threshold;
a block with a single unit residual is kept exactly while lambda is below
the closed form w 2^16 / (5 + payload bits).  The features are pinned on
blocks whose statistics are known by hand (residual spread, a flat parent, a
horizontal ramp).

The network's oracle (oracle/mlp.py) is pinned by bfloat16 rounding cases,
a forward pass on hand-set weights, the gradient against central finite
differences and Adam's first step.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_1805_06019_amd import lfc, synth

TAUS = [0, 2, 3, 4, 5, 6, 8, 12, 16]
CASES = [
    # U, V, W, H, kw
    (4, 4, 32, 24, dict(block=4, levels=2, cluster=(2,), quant_bits=1)),
    (6, 3, 30, 10, dict(block=2, levels=3, cluster=(2, 2))),
    (5, 4, 40, 24, dict(block=8, levels=2, cluster=(3,), quant_bits=2)),
    (9, 9, 24, 20, dict(block=4, levels=3, cluster=(2, 2), quant_bits=2, range_mask=0x3FFFFFF & ~0x7F000)),
]


def lf_of(U, V, W, H, seed):
    return synth.light_field(synth.LFSpec(U, V, W, H, 3, 1.5, 2.0, seed), threads=1)


def body(stream):
    """The stream without the two threshold fields of its header (bytes
    72..79), which record the parameters and not the coded data."""
    return stream[:72] + stream[80:]


def weighted_sse(ycc, r0):
    d = (ycc.astype(np.int64) - r0.astype(np.int64)) ** 2
    return int(6 * d[:, 0].sum() + d[:, 1].sum() + d[:, 2].sum())


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}x{c[3]}-B{c[4]['block']}" for c in CASES])
def test_search_at_zero_lambda_is_the_unthresholded_encoder(case):
    U, V, W, H, kw = case
    rgb = lf_of(U, V, W, H, 11 + U)
    p = oracle.Params(U, V, W, H, **kw)
    enc, cls, rng, _ = oracle.encode_ctl(rgb, p, oracle.CTL_SEARCH, 0)
    assert enc.stream == oracle.encode(rgb, p).stream        # pix 0, blk 0
    assert (cls == 0).all()


@pytest.mark.parametrize("case", CASES[:2])
def test_search_at_largest_lambda_drops_everything(case):
    U, V, W, H, kw = case
    rgb = lf_of(U, V, W, H, 12 + U)
    p = oracle.Params(U, V, W, H, **kw)
    enc, cls, rng, _ = oracle.encode_ctl(rgb, p, oracle.CTL_SEARCH, 1 << 52)
    drop = oracle.Params(U, V, W, H, **{**kw, "blk_threshold": 2 ** 31 - 1})
    assert body(enc.stream) == body(oracle.encode(rgb, drop).stream)
    # every block absent (a class that thresholds a block away ties with the
    # drop and, being lower, is the one recorded)
    assert (rng == 26).all() and (cls == 9).any()
    # the same through a table of drops and of absent ranges
    rows = oracle.control_rows(p)
    t1, _, _, _ = oracle.encode_ctl(rgb, p, oracle.CTL_TABLE, classes=np.full(rows, 9), ranges=np.zeros(rows))
    t2, _, _, _ = oracle.encode_ctl(rgb, p, oracle.CTL_TABLE, classes=np.zeros(rows), ranges=np.full(rows, 26))
    assert t1.stream == enc.stream and t2.stream == enc.stream


def test_search_rate_distortion_monotone_and_below_every_global_threshold():
    U, V, W, H = 6, 6, 48, 40
    rgb = lf_of(U, V, W, H, 21)
    kw = dict(block=4, levels=2, cluster=(3,), quant_bits=1)
    p = oracle.Params(U, V, W, H, **kw)
    ycc = oracle.encode(rgb, p).ycocg
    S = 16
    bits = np.array([5 + oracle.bise_bits(k, S) for k in range(26)] + [0])
    prev_rate, prev_dist = None, None
    for lam in [0, 1 << 12, 1 << 16, 1 << 18, 1 << 20, 1 << 22, 1 << 26]:
        enc, cls, rng, _ = oracle.encode_ctl(rgb, p, oracle.CTL_SEARCH, lam)
        rate = int(bits[rng.astype(np.int64)].sum())
        dist = weighted_sse(ycc, enc.r0)
        assert rate == int((enc.hist * bits[:26]).sum())
        if prev_rate is not None:
            assert rate <= prev_rate and dist >= prev_dist, lam
        prev_rate, prev_dist = rate, dist
        # no single global pixel threshold does better at this lambda
        cost = dist * 65536 + lam * rate
        for tau in TAUS:
            g = oracle.encode(rgb, oracle.Params(U, V, W, H, **kw, pix_threshold=tau))
            gcost = weighted_sse(ycc, g.r0) * 65536 + lam * int((g.hist * bits[:26]).sum())
            assert cost <= gcost, (lam, tau)


def test_table_replays_the_search_and_clamps_into_a_given_range():
    U, V, W, H, kw = CASES[0]
    rgb = lf_of(U, V, W, H, 31)
    p = oracle.Params(U, V, W, H, **kw)
    enc, cls, rng, _ = oracle.encode_ctl(rgb, p, oracle.CTL_SEARCH, 1 << 18)
    rep, c2, r2, _ = oracle.encode_ctl(rgb, p, oracle.CTL_TABLE, classes=cls, ranges=rng)
    assert rep.stream == enc.stream and (c2 == cls).all() and (r2 == rng).all()
    # range code 0 holds zigzag values 0 and 1 (residuals 0 and -1): every
    # stored value becomes 0 or -1 and the decoded residual never exceeds it
    rows = oracle.control_rows(p)
    small, _, r3, _ = oracle.encode_ctl(rgb, p, oracle.CTL_TABLE, classes=np.zeros(rows), ranges=np.zeros(rows))
    assert set(np.unique(r3)) <= {0, 26}
    q = kw["quant_bits"]
    base = oracle.encode(rgb, oracle.Params(U, V, W, H, **{**kw, "blk_threshold": 2 ** 31 - 1}))
    d = small.r0.astype(np.int32) - base.r0.astype(np.int32)
    assert set(np.unique(d)) <= {0, -(1 << q)}


def test_features_on_blocks_with_known_statistics():
    # two grey views in one cluster: Y = 100 and 110, Co = Cg = 0; the key view
    # is their mean 105, so every residual is -5 or +5 and the parent is flat
    rgb = np.zeros((1, 2, 8, 8, 3), dtype=np.uint8)
    rgb[0, 0] = 100
    rgb[0, 1] = 110
    p = oracle.Params(2, 1, 8, 8, block=4, levels=2, cluster=(2,), quant_bits=2)
    lam = 3 << 16
    _, _, _, f = oracle.encode_ctl(rgb, p, oracle.CTL_SEARCH, lam, want_features=True)
    f = f.reshape(2, 4, 3, 16)   # node, block, channel
    y = f[:, :, 0]
    assert np.allclose(y[..., 0], 0) and np.allclose(y[..., 1], 1)
    assert np.allclose(y[..., 2], np.log2(6) / 8) and np.allclose(y[..., 3], np.log2(6) / 8)
    assert np.allclose(y[..., 4], 0)                               # |r| constant
    assert np.allclose(y[..., 5:7], 1) and np.allclose(y[..., 7:9], 0)
    assert np.allclose(y[..., 9:13], 0)                            # flat parent
    assert np.allclose(f[..., 13], 0.5) and np.allclose(f[..., 14], 2 / 24) and np.allclose(f[..., 15], 0.5)
    chroma = f[:, :, 1:]
    assert np.allclose(chroma[..., 1:13], 0)


def test_single_unit_residuals_are_kept_exactly_below_their_closed_form_lambda():
    # two grey views in one cluster differ at one pixel (100 vs 102): the key
    # view holds 101 there, so each view's block carries one unit residual in
    # Y.  -1 has zigzag value 1: range code 0 (2 values, 16 payload bits); +1
    # has zigzag value 2: code 12 (a trit and no low bits, 3 values, ceil(8 *
    # 16 / 5) = 26 bits).  Keeping costs lambda * (5 + payload bits), dropping
    # costs 6 * 1 * 2^16, so a block is kept exactly while lambda < 393216 / 21
    # = 18724.6 (view 0) or 393216 / 31 = 12684.4 (view 1).
    rgb = np.full((1, 2, 4, 4, 3), 100, dtype=np.uint8)
    rgb[0, 1, 2, 1] = 102
    p = oracle.Params(2, 1, 4, 4, block=4, levels=2, cluster=(2,))
    for lam, keep0, keep1 in ((10000, True, True), (12684, True, True), (12685, True, False),
                              (13500, True, False), (18724, True, False), (18725, False, False),
                              (20000, False, False)):
        _, cls, rng, _ = oracle.encode_ctl(rgb, p, oracle.CTL_SEARCH, lam)
        y = rng.reshape(2, 1, 3)[:, 0, 0]          # node, block, channel
        assert (y[0] != 26) == keep0 and (y[1] != 26) == keep1, lam
        if keep0:
            assert y[0] == 0
        if keep1:
            assert y[1] == 12


def test_gradient_features_follow_the_parent_axes():
    # identical views of a horizontal ramp (Y = 10 + 4x): zero residuals, the
    # parent has horizontal steps of 4 and no vertical change
    x = np.arange(8)
    img = np.repeat((10 + 4 * x)[None, :, None], 8, axis=0).repeat(3, axis=2).astype(np.uint8)
    rgb = np.stack([img, img])[None]
    p = oracle.Params(2, 1, 8, 8, block=4, levels=2, cluster=(2,))
    _, _, _, f = oracle.encode_ctl(rgb, p, oracle.CTL_SEARCH, 0, want_features=True)
    y = f.reshape(2, 4, 3, 16)[:, :, 0]
    assert np.allclose(y[..., 2:9], 0)                               # no residual
    assert np.allclose(y[..., 9], np.log2(5) / 8) and np.allclose(y[..., 10], 0)
    assert np.allclose(y[..., 11], np.log2(5) / 8)
    # variance of a 4-wide ramp with steps of 4 (values a, a+4, a+8, a+12 on every row): 20
    assert np.allclose(y[..., 12], np.log2(21) / 16)


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}x{c[3]}-B{c[4]['block']}" for c in CASES])
def test_library_search_table_and_features_equal_the_oracle(case):
    U, V, W, H, kw = case
    rgb = lf_of(U, V, W, H, 41 + U)
    p = oracle.Params(U, V, W, H, **kw)
    P = lfc.Params(U, V, W, H, **kw)
    assert lfc.lfc_control_rows(P) == oracle.control_rows(p)
    for lam in (0, 1 << 16, 1 << 19, 1 << 23):
        enc, cls, rng, feat = oracle.encode_ctl(rgb, p, oracle.CTL_SEARCH, lam, want_features=True)
        data, st = lfc.lfc_encode_ctl(rgb, P, lfc.CTL_SEARCH, lam, want_features=True, want_search=True)
        assert data == enc.stream, lam
        assert (st["classes"] == cls).all() and (st["ranges"] == rng).all()
        assert (st["search_classes"] == cls).all() and (st["search_ranges"] == rng).all()
        assert np.array_equal(st["features"], feat)
    # a table of mixed classes and ranges, clamping included
    r = np.random.default_rng(U)
    rows = oracle.control_rows(p)
    allowed = [k for k in range(26) if not kw.get("range_mask") or (kw["range_mask"] >> k) & 1] + [26]
    tc = r.integers(0, 10, rows).astype(np.int8)
    tr = r.choice(allowed, rows).astype(np.int8)
    enc, _, _, _ = oracle.encode_ctl(rgb, p, oracle.CTL_TABLE, classes=tc, ranges=tr)
    data, st = lfc.lfc_encode_ctl(rgb, P, lfc.CTL_TABLE, classes=tc, ranges=tr)
    assert data == enc.stream


def test_library_control_argument_errors():
    U, V, W, H, kw = CASES[0]
    rgb = lf_of(U, V, W, H, 51)
    P = lfc.Params(U, V, W, H, **kw)
    rows = lfc.lfc_control_rows(P)
    with pytest.raises(lfc.LFCError):
        lfc.lfc_encode_ctl(rgb, P, 7)
    with pytest.raises(lfc.LFCError):
        lfc.lfc_encode_ctl(rgb, P, lfc.CTL_SEARCH, -1)
    with pytest.raises(lfc.LFCError):
        lfc.lfc_encode_ctl(rgb, P, lfc.CTL_SEARCH, (1 << 52) + 1)
    with pytest.raises(lfc.LFCError):
        lfc.lfc_encode_ctl(rgb, P, lfc.CTL_TABLE, classes=np.full(rows, 10), ranges=np.zeros(rows))
    with pytest.raises(lfc.LFCError):
        lfc.lfc_encode_ctl(rgb, P, lfc.CTL_TABLE, classes=np.zeros(rows), ranges=np.full(rows, 27))
    masked = lfc.Params(U, V, W, H, **{**kw, "range_mask": 0x3FFFFFE})
    with pytest.raises(lfc.LFCError):
        lfc.lfc_encode_ctl(rgb, masked, lfc.CTL_TABLE, classes=np.zeros(rows), ranges=np.zeros(rows))
    with pytest.raises(lfc.LFCError):
        lfc.lfc_encode_ctl(rgb, P, lfc.CTL_MLP)          # no weights
    with pytest.raises(ValueError):
        lfc.lfc_encode_ctl(rgb, P, lfc.CTL_TABLE, classes=np.zeros(rows - 1), ranges=np.zeros(rows - 1))
    with pytest.raises(lfc.LFCError):
        lfc.lfc_control_rows(lfc.Params(U, V, W, H, block=3, levels=2, cluster=(2,)))


# -- the network's oracle ------------------------------------------------------

def test_bf16_rounding_cases():
    one = 1.0
    cases = [(1.0, 1.0), (one + 2 ** -8, 1.0), (one + 3 * 2 ** -8, one + 2 ** -6),
             (one + 2 ** -8 + 2 ** -20, one + 2 ** -7), (-(one + 2 ** -8 + 2 ** -20), -(one + 2 ** -7)),
             (3.4e38, np.inf), (np.inf, np.inf), (0.0, 0.0), (2 ** -130, 2 ** -130)]
    x = np.array([c[0] for c in cases], dtype=np.float32)
    got = omlp.bf16_round(x)
    assert np.array_equal(got, np.array([c[1] for c in cases], dtype=np.float32))
    assert np.isnan(omlp.bf16_round(np.array([np.nan], dtype=np.float32)))[0]
    assert np.array_equal(omlp.from_bf16_bits(omlp.bf16_bits(x)), got)


def test_forward_on_hand_set_weights():
    # layer 1 copies features 0..15 into units 0..15, layer 2 copies units,
    # threshold logit k = feature k, range logit j = 2 * feature 0 - j
    p = {name: np.zeros(shape) for name, shape in omlp.SHAPES}
    p["W1"][:16, :16] = np.eye(16)
    p["W2"][:16, :16] = np.eye(16)
    p["W3"][:10, :10] = np.eye(10)
    p["W3"][10:, 0] = 2.0
    p["b3"][10:] = -np.arange(27)
    # biases: unit 20 of layer 2 is its bias 0.75, unit 21 twice layer 1's
    # unit 30 (bias 0.5); they feed threshold logits 9 and 8
    p["b2"][20] = 0.75
    p["b1"][30] = 0.5
    p["W2"][21, 30] = 2.0
    p["W3"][9, 9], p["W3"][9, 20] = 0.0, 1.0
    p["W3"][8, 8], p["W3"][8, 21] = 0.0, 1.0
    w = omlp.pack(p)
    x = np.abs(np.random.default_rng(1).normal(size=(5, 16))) + 0.1
    z, h1, h2 = omlp.forward(w, x)
    assert np.allclose(z[:, :8], x[:, :8]) and np.allclose(z[:, 10:], 2 * x[:, :1] - np.arange(27))
    assert np.allclose(z[:, 9], 0.75) and np.allclose(z[:, 8], 1.0)
    p["W3"][9, 9], p["W3"][9, 20] = 1.0, 0.0
    p["W3"][8, 8], p["W3"][8, 21] = 1.0, 0.0
    w = omlp.pack(p)
    x2 = x.copy()
    x2[:, 3] = -1.0     # ReLU cuts it
    assert np.allclose(omlp.forward(w, x2)[0][:, 3], 0.0)
    ct, cr, conf, _ = omlp.predict(w, x)
    assert (ct == np.argmax(x[:, :10], axis=1)).all() and (cr == 0).all()
    e = np.exp(x[:, :10] - x[:, :10].max(axis=1, keepdims=True))
    assert np.allclose(conf, 1 / e.sum(axis=1), rtol=1e-5)


def test_gradient_matches_central_differences():
    r = np.random.default_rng(2)
    w = r.normal(scale=0.3, size=omlp.N_PARAMS)
    x = r.normal(size=(7, 16))
    cls, rng = r.integers(0, 10, 7), r.integers(0, 27, 7)
    l0, g = omlp.loss_and_grad(w, x, cls, rng)
    assert abs(l0 - omlp.loss(w, x, cls, rng)) < 1e-12
    h = 1e-6
    for i in r.choice(omlp.N_PARAMS, 60, replace=False):
        e = np.zeros(omlp.N_PARAMS)
        e[i] = h
        num = (omlp.loss(w + e, x, cls, rng) - omlp.loss(w - e, x, cls, rng)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 + 1e-5 * abs(num), i


def test_adam_first_step_moves_each_weight_by_lr_against_its_gradient_sign():
    r = np.random.default_rng(3)
    master = r.normal(size=omlp.N_PARAMS)
    g = r.normal(size=omlp.N_PARAMS)
    new, m, v, bits = omlp.adam(master, np.zeros_like(master), np.zeros_like(master), g, 1, 1e-3)
    # bias correction makes the first moments g and g^2: a step of lr * g / (|g| + eps)
    assert np.allclose(new - master, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    assert np.array_equal(omlp.from_bf16_bits(bits), omlp.bf16_round(new.astype(np.float32)))
