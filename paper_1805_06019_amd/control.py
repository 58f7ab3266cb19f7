"""Learned encoder control: data, training and evaluation of the per-block
network (the GPU kernels and the encoder modes are in liblfc, include/lfc.h).

The paper's encoder uses one pixel threshold and one block-energy threshold
for every block (Sec. 3.2) and notes the lack of finer control (Sec. 5).
Here every residual block gets its own threshold class (and range class),
chosen by an exhaustive rate-distortion search (the labeller, the fallback
and the reference for rate and quality) or predicted by a small network trained on the search's
labels.  The decoder does not change.

    python -m paper_1805_06019_amd.control [--rows N] [--epochs E] [--quick]

prints one JSON record: the training curve and, at 40 and 50 dB on a light
field not seen in training, the bits per pixel of the global thresholds,
the search and the network.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import lfc, synth
from .workloads import FULL_SPEC

# the range of lambda_q16 the training labels are drawn from (2^10 .. 2^26)
LOG2_LAMBDA = (10.0, 26.0)
# quantiser step per PSNR target (the global operating points of the 40 and
# 50 dB workloads use q = 2 and q = 1)
TARGETS = ((40.0, 2), (50.0, 1))


def collect(specs, params_of, n_rows: int, seed: int, log=print):
    """n_rows (features, threshold class, range class) rows labelled by the
    search, spread evenly over the light fields, the quantiser steps of
    TARGETS and lambda."""
    rng = np.random.default_rng(seed)
    per = int(math.ceil(n_rows / len(specs)))
    xs, cs, rs = [], [], []
    for i, spec in enumerate(specs):
        rgb = synth.light_field(spec)
        runs = [(q, int(2 ** rng.uniform(*LOG2_LAMBDA))) for _, q in TARGETS for _ in range(2)]
        for q, lam in runs:
            t = time.time()
            p = params_of(spec, q)
            _, st = lfc.lfc_encode_ctl(rgb, p, lfc.CTL_SEARCH, lam, want_features=True, want_stream=False)
            take = rng.choice(st["classes"].size, size=min(per // len(runs) + 1, st["classes"].size), replace=False)
            xs.append(st["features"][take])
            cs.append(st["classes"][take])
            rs.append(st["ranges"][take])
            log(f"labels: light field {i} q={q} lambda 2^{math.log2(lam):.1f}: {take.size} rows "
                f"({time.time() - t:.1f} s)")
    x = np.concatenate(xs)[:n_rows]
    return x, np.concatenate(cs)[:n_rows], np.concatenate(rs)[:n_rows]


def init_weights(seed: int) -> np.ndarray:
    """He-normal weights, zero biases (float32, packed as in include/lfc.h)."""
    r = np.random.default_rng(seed)
    parts = [r.normal(0, math.sqrt(2 / 16), 64 * 16), np.zeros(64), r.normal(0, math.sqrt(2 / 64), 64 * 64),
             np.zeros(64), r.normal(0, math.sqrt(1 / 64), 37 * 64), np.zeros(37)]
    return np.concatenate(parts).astype(np.float32)


def to_bf16_bits(w: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(w, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


class Trainer:
    """Adam on the GPU kernels: float32 master weights, bfloat16 copy."""

    def __init__(self, seed: int = 0, lr: float = 2e-3):
        import torch
        self.torch = torch
        w = init_weights(seed)
        self.master = torch.from_numpy(w).cuda()
        self.w = torch.from_numpy(to_bf16_bits(w).view(np.int16)).cuda()
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.step_no = 0
        self.lr = lr
        self.part = None

    def step(self, x, c, r):
        grad, loss = lfc.mlp_grad(self.w, x, c, r, part=self.part)
        self.step_no += 1
        lfc.mlp_adam(self.master, self.w, self.m, self.v, grad, self.step_no, self.lr)
        return loss

    def fit(self, x: np.ndarray, c: np.ndarray, r: np.ndarray, epochs: int, batch: int = 1024, seed: int = 0,
            log=print):
        torch = self.torch
        X = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
        Yc = torch.from_numpy(np.ascontiguousarray(c, dtype=np.int8)).cuda()
        Yr = torch.from_numpy(np.ascontiguousarray(r, dtype=np.int8)).cuda()
        n = X.shape[0]
        self.part = torch.empty(((batch + 127) // 128) * (lfc.MLP_PARAMS + 1), dtype=torch.float32, device="cuda")
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        curve = []
        t0 = time.time()
        for ep in range(epochs):
            perm = torch.randperm(n, device="cuda", generator=g)
            losses = []
            for b0 in range(0, n - batch + 1, batch):
                idx = perm[b0:b0 + batch]
                losses.append(self.step(X[idx].contiguous(), Yc[idx].contiguous(), Yr[idx].contiguous()))
            mean = float(torch.cat(losses).mean())
            curve.append(round(mean, 5))
            log(f"epoch {ep}: mean loss {mean:.4f}")
        torch.cuda.synchronize()
        return curve, time.time() - t0


def accuracy(w, x: np.ndarray, c: np.ndarray, r: np.ndarray):
    import torch
    X = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    pc, pr, _ = lfc.mlp_infer(w, X)
    return float((pc.cpu().numpy() == c).mean()), float((pr.cpu().numpy() == r).mean())


def bpp_at(rgb, p, target: float, mode: int, mlp=None, min_confidence: float = 0.0, iters: int = 12):
    """Bisects log2(lambda) for the largest lambda whose PSNR reaches the
    target; returns (bpp, psnr, lambda_q16, fallback fraction)."""
    npix = p.grid_u * p.grid_v * p.width * p.height
    rows = lfc.lfc_control_rows(p)

    def run(e):
        _, st = lfc.lfc_encode_ctl(rgb, p, mode, int(2 ** e), mlp=mlp, min_confidence=min_confidence,
                                   want_stream=False)
        return st

    lo, hi = 0.0, 40.0
    best = run(lo)
    if best["psnr"] < target:
        return None
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        st = run(mid)
        if st["psnr"] >= target:
            lo, best = mid, st
        else:
            hi = mid
    return (8.0 * best["stream_bytes"] / npix, best["psnr"], int(2 ** lo), best["fallbacks"] / rows)


def global_bpp_at(rgb, p, target: float, qs=(0, 1, 2)):
    """The paper's global thresholds: per quantiser step the largest block
    threshold reaching the target, best over the steps."""
    from .tune import search
    spec = synth.LFSpec(p.grid_u, p.grid_v, p.width, p.height, 0, 0, 0, 0)
    base = dict(block=p.block, levels=p.levels, cluster=tuple(p.cluster))
    best = search(rgb, spec, base, target, qs=qs, log=lambda *a: None)
    return None if best is None else (best[2], best[3], best[0], best[1])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--rows", type=int, default=1_000_000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--train-fields", type=int, default=4)
    ap.add_argument("--quick", action="store_true", help="small light fields (a smoke run)")
    args = ap.parse_args(argv)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    import torch  # noqa: F401  (device memory for the kernels)

    if args.quick:
        mk = lambda seed: synth.LFSpec(9, 9, 128, 128, 6, 3.0, 1.5, seed)
        base = dict(block=4, levels=3, cluster=(2, 3))
    else:
        mk = lambda seed: synth.LFSpec(FULL_SPEC.grid_u, FULL_SPEC.grid_v, FULL_SPEC.width, FULL_SPEC.height,
                                       FULL_SPEC.layers, FULL_SPEC.disparity, FULL_SPEC.noise_sigma, seed)
        base = dict(block=4, levels=3, cluster=(2, 3))
    params_of = lambda s, q: lfc.Params(s.grid_u, s.grid_v, s.width, s.height, quant_bits=q, **base)
    train_specs = [mk(700 + i) for i in range(args.train_fields)]
    t = time.time()
    x, c, r = collect(train_specs, params_of, args.rows, seed=1, log=log)
    label_s = time.time() - t
    n_val = min(len(x) // 10, 100_000)
    tr = Trainer(seed=2)
    curve, train_s = tr.fit(x[n_val:], c[n_val:], r[n_val:], args.epochs, log=log)
    acc_c, acc_r = accuracy(tr.w, x[:n_val], c[:n_val], r[:n_val])
    rec = dict(rows=int(len(x)), label_s=round(label_s, 1), epochs=args.epochs, train_s=round(train_s, 2),
               loss_curve=curve, val_accuracy=dict(threshold_class=round(acc_c, 4), range_class=round(acc_r, 4)),
               class_hist=np.bincount(c, minlength=10).tolist())
    test = mk(799)
    rgb = synth.light_field(test)
    rec["test_field"] = f"{test.grid_u}x{test.grid_v} views of {test.width}x{test.height}, seed {test.seed}"
    for target, q in TARGETS:
        p = params_of(test, q)
        row = {"quant_bits": q}
        g = global_bpp_at(rgb, p, target, qs=(q,))
        if g:
            row["global"] = dict(bpp=round(g[0], 4), psnr=round(g[1], 3), blk_threshold=g[3])
        s = bpp_at(rgb, p, target, lfc.CTL_SEARCH)
        if s:
            row["search"] = dict(bpp=round(s[0], 4), psnr=round(s[1], 3), lambda_q16=s[2])
        for conf in (0.0, 0.6):
            m = bpp_at(rgb, p, target, lfc.CTL_MLP, mlp=tr.w, min_confidence=conf)
            if m:
                row[f"mlp_conf{conf}"] = dict(bpp=round(m[0], 4), psnr=round(m[1], 3), lambda_q16=m[2],
                                              fallback_frac=round(m[3], 4))
        rec[f"{int(target)}dB"] = row
        log(f"{target} dB: {row}")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
