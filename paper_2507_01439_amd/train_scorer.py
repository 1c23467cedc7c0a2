"""Train the learned pivot scorer with the library's own GPU kernels.

Pairs are drawn from the generator (N ~ U{1000..5000}, inlier ratio ~ U[2%, 30%],
indoor geometry, seeds disjoint from every evaluation seed); per-match features
come from `tr_features_batch`; labels are the generator's inlier flags. The MLP
is trained by `tr_train_step` (BF16 forward/backward with float32 accumulation,
Adam on float32 master weights) on shuffled minibatches and saved as the
checksummed weights blob `tr_scorer_save` writes.

    python -m paper_2507_01439_amd.train_scorer --pairs 100000 --out weights/scorer_indoor.bin
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2507_01439_amd import synth  # noqa: E402
from paper_2507_01439_amd import turboreg as T  # noqa: E402

TRAIN_SALT = 11   # seeds of training pairs: synth.pair_seed(3, index, TRAIN_SALT)


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases (TR_MLP_NPARAM float32, library order)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((19, 64), (64, 64), (64, 1)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-lim, lim, size=(fan_out, fan_in)).reshape(-1))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def build_features(reg, torch, n_pairs, batch, seed0, log):
    """Features (M x 19 bfloat16 bits, int16 tensor) and labels (M uint8) of n_pairs generated pairs."""
    base = synth.CONFIGS["indoor_n1000"]
    rng = np.random.default_rng(seed0)
    ns = rng.integers(1000, 5001, size=n_pairs)
    ratios = rng.uniform(0.02, 0.30, size=n_pairs)
    total = int(ns.sum())
    feat = torch.empty((total, 19), dtype=torch.int16, device="cuda")
    labels = torch.empty(total, dtype=torch.uint8, device="cuda")
    prm = T.make_params(base.tau, base.theta, 1, 1)
    row = 0
    t0 = time.time()
    for b0 in range(0, n_pairs, batch):
        pairs = [synth.make_pair(base.replace(n=int(ns[b]), inlier_ratio=float(ratios[b])),
                                 synth.pair_seed(3, b, TRAIN_SALT)) for b in range(b0, min(n_pairs, b0 + batch))]
        cnt = [p.src.shape[0] for p in pairs]
        offs = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
        src = torch.from_numpy(np.concatenate([p.src for p in pairs])).cuda()
        dst = torch.from_numpy(np.concatenate([p.dst for p in pairs])).cuda()
        m = int(offs[-1])
        T.tr_features_batch(reg.h, src, dst, torch.from_numpy(offs).cuda(), len(pairs), 5000, prm,
                            feat[row:row + m])
        labels[row:row + m] = torch.from_numpy(np.concatenate([p.labels for p in pairs]).astype(np.uint8)).cuda()
        row += m
        if (b0 // batch) % 50 == 0:
            log(f"features: {b0 + len(pairs)}/{n_pairs} pairs, {row} matches, {time.time() - t0:.1f}s")
    torch.cuda.synchronize()
    return feat, labels


def train(args):
    import torch
    log = (lambda s: print(s, flush=True))
    reg = T.Registrar(max_n=5000, max_batch=args.batch, max_k1=1, max_k2=1)
    T.tr_scorer_set(reg.h, init_params(args.seed))
    feat, labels = build_features(reg, torch, args.pairs, args.batch, args.seed, log)
    M = feat.shape[0]
    log(f"training on {M} matches ({float(labels.float().mean()):.3f} inliers)")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed)
    mb = args.minibatch
    xb = torch.empty((mb, 19), dtype=torch.int16, device="cuda")
    yb = torch.empty(mb, dtype=torch.uint8, device="cuda")
    step = 0
    t0 = time.time()
    for epoch in range(args.epochs):
        perm = torch.randperm(M, device="cuda", generator=g)
        acc, cnt = 0.0, 0
        for s in range(0, M - mb + 1, mb):
            idx = perm[s:s + mb]
            torch.index_select(feat, 0, idx, out=xb)
            torch.index_select(labels, 0, idx, out=yb)
            lr = args.lr * (0.1 if epoch == args.epochs - 1 and args.epochs > 1 else 1.0)
            T.tr_train_step(reg.h, xb, yb, mb, lr, loss)
            step += 1
            if step % 200 == 0:
                acc += float(loss.item())
                cnt += 1
            if step % 2000 == 0:
                log(f"epoch {epoch} step {step} loss {acc / max(cnt, 1):.4f} ({time.time() - t0:.1f}s)")
                acc, cnt = 0.0, 0
    blob = T.tr_scorer_save(reg.h)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    with open(args.out, "wb") as f:
        f.write(blob)
    log(f"saved {args.out} ({len(blob)} bytes) after {step} steps")
    reg.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--pairs", type=int, default=100000)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--minibatch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                                                  "scorer_indoor.bin"))
    train(ap.parse_args())


if __name__ == "__main__":
    main()
