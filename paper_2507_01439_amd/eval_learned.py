"""Learned vs plain pivots at equal success rate on held-out pairs.

Held-out pairs use seeds disjoint from training. For each pivot mode and each
K1 of a sweep, every pair is registered on the GPU (one pair per call, inputs
resident) and judged a success by the workload's thresholds (RE <= 15 deg and
TE <= 0.3 m indoors, RE <= 5 deg and TE <= 0.6 m outdoors). The plain
method at the reference K1 fixes the target success rate; each mode's
operating point is its smallest K1 reaching that rate, and the two are
compared in registrations/s there.

    python -m paper_2507_01439_amd.eval_learned --weights weights/scorer_indoor.bin
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2507_01439_amd import synth  # noqa: E402
from paper_2507_01439_amd import turboreg as T  # noqa: E402

EVAL_SALT = 12
HARD_SALT = 13


def held_out(n_pairs, n_hard, n=5000, seed=5):
    base = synth.CONFIGS["indoor_n5000"]
    rng = np.random.default_rng(seed)
    pairs = [synth.make_pair(base.replace(n=n, inlier_ratio=float(r)), synth.pair_seed(3, b, EVAL_SALT))
             for b, r in enumerate(rng.uniform(0.02, 0.30, size=n_pairs))]
    hard = [synth.make_pair(base.replace(n=n, inlier_ratio=float(r)), synth.pair_seed(3, b, HARD_SALT))
            for b, r in enumerate(rng.uniform(0.005, 0.01, size=n_hard))]
    return pairs, hard


def run_mode(reg, torch, dev, pairs, k1, learned, pool_factor=4, reps=1):
    cfg = pairs[0].cfg   # tau, theta and the success thresholds of the workload
    prm = T.make_params(cfg.tau, cfg.theta, k1, 2, pivot_mode=T.TR_PIVOTS_LEARNED if learned else T.TR_PIVOTS_PLAIN,
                        pool_factor=pool_factor)
    outs = [torch.empty(80, dtype=torch.uint8, device="cuda") for _ in pairs]
    mask = torch.empty(max(p.src.shape[0] for p in pairs), dtype=torch.uint8, device="cuda")
    for (s, d), o in zip(dev, outs):                       # warm-up pass
        T.tr_register(reg.h, s, d, s.shape[0], prm, o, mask)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for (s, d), o in zip(dev, outs):
            T.tr_register(reg.h, s, d, s.shape[0], prm, o, mask)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = [T.parse_results(o)[0] for o in outs]
    ok = [synth.success(np.array(r.R).reshape(3, 3), np.array(r.t), p) for r, p in zip(res, pairs)]
    return float(np.mean(ok)), reps * len(pairs) / dt


def compare(reg, torch, pairs, k1_sweep=(8, 16, 32, 64, 125, 250, 500, 1000), ref_k1=1000, pool_factor=4, reps=1):
    dev = [(torch.from_numpy(p.src).cuda(), torch.from_numpy(p.dst).cuda()) for p in pairs]
    table = {"plain": {}, "learned": {}}
    for k1 in k1_sweep:
        for mode in ("plain", "learned"):
            sr, rate = run_mode(reg, torch, dev, pairs, k1, mode == "learned", pool_factor, reps)
            table[mode][k1] = {"success_rate": sr, "registrations_per_s": rate}
    target = table["plain"][ref_k1]["success_rate"]

    def operating(mode):
        for k1 in sorted(table[mode]):
            if table[mode][k1]["success_rate"] >= target:
                return k1
        return None
    op = {m: operating(m) for m in table}
    out = {"target_success_rate": target, "ref_k1": ref_k1, "table": table, "operating_k1": op}
    for m in table:
        out[f"{m}_registrations_per_s_at_target"] = table[m][op[m]]["registrations_per_s"] if op[m] else None
    return out


def main():
    import torch
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--weights", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                                                      "scorer_indoor.bin"))
    ap.add_argument("--pairs", type=int, default=256)
    ap.add_argument("--hard", type=int, default=64)
    args = ap.parse_args()
    reg = T.Registrar(max_n=5000, max_batch=1, max_k1=1000, max_k2=2)
    with open(args.weights, "rb") as f:
        T.tr_scorer_load(reg.h, f.read())
    pairs, hard = held_out(args.pairs, args.hard)
    res = {"held_out": compare(reg, torch, pairs), "hard_slice": compare(reg, torch, hard)}
    print(json.dumps(res), flush=True)
    reg.close()


if __name__ == "__main__":
    main()
