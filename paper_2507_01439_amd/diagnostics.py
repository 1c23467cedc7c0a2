"""Ranking-based registration recalls on generated pairs (the study of the
paper's supplementary Table 6: hypotheses ranked by inlier number, MAE or MSE).

For every pair the registration runs with the chosen ranking; its K1*K2
hypotheses are ranked by the same score (larger first, lower h on ties):

  RR      the selected pose is a successful registration;
  TQRR    the selected hypothesis scores at least as high as the generator's
          ground-truth pose, scored by tr_score_poses in the same arithmetic;
  ICRR    the selected hypothesis's clique holds three inliers (generator labels);
  TKRR@K  some hypothesis among the K best is a successful registration.

    python -m paper_2507_01439_amd.diagnostics --pairs 64
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2507_01439_amd import synth  # noqa: E402
from paper_2507_01439_amd import turboreg as T  # noqa: E402

RANKINGS = {"IN": (0, 0), "MSE": (T.TR_FLAG_RANK_MSE, 2), "MAE": (T.TR_FLAG_RANK_MAE, 1)}


def ranking_recalls(reg, torch, pairs, k1, k2=2, ranking="IN", ks=(2, 3, 5, 50)):
    flag, metric = RANKINGS[ranking]
    cfg = pairs[0].cfg
    prm = T.make_params(cfg.tau, cfg.theta, k1, k2, flags=flag)
    hits = {"RR": 0, "TQRR": 0, "ICRR": 0, **{f"TKRR@{k}": 0 for k in ks}}
    for p in pairs:
        n = p.src.shape[0]
        src, dst = torch.from_numpy(p.src).cuda(), torch.from_numpy(p.dst).cuda()
        out = torch.empty(80, dtype=torch.uint8, device="cuda")
        mask = torch.empty(n, dtype=torch.uint8, device="cuda")
        T.tr_register(reg.h, src, dst, n, prm, out, mask)
        torch.cuda.synchronize()
        r = T.parse_results(out)[0]
        IN, poses, cliques = reg.debug(T.TR_TAP_IN), reg.debug(T.TR_TAP_POSES), reg.debug(T.TR_TAP_CLIQUES)
        score = reg.debug(T.TR_TAP_RANK_SCORES) if metric else IN.astype(np.float64)
        valid = np.nonzero(IN >= 0)[0]
        order = valid[np.lexsort((valid, -score[valid]))]   # larger score first, then lower h
        if r.best_hyp < 0:
            continue
        assert order[0] == r.best_hyp
        ok = lambda h: synth.success(poses[h, :9].reshape(3, 3), poses[h, 9:], p)  # noqa: E731
        hits["RR"] += ok(r.best_hyp)
        # the ground-truth pose, scored like the hypotheses
        gt = np.concatenate([np.asarray(p.R).reshape(9), np.asarray(p.t)]).astype(np.float32)[None]
        gin = torch.empty(1, dtype=torch.int32, device="cuda")
        gsc = torch.empty(1, dtype=torch.float32, device="cuda")
        T.tr_score_poses(reg.h, src, dst, n, torch.from_numpy(gt).cuda(), 1, cfg.theta, metric, gin,
                         gsc if metric else None)
        torch.cuda.synchronize()
        g = float(gsc.item()) if metric else float(gin.item())
        hits["TQRR"] += score[r.best_hyp] >= g
        i, j, z = cliques[r.best_hyp]
        hits["ICRR"] += bool(p.labels[i] and p.labels[j] and z >= 0 and p.labels[z])
        good = [ok(h) for h in order[:max(ks)]]
        for k in ks:
            hits[f"TKRR@{k}"] += any(good[:k])
    return {k: v / len(pairs) for k, v in hits.items()}


def main():
    import torch
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--pairs", type=int, default=64)
    ap.add_argument("--k1", type=int, default=1000)
    ap.add_argument("--ratio-lo", type=float, default=0.005)
    ap.add_argument("--ratio-hi", type=float, default=0.02)
    args = ap.parse_args()
    base = synth.CONFIGS["indoor_n5000"]
    rng = np.random.default_rng(17)
    pairs = [synth.make_pair(base.replace(inlier_ratio=float(q)), synth.pair_seed(8, b))
             for b, q in enumerate(rng.uniform(args.ratio_lo, args.ratio_hi, size=args.pairs))]
    reg = T.Registrar(max_n=base.n, max_batch=1, max_k1=args.k1, max_k2=2)
    table = {name: ranking_recalls(reg, torch, pairs, args.k1, ranking=name) for name in RANKINGS}
    print(json.dumps({"pairs": args.pairs, "inlier_ratio": [args.ratio_lo, args.ratio_hi], "k1": args.k1,
                      "table": table}), flush=True)
    reg.close()


if __name__ == "__main__":
    main()
