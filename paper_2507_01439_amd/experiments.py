"""Synthetic reruns of the paper's ablations on generated pairs (their trends, not
their numbers: the paper measures on 3DMatch / 3DLoMatch, which are absent).

  correct_hypotheses  our side of the correct-hypothesis counts (Table 8): of the
                      H = K1*K2 hypotheses of a registration, how many poses are
                      successful registrations, and how many cliques hold three inliers;
  sweep               success rate and correct-hypothesis counts as tau, K1 or K2
                      varies (the trends of Table 5);
  clique_discrepancy  3-clique against 10-clique pose estimates as tau varies
                      (Appendix A.2): 10-cliques of the compatibility graph, one
                      least-squares pose from all ten matches, and the
                      registration's own 3-point fit (tr_fit_triplets) for each of the
                      120 triplets; rotation and translation differences.

    python -m paper_2507_01439_amd.experiments
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2507_01439_amd import synth  # noqa: E402
from paper_2507_01439_amd import turboreg as T  # noqa: E402


def _register(reg, torch, p, tau, theta, k1, k2):
    n = p.src.shape[0]
    src, dst = torch.from_numpy(p.src).cuda(), torch.from_numpy(p.dst).cuda()
    out = torch.empty(80, dtype=torch.uint8, device="cuda")
    mask = torch.empty(n, dtype=torch.uint8, device="cuda")
    T.tr_register(reg.h, src, dst, n, T.make_params(tau, theta, k1, k2), out, mask)
    torch.cuda.synchronize()
    return T.parse_results(out)[0]


def _counts(reg, p):
    """(successful hypothesis poses, all-inlier cliques) of the last registration."""
    IN, poses, cl = reg.debug(T.TR_TAP_IN), reg.debug(T.TR_TAP_POSES), reg.debug(T.TR_TAP_CLIQUES)
    good = sum(synth.success(poses[h, :9].reshape(3, 3), poses[h, 9:], p) for h in np.nonzero(IN >= 0)[0])
    lab = np.asarray(p.labels)
    ok = (cl >= 0).all(1)
    pure = int((ok & lab[np.where(cl >= 0, cl, 0)].all(1)).sum())
    return int(good), pure


def correct_hypotheses(reg, torch, pairs, hs=(100, 200, 500, 1000, 2000), k2=2):
    out = {}
    for H in hs:
        good = pure = 0
        for p in pairs:
            _register(reg, torch, p, p.cfg.tau, p.cfg.theta, H // k2, k2)
            g, q = _counts(reg, p)
            good += g
            pure += q
        out[H] = {"successful_poses": good / len(pairs), "inlier_cliques": pure / len(pairs)}
    return out


def sweep_point(reg, torch, pairs, tau, k1, k2):
    """Success rate and successful hypothesis poses per pair at one (tau, K1, K2)."""
    ok = good = 0
    for p in pairs:
        r = _register(reg, torch, p, tau, p.cfg.theta, k1, k2)
        ok += r.best_hyp >= 0 and synth.success(np.array(r.R).reshape(3, 3), np.array(r.t), p)
        good += _counts(reg, p)[0]
    return {"success_rate": ok / len(pairs), "successful_poses": good / len(pairs)}


def sweep(reg, torch, pairs, taus=(0.025, 0.05, 0.1, 0.2, 0.4), k1s=(125, 250, 500, 1000),
          k2s=(1, 2, 3, 5, 8), tau0=0.1, k10=1000, k20=2):
    def run(tau, k1, k2):
        return sweep_point(reg, torch, pairs, tau, k1, k2)
    return {"tau": {t: run(t, k10, k20) for t in taus}, "k1": {k: run(tau0, k, k20) for k in k1s},
            "k2": {k: run(tau0, k10, k) for k in k2s}}


def _kabsch64(P, Q):
    """Least-squares rotation and translation of matched point sets (SVD, float64)."""
    pc, qc = P.mean(0), Q.mean(0)
    U, _, Vt = np.linalg.svd((P - pc).T @ (Q - qc))
    D = np.diag([1.0, 1.0, np.sign(np.linalg.det(Vt.T @ U.T))])
    R = Vt.T @ D @ U.T
    return R, qc - R @ pc


def _ten_cliques(C, rng, want, size=10, attempts=2000):
    """Cliques of `size` matches of the compatibility graph C (any matches, inliers or not), grown
    greedily from random seeds: each step adds the first match, in a random order, that is
    compatible with every member so far."""
    n = C.shape[0]
    Cb = C.astype(bool)
    found, seen = [], set()
    for _ in range(attempts):
        if len(found) >= want:
            break
        order = rng.permutation(n)
        clique = [int(order[0])]
        cand = Cb[order[0]][order].copy()   # candidates, in the permuted order
        while len(clique) < size and cand.any():
            k = int(np.argmax(cand))
            v = int(order[k])
            clique.append(v)
            cand &= Cb[v][order]
            cand[k] = False
        key = tuple(sorted(clique))
        if len(clique) == size and key not in seen:
            seen.add(key)
            found.append(key)
    return found


def clique_discrepancy(reg, torch, taus=(0.01, 0.1, 0.5, 1.0), n=2000, ratio=0.1, sigma=0.005, cliques=20, seed=3):
    base = synth.CONFIGS["indoor_n1000"].replace(n=n, inlier_ratio=ratio, sigma=sigma)
    p = synth.make_pair(base, synth.pair_seed(9, seed))
    src, dst = torch.from_numpy(p.src).cuda(), torch.from_numpy(p.dst).cuda()
    trip = np.array(list(itertools.combinations(range(10), 3)), np.int32)
    out = {}
    for tau in taus:
        _register(reg, torch, p, tau, tau, 100, 2)
        C = reg.debug(T.TR_TAP_C)
        found = _ten_cliques(C, np.random.default_rng(seed), cliques)
        dr, dt = [], []
        for cl in found:
            cl = np.array(cl, np.int32)
            R10, t10 = _kabsch64(p.src[cl].astype(np.float64), p.dst[cl].astype(np.float64))
            tri = torch.from_numpy(cl[trip].copy()).cuda()
            poses = torch.empty((len(trip), 12), dtype=torch.float32, device="cuda")
            ok = torch.empty(len(trip), dtype=torch.int32, device="cuda")
            T.tr_fit_triplets(reg.h, src, dst, n, tri, len(trip), poses, ok)
            torch.cuda.synchronize()
            poses, ok = poses.cpu().numpy().astype(np.float64), ok.cpu().numpy()
            for k in np.nonzero(ok)[0]:
                R3, t3 = poses[k, :9].reshape(3, 3), poses[k, 9:]
                c = (np.trace(R10.T @ R3) - 1.0) / 2.0
                dr.append(math.degrees(math.acos(max(-1.0, min(1.0, c)))))
                dt.append(float(np.linalg.norm(t10 - t3)))
        q = lambda a, f: float(np.quantile(a, f)) if a else None  # noqa: E731
        pure = sum(all(p.labels[v] for v in cl) for cl in found)
        out[tau] = {"cliques": len(found), "inlier_cliques": pure, "fits": len(dr),
                    "rot_deg_median": q(dr, 0.5), "rot_deg_p95": q(dr, 0.95),
                    "trans_m_median": q(dt, 0.5), "trans_m_p95": q(dt, 0.95)}
    return out


def main():
    import torch
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--pairs", type=int, default=16)
    args = ap.parse_args()
    base = synth.CONFIGS["indoor_n5000"]
    rng = np.random.default_rng(21)
    pairs = [synth.make_pair(base.replace(inlier_ratio=float(q)), synth.pair_seed(10, b))
             for b, q in enumerate(rng.uniform(0.01, 0.05, size=args.pairs))]
    reg = T.Registrar(max_n=base.n, max_batch=1, max_k1=1000, max_k2=8)
    res = {"pairs": args.pairs, "inlier_ratio": [0.01, 0.05],
           "correct_hypotheses": correct_hypotheses(reg, torch, pairs),
           "sweep": sweep(reg, torch, pairs),
           "clique_discrepancy": clique_discrepancy(reg, torch)}
    print(json.dumps(res), flush=True)
    reg.close()


if __name__ == "__main__":
    main()
