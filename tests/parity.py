"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and compare every intermediate with the CPU oracle on the same inputs."""
import math
import sys

import numpy as np

import oracle
from paper_2507_01439_amd import turboreg as T

POSE_RAD = 1e-4   # rotation tolerance vs the float64 oracle
POSE_M = 1e-4     # translation tolerance vs the float64 oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rot_angle(Ra, Rb):
    """Angle of Ra Rb^T, accurate for small angles: |Ra - Rb|_F = 2 sqrt(2) sin(theta / 2)."""
    d = np.linalg.norm(np.asarray(Ra, np.float64) - np.asarray(Rb, np.float64))
    return 2.0 * math.asin(min(1.0, d / (2.0 * math.sqrt(2.0))))


def to_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_single(reg, torch, X, Y, params):
    src, dst = to_dev(torch, X), to_dev(torch, Y)
    out, mask = reg.register(src, dst, params)
    torch.cuda.synchronize()
    r = T.parse_results(out)[0]
    return r, mask.cpu().numpy()


def check_taps(reg, X, Y, params, r, mask, pair=0, label="", dense=True):
    """Stage-by-stage comparison of pair `pair` of the last call with the oracle.
    dense=False skips the two N x N taps (C and the SC2 weights); the edge and
    boundary counts of the record, the pivots, cliques, poses, inlier numbers,
    selection and mask are still compared. Returns a dict of diagnostics
    (boundary counts, pose errors)."""
    tau, theta, k1, k2 = params.tau, params.inlier_thresh, params.k1, params.k2
    n = X.shape[0]
    Co, b32, b64, flips = oracle.compat(X, Y, tau)
    if dense:
        C = reg.debug(T.TR_TAP_C, pair)
        assert np.array_equal(C, Co), f"{label}: C differs at {np.argwhere(C != Co)[:5].tolist()}"
    assert r.n_boundary_pairs == b32, (label, r.n_boundary_pairs, b32)
    assert r.n_edges == int(Co.sum()) // 2, label
    Gh = oracle.sc2(Co)
    Gt = oracle.o2graph(Gh)
    if dense:
        G = reg.debug(T.TR_TAP_G, pair).astype(np.int32)
        Gu = np.triu(G, 1)
        del G
        assert np.array_equal(Gu, Gt), f"{label}: G differs at {np.argwhere(Gu != Gt)[:5].tolist()}"
        del Gu
    Gbar = Gt if params.graph == T.TR_GRAPH_O2 else Gh
    if params.pivot_mode == T.TR_PIVOTS_PLAIN:
        P = reg.debug(T.TR_TAP_PIVOTS, pair)
        Po, npv = oracle.pivots(Gbar if params.graph == T.TR_GRAPH_O2 else Gt, k1)
        assert np.array_equal(P, Po), f"{label}: pivots differ at {np.argwhere((P != Po).any(1))[:5].ravel().tolist()}"
        assert r.n_pivots == npv
    else:
        pool = k1 * params.pool_factor
        Pp = reg.debug(T.TR_TAP_PLAIN_PIVOTS, pair)
        Ppo, nppo = oracle.pivots(Gt, pool)
        assert np.array_equal(Pp, Ppo), f"{label}: plain pool differs"
        s = reg.debug(T.TR_TAP_SCORES, pair)
        if dense:
            # the features of the rows the scorer read (the plain pool's endpoints), bit-exact
            rows = np.unique(Pp[:, :2])
            rows = rows[rows >= 0]
            F = oracle.features(X, Y, tau, Co, Gh)[rows]
            u = F.astype(np.float32).view(np.uint32).astype(np.uint64)
            want = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)
            assert np.array_equal(reg.debug(T.TR_TAP_FEATURES, pair)[rows], want), f"{label}: features differ"
        Po, _ = oracle.pivots_learned(Ppo, s, k1)
        P = reg.debug(T.TR_TAP_PIVOTS, pair)
        assert np.array_equal(P, Po), f"{label}: learned pivots differ"
        npv = min(k1, nppo)
        assert r.n_pivots == npv
    cl = reg.debug(T.TR_TAP_CLIQUES, pair)
    clo = oracle.cliques(Gbar, Po, npv, k1, k2)
    assert np.array_equal(cl, clo), f"{label}: cliques differ at {np.argwhere((cl != clo).any(1))[:5].ravel().tolist()}"
    poses = reg.debug(T.TR_TAP_POSES, pair)
    R64, t64, flags = oracle.kabsch(X, Y, cl)
    worst_r = worst_t = 0.0
    for h in np.nonzero(flags == 1)[0]:
        Rg = poses[h, :9].reshape(3, 3)
        worst_r = max(worst_r, rot_angle(Rg, R64[h]))
        worst_t = max(worst_t, float(np.abs(poses[h, 9:].astype(np.float64) - t64[h]).max()))
    assert worst_r <= POSE_RAD and worst_t <= POSE_M, (label, worst_r, worst_t)
    IN = reg.debug(T.TR_TAP_IN, pair)
    INo = oracle.score(X, Y, poses, (flags != 0).astype(np.int32), theta)
    assert np.array_equal(IN, INo), f"{label}: IN differs at {np.nonzero(IN != INo)[0][:5].tolist()}"
    hb = oracle.select(INo)
    assert r.best_hyp == hb, (label, r.best_hyp, hb)
    assert r.n_valid_hyp == int((flags != 0).sum())
    if hb >= 0:
        assert r.best_inliers == INo[hb]
        assert np.array_equal(np.array(r.R, np.float32), poses[hb, :9]) and np.array_equal(np.array(r.t, np.float32), poses[hb, 9:])
        mo = oracle.mask(X, Y, poses[hb], theta)
        assert np.array_equal(mask[:n], mo), label
        assert r.status in (T.TR_OK, T.TR_ERR_NONFINITE, T.TR_WARN_SCORER_FALLBACK)
    else:
        assert r.status in (T.TR_ERR_NO_HYPOTHESIS, T.TR_ERR_NONFINITE) and not mask[:n].any()
    return dict(b32=b32, b64=b64, flips=flips, worst_rad=worst_r, worst_m=worst_t,
                ill=int((flags == 2).sum()), edges=r.n_edges)
