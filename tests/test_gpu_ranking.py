"""GPU: hypothesis selection by the error-based scores (MAE and MSE forms).

Everything before the scoring is unchanged by the ranking flag, so C, the
weights, pivots, cliques, poses and inlier numbers must equal the inlier-number
run bit for bit. The scores are float32 sums in the kernel's order against the
oracle's float64 sums: within a relative 2e-5. The selected hypothesis must
score the oracle's maximum (within that tolerance), its inlier number, pose and
mask must follow from it, and a repeated call must give the same bits.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2507_01439_amd import synth
from paper_2507_01439_amd import turboreg as T
from parity import run_single, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

RTOL, ATOL = 2e-5, 1e-5
METRICS = {T.TR_FLAG_RANK_MAE: oracle.METRIC_MAE, T.TR_FLAG_RANK_MSE: oracle.METRIC_MSE}
UPSTREAM = (T.TR_TAP_C, T.TR_TAP_G, T.TR_TAP_PIVOTS, T.TR_TAP_CLIQUES, T.TR_TAP_POSES, T.TR_TAP_IN)


@pytest.fixture(scope="module")
def reg():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    r = T.Registrar(max_n=5000, max_batch=6, max_k1=1000, max_k2=3)
    yield r
    r.close()


def check_ranked(reg, p, prm_in, flag, label, pair=0, r=None, mask=None):
    theta = prm_in.inlier_thresh
    if r is None:
        r0, _ = run_single(reg, torch, p.src, p.dst, prm_in)
        ref = [reg.debug(t) for t in UPSTREAM]
        prm = T.make_params(prm_in.tau, theta, prm_in.k1, prm_in.k2, flags=flag)
        r, mask = run_single(reg, torch, p.src, p.dst, prm)
        for t, a in zip(UPSTREAM, ref):
            assert np.array_equal(reg.debug(t), a), (label, t)
        s1 = reg.debug(T.TR_TAP_RANK_SCORES)
        run_single(reg, torch, p.src, p.dst, prm)   # the same call again: the same bits
        assert np.array_equal(reg.debug(T.TR_TAP_RANK_SCORES).view(np.uint32), s1.view(np.uint32)), label
    poses = reg.debug(T.TR_TAP_POSES, pair)
    IN = reg.debug(T.TR_TAP_IN, pair)
    S = reg.debug(T.TR_TAP_RANK_SCORES, pair)
    valid = (IN >= 0).astype(np.int32)
    So = oracle.score_metric(p.src, p.dst, poses, valid, theta, METRICS[flag])
    assert np.array_equal(S[valid == 0], np.full(int((valid == 0).sum()), -1, np.float32)), label
    ok = valid == 1
    err = np.abs(S[ok].astype(np.float64) - So[ok]) / (ATOL + RTOL * np.abs(So[ok]))
    assert err.max(initial=0) <= 1.0, (label, float(err.max()))
    hg = r.best_hyp
    if ok.any():
        best = float(So.max())
        assert hg >= 0 and valid[hg] and So[hg] >= best - (ATOL + RTOL * best), (label, hg, So[hg], best)
        order = np.sort(So[ok])[::-1]
        if order.size > 1 and order[0] - order[1] > 2 * (ATOL + RTOL * order[0]):
            assert hg == oracle.select_score(So), label
        assert r.best_inliers == IN[hg], label
        assert np.array_equal(np.array(r.R, np.float32), poses[hg, :9]), label
        assert np.array_equal(mask[:p.src.shape[0]], oracle.mask(p.src, p.dst, poses[hg], theta)), label
    else:
        assert hg == -1
    return dict(best=hg, score=float(S[hg]) if hg >= 0 else None)


@pytest.mark.parametrize("flag", [T.TR_FLAG_RANK_MAE, T.TR_FLAG_RANK_MSE])
@pytest.mark.parametrize("wl,seed", [("indoor_n1000", 0), ("indoor_n1000", 1), ("indoor_n5000", 0)])
def test_ranked_selection_matches_oracle(reg, flag, wl, seed):
    cfg = synth.CONFIGS[wl]
    p = synth.make_pair(cfg, synth.pair_seed(7, seed))
    say(f"ranking {flag} {wl} seed {seed}")
    d = check_ranked(reg, p, T.params_from_config(cfg), flag, f"{wl} {seed} {flag}")
    say(d)


def test_ranked_k2_three_and_low_inlier_ratio(reg):
    cfg = synth.CONFIGS["indoor_n1000"].replace(n=2000, inlier_ratio=0.02, k1=400, k2=3)
    p = synth.make_pair(cfg, synth.pair_seed(7, 9))
    for flag in METRICS:
        check_ranked(reg, p, T.params_from_config(cfg), flag, f"k2=3 {flag}")


def test_ranked_batch_equals_single(reg):
    ns = [900, 1500, 2, 640, 1200]
    pairs = [synth.make_pair(synth.CONFIGS["indoor_n1000"].replace(n=max(n, 3), inlier_ratio=0.1),
                             synth.pair_seed(7, 20 + b)) for b, n in enumerate(ns)]
    src = np.concatenate([q.src[:n] for q, n in zip(pairs, ns)])
    dst = np.concatenate([q.dst[:n] for q, n in zip(pairs, ns)])
    offs = to_dev(torch, np.concatenate([[0], np.cumsum(ns)]).astype(np.int32))
    prm = T.make_params(0.1, 0.1, 300, 2, flags=T.TR_FLAG_RANK_MSE)
    out, masks = reg.register_batch(to_dev(torch, src), to_dev(torch, dst), offs, prm, max_n=max(ns))
    torch.cuda.synchronize()
    res = T.parse_results(out, len(ns))
    masks = masks.cpu().numpy()
    assert res[2].status == T.TR_ERR_INVALID_ARG
    off = np.concatenate([[0], np.cumsum(ns)])
    live = [b for b, n in enumerate(ns) if n >= 3]
    cut = {b: dataclasses.replace(pairs[b], src=pairs[b].src[:ns[b]], dst=pairs[b].dst[:ns[b]]) for b in live}
    for b in live:   # every pair's taps of the batch call first
        check_ranked(reg, cut[b], prm, T.TR_FLAG_RANK_MSE, f"batch pair {b}", pair=b, r=res[b],
                     mask=masks[off[b]:off[b + 1]])
    for b in live:
        single, smask = run_single(reg, torch, cut[b].src, cut[b].dst, prm)
        assert bytes(single) == bytes(res[b]) and np.array_equal(smask[:ns[b]], masks[off[b]:off[b + 1]]), b


def test_both_rankings_rejected(reg):
    p = synth.make_pair(synth.CONFIGS["indoor_n1000"], synth.pair_seed(7, 3))
    prm = T.make_params(0.1, 0.1, 100, 2, flags=T.TR_FLAG_RANK_MAE | T.TR_FLAG_RANK_MSE)
    with pytest.raises(T.TurboRegError) as e:
        run_single(reg, torch, p.src, p.dst, prm)
    assert e.value.status == T.TR_ERR_INVALID_ARG


@pytest.mark.parametrize("metric", [0, 1, 2])
def test_score_poses_matches_registration_and_oracle(reg, metric):
    cfg = synth.CONFIGS["indoor_n1000"].replace(n=1700, k1=300)
    p = synth.make_pair(cfg, synth.pair_seed(7, 40))
    flag = {0: 0, 1: T.TR_FLAG_RANK_MAE, 2: T.TR_FLAG_RANK_MSE}[metric]
    prm = T.make_params(cfg.tau, cfg.theta, cfg.k1, cfg.k2, flags=flag)
    run_single(reg, torch, p.src, p.dst, prm)
    poses, IN = reg.debug(T.TR_TAP_POSES), reg.debug(T.TR_TAP_IN)
    S = reg.debug(T.TR_TAP_RANK_SCORES) if metric else None
    # the hypothesis poses and the generator's pose, scored by the entry point
    R, t = np.asarray(p.R, np.float64), np.asarray(p.t, np.float64)
    gt = np.concatenate([R.reshape(9), t]).astype(np.float32)[None]
    allp = np.concatenate([poses, gt]).astype(np.float32)
    P = allp.shape[0]
    src, dst = to_dev(torch, p.src), to_dev(torch, p.dst)
    pin = torch.full((P,), -7, dtype=torch.int32, device="cuda")
    psc = torch.full((P,), -7.0, dtype=torch.float32, device="cuda")
    T.tr_score_poses(reg.h, src, dst, cfg.n, to_dev(torch, allp), P, cfg.theta, metric, pin, psc if metric else None)
    torch.cuda.synchronize()
    pin, psc = pin.cpu().numpy(), psc.cpu().numpy()
    ok = IN >= 0
    assert np.array_equal(pin[:-1][ok], IN[ok])
    if metric:
        assert np.array_equal(psc[:-1][ok].view(np.uint32), S[ok].view(np.uint32))   # the same bits
        so = oracle.score_metric(p.src, p.dst, gt, np.ones(1, np.int32), cfg.theta, metric)[0]
        assert abs(psc[-1] - so) <= ATOL + RTOL * abs(so)
    else:
        assert np.all(psc == -7.0)   # untouched
    assert pin[-1] == oracle.score(p.src, p.dst, gt, np.ones(1, np.int32), cfg.theta)[0]


def test_score_poses_argument_errors(reg):
    x = torch.zeros((5, 3), dtype=torch.float32, device="cuda")
    poses = torch.zeros((2, 12), dtype=torch.float32, device="cuda")
    out = torch.zeros(2, dtype=torch.int32, device="cuda")
    sc = torch.zeros(2, dtype=torch.float32, device="cuda")
    for args in [(0, 0.1, 0, sc), (5, 0.1, 3, sc), (5, 0.1, 1, None), (5, -1.0, 0, sc), (5, float("nan"), 0, sc)]:
        n, th, m, s = args
        with pytest.raises(T.TurboRegError) as e:
            T.tr_score_poses(reg.h, x, x, n, poses, 2, th, m, out, s)
        assert e.value.status == T.TR_ERR_INVALID_ARG
    T.tr_score_poses(reg.h, x, x, 5, poses, 0, 0.1, 1, out, sc)   # no poses: nothing to do


def test_ranking_recalls_on_generated_pairs(reg):
    from paper_2507_01439_amd import diagnostics
    base = synth.CONFIGS["indoor_n1000"].replace(n=1500, inlier_ratio=0.03)
    pairs = [synth.make_pair(base, synth.pair_seed(7, 60 + b)) for b in range(4)]
    for name in diagnostics.RANKINGS:
        t = diagnostics.ranking_recalls(reg, torch, pairs, k1=300, ranking=name)
        say(name, t)
        assert all(0.0 <= v <= 1.0 for v in t.values())
        assert t["TKRR@2"] >= t["RR"] and t["TKRR@50"] >= t["TKRR@5"] >= t["TKRR@3"] >= t["TKRR@2"]
