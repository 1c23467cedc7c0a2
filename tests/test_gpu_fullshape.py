"""GPU: batched registration at the full sizes of the batched workloads, against the oracle.

batch256: 256 pairs in one call, N ~ U{500..5000}, inlier ratio ~ U[2 %, 30 %], K1 = 500, K2 = 2.
outdoor16: 16 pairs of N = 20000 (1 % inliers, tau = theta = 0.6 m), K1 = 2500, K2 = 2.
Both run with plain pivots and with the learned scorer (the committed weights). These are the
first shapes whose C and SC2-weight arenas hold more than 2^31 entries, so the int64 offset
arithmetic of every stage is exercised on pairs placed beyond that point.

Every pair's outputs are compared with the oracle run on the same inputs (pivots, cliques,
inlier numbers, selection and mask exactly; poses within the pose bar); the two N x N taps (C
and the weights) are compared in full for the first pair, the last pair and the first pair
whose arena offset is at least 2^31 entries.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2507_01439_amd import synth
from paper_2507_01439_amd import turboreg as T
from parity import POSE_M, POSE_RAD, check_taps, rot_angle, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2507_01439_amd",
                       "weights", "scorer_indoor.bin")
ARENA_2_31 = 1 << 31


def arena_offsets(ns):
    """Entry offsets of each pair's C / weight matrix in the arenas: pairs packed by npad^2."""
    npad = [(n + 255) // 256 * 256 for n in ns]
    return np.concatenate([[0], np.cumsum([p * p for p in npad])])[:-1].astype(np.int64)


def workload(name):
    if name == "batch256":
        cfgs = synth.batch_configs(256, seed=2, n_lo=500, n_hi=5000)
        pairs = [synth.make_pair(c.replace(k1=500), synth.pair_seed(2, b)) for b, c in enumerate(cfgs)]
        return pairs, pairs[0].cfg.replace(n=5000, k1=500)
    cfg = synth.CONFIGS["outdoor_n20000"]
    return [synth.make_pair(cfg, synth.pair_seed(4, b)) for b in range(16)], cfg


def run_batch(name, learned):
    pairs, cfg = workload(name)
    ns = [p.src.shape[0] for p in pairs]
    offs = np.concatenate([[0], np.cumsum(ns)]).astype(np.int32)
    reg = T.Registrar(max_n=max(ns), max_batch=len(pairs), max_k1=cfg.k1, max_k2=cfg.k2)
    if learned:
        with open(WEIGHTS, "rb") as f:
            T.tr_scorer_load(reg.h, f.read())
    prm = T.make_params(cfg.tau, cfg.theta, cfg.k1, cfg.k2,
                        pivot_mode=T.TR_PIVOTS_LEARNED if learned else T.TR_PIVOTS_PLAIN, pool_factor=4)
    src = np.concatenate([p.src for p in pairs])
    dst = np.concatenate([p.dst for p in pairs])
    say(f"{name} learned={learned}: {len(pairs)} pairs, N {min(ns)}..{max(ns)}, "
        f"last arena offset {arena_offsets(ns)[-1]}")
    out, masks = reg.register_batch(to_dev(torch, src), to_dev(torch, dst), to_dev(torch, offs), prm,
                                    max_n=max(ns))
    torch.cuda.synchronize()
    res = T.parse_results(out, len(pairs))
    return dict(reg=reg, pairs=pairs, cfg=cfg, prm=prm, res=res, masks=masks.cpu().numpy(), offs=offs, ns=ns)


def tapped(ns):
    """First pair, last pair and the first pair whose arena offset reaches 2^31 entries."""
    beyond = int(np.argmax(arena_offsets(ns) >= ARENA_2_31))
    assert arena_offsets(ns)[beyond] >= ARENA_2_31, "the workload does not reach 2^31 arena entries"
    return {"first": 0, "beyond_2_31": beyond, "last": len(ns) - 1}


def check_dense(run, b):
    """Every stage of pair b against the oracle, the N x N taps (and in learned mode the
    features of the scored rows) included."""
    prev = oracle.set_threaded(True)
    try:
        p, r = run["pairs"][b], run["res"][b]
        o0, o1 = run["offs"][b], run["offs"][b + 1]
        say(f"  pair {b} n={run['ns'][b]} (all taps)")
        assert r.status in (T.TR_OK, T.TR_ERR_NO_HYPOTHESIS), (b, r.status)
        check_taps(run["reg"], p.src, p.dst, run["prm"], r, run["masks"][o0:o1], pair=b, label=f"pair {b}")
    finally:
        oracle.set_threaded(prev)


def check_records(run, which):
    """The result record, mask, pivots, cliques, poses and inlier numbers of the pairs `which`
    against the oracle's whole path (run with the GPU's learned scores in learned mode, and
    scoring the GPU's float32 poses, on which inlier numbers are defined)."""
    reg, prm = run["reg"], run["prm"]
    learned = prm.pivot_mode == T.TR_PIVOTS_LEARNED
    for b in which:
        p, r = run["pairs"][b], run["res"][b]
        mask = run["masks"][run["offs"][b]:run["offs"][b + 1]]
        poses = reg.debug(T.TR_TAP_POSES, b)
        scores = reg.debug(T.TR_TAP_SCORES, b) if learned else None
        ro, mo, o = oracle.register_ex(p.src, p.dst, prm.tau, prm.inlier_thresh, prm.k1, prm.k2,
                                       pool_factor=prm.pool_factor if learned else 0, scores=scores,
                                       poses=poses, threaded=True)
        lab = f"pair {b} n={run['ns'][b]}"
        assert np.array_equal(reg.debug(T.TR_TAP_PIVOTS, b), o["pivots"]), lab
        assert np.array_equal(reg.debug(T.TR_TAP_CLIQUES, b), o["cliques"]), lab
        for h in np.nonzero(o["flags"] == 1)[0]:
            assert rot_angle(poses[h, :9].reshape(3, 3), o["R"][h]) <= POSE_RAD, (lab, h)
            assert np.abs(poses[h, 9:].astype(np.float64) - o["t"][h]).max() <= POSE_M, (lab, h)
        assert np.array_equal(reg.debug(T.TR_TAP_IN, b), o["IN"]), lab
        assert (r.best_hyp, r.best_inliers, r.n_valid_hyp, r.n_pivots, r.n_boundary_pairs) == \
            (ro.best_hyp, ro.best_inliers, ro.n_valid_hyp, ro.n_pivots, ro.n_boundary32), lab
        want_status = T.TR_OK if ro.status == 0 else T.TR_ERR_NO_HYPOTHESIS
        assert r.status == want_status, (lab, r.status, ro.status)
        assert np.array_equal(np.array(r.R, np.float32), np.array(ro.R32, np.float32)), lab
        assert np.array_equal(np.array(r.t, np.float32), np.array(ro.t32, np.float32)), lab
        assert np.array_equal(mask, mo), lab


class _Batch:
    name, learned = None, False

    @pytest.fixture(scope="class")
    def run(self):
        assert torch.cuda.is_available(), "GPU tests need a ROCm device"
        if self.learned and not os.path.exists(WEIGHTS):
            pytest.skip("no committed scorer weights")
        r = run_batch(self.name, self.learned)
        yield r
        r["reg"].close()

    @pytest.mark.parametrize("which", ["first", "beyond_2_31", "last"])
    def test_taps(self, run, which):
        check_dense(run, tapped(run["ns"])[which])

    @pytest.mark.parametrize("part", range(4))
    def test_every_pair(self, run, part):
        B = len(run["pairs"])
        if part == 0:
            ok = [synth.success(np.array(r.R).reshape(3, 3), np.array(r.t), p)
                  for r, p in zip(run["res"], run["pairs"])]
            say(f"  success rate {np.mean(ok):.3f}")
        which = range(part * B // 4, (part + 1) * B // 4)
        say(f"  pairs {which.start}..{which.stop - 1}")
        check_records(run, which)


class TestBatch256Plain(_Batch):
    name, learned = "batch256", False


class TestBatch256Learned(_Batch):
    name, learned = "batch256", True


class TestOutdoor16Plain(_Batch):
    name, learned = "outdoor16", False


class TestOutdoor16Learned(_Batch):
    name, learned = "outdoor16", True
