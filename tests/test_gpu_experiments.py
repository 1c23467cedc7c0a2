"""GPU: the triplet-fit entry point against the oracle's fits, and the synthetic
ablation reruns (correct-hypothesis counts, tau/K1/K2 sweeps, 3- vs 10-clique
discrepancy) on small inputs."""
import numpy as np
import pytest

import oracle
from paper_2507_01439_amd import synth
from paper_2507_01439_amd import turboreg as T
from parity import POSE_M, POSE_RAD, rot_angle, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def reg():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    r = T.Registrar(max_n=2000, max_batch=1, max_k1=500, max_k2=8)
    yield r
    r.close()


def test_fit_triplets_matches_oracle(reg):
    p = synth.make_pair(synth.CONFIGS["indoor_n1000"], synth.pair_seed(11, 0))
    rng = np.random.default_rng(5)
    tri = rng.integers(0, 1000, (600, 3)).astype(np.int32)
    tri[:5] = [[1, 1, 2], [3, 3, 3], [-1, 2, 3], [0, 1, 1000], [7, 8, 9]]   # repeats, out of range
    poses = torch.empty((600, 12), dtype=torch.float32, device="cuda")
    ok = torch.empty(600, dtype=torch.int32, device="cuda")
    T.tr_fit_triplets(reg.h, to_dev(torch, p.src), to_dev(torch, p.dst), 1000, to_dev(torch, tri), 600, poses, ok)
    torch.cuda.synchronize()
    poses, ok = poses.cpu().numpy(), ok.cpu().numpy()
    assert ok[2] == 0 and ok[3] == 0
    ident = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0], np.float32)
    assert np.array_equal(poses[2], ident) and np.array_equal(poses[3], ident)
    inr = (tri >= 0).all(1) & (tri < 1000).all(1)
    R64, t64, fl = oracle.kabsch(p.src, p.dst, np.where(inr[:, None], tri, -1))
    worst_r = worst_t = 0.0
    for k in np.nonzero(fl == 1)[0]:   # well-conditioned triplets: the same fit within the pose bar
        assert ok[k] == 1
        worst_r = max(worst_r, rot_angle(poses[k, :9].reshape(3, 3), R64[k]))
        worst_t = max(worst_t, float(np.abs(poses[k, 9:].astype(np.float64) - t64[k]).max()))
    say(worst_r, worst_t)
    assert worst_r <= POSE_RAD and worst_t <= POSE_M
    dposes = torch.empty((600, 12), dtype=torch.float32, device="cuda")
    dok = torch.empty(600, dtype=torch.int32, device="cuda")
    with pytest.raises(T.TurboRegError):   # n < 3
        T.tr_fit_triplets(reg.h, to_dev(torch, p.src), to_dev(torch, p.dst), 2, to_dev(torch, tri), 600, dposes, dok)



def test_fit_nearly_collinear_matches_oracle(reg):
    """Nearly collinear triplets at outdoor scale (down to sigma_2 / sigma_1 ~ 1e-8): the fit's
    accuracy where the top two eigenvalues of the quaternion matrix nearly coincide; the same
    rotation within 1e-4 rad and translation within 1e-4 m at 100 m from the origin."""
    X, Y, cl = synth.near_collinear_triplets(32, 300)
    H = cl.shape[0]
    poses = torch.empty((H, 12), dtype=torch.float32, device="cuda")
    ok = torch.empty(H, dtype=torch.int32, device="cuda")
    T.tr_fit_triplets(reg.h, to_dev(torch, X), to_dev(torch, Y), X.shape[0], to_dev(torch, cl), H, poses, ok)
    torch.cuda.synchronize()
    poses, ok = poses.cpu().numpy(), ok.cpu().numpy()
    R64, t64, fl = oracle.kabsch(X, Y, cl)
    assert (ok == 1).all() and (fl == 1).sum() >= 200
    worst_r = worst_t = 0.0
    for k in np.nonzero(fl == 1)[0]:
        worst_r = max(worst_r, rot_angle(poses[k, :9].reshape(3, 3), R64[k]))
        worst_t = max(worst_t, float(np.abs(poses[k, 9:].astype(np.float64) - t64[k]).max()))
    say(f"nearly collinear: {int((fl == 1).sum())} fits, worst {worst_r:.2e} rad, {worst_t:.2e} m")
    assert worst_r <= POSE_RAD and worst_t <= POSE_M

def test_experiments_small(reg):
    from paper_2507_01439_amd import experiments
    base = synth.CONFIGS["indoor_n1000"].replace(inlier_ratio=0.05)
    pairs = [synth.make_pair(base, synth.pair_seed(11, 10 + b)) for b in range(2)]
    ch = experiments.correct_hypotheses(reg, torch, pairs, hs=(100, 400))
    say(ch)
    assert ch[400]["successful_poses"] >= ch[100]["successful_poses"] >= 0
    sw = experiments.sweep(reg, torch, pairs, taus=(0.05, 0.1), k1s=(100, 200), k2s=(1, 3), k10=200)
    say(sw)
    assert all(0 <= v["success_rate"] <= 1 for part in sw.values() for v in part.values())
    cd = experiments.clique_discrepancy(reg, torch, taus=(0.02, 0.2), n=800, cliques=3)
    say(cd)
    assert cd[0.02]["cliques"] > 0 and cd[0.02]["fits"] > 0


def oracle_sweep_point(pairs, tau, k1, k2):
    """The same two numbers from the oracle's whole path and its own float64 fits."""
    ok = good = 0
    for p in pairs:
        r, _, o = oracle.register_ex(p.src, p.dst, tau, p.cfg.theta, k1, k2)
        ok += r.best_hyp >= 0 and synth.success(np.array(r.R).reshape(3, 3), np.array(r.t), p)
        good += sum(synth.success(o["R"][h], o["t"][h], p) for h in np.nonzero(o["flags"] != 0)[0])
    return {"success_rate": ok / len(pairs), "successful_poses": good / len(pairs)}


@pytest.mark.parametrize("param,point", [("tau", (0.05, 150, 2)), ("k1", (0.1, 60, 2)), ("k2", (0.1, 150, 3))])
def test_sweep_point_matches_oracle(reg, param, point):
    # one point of each swept parameter: the success rate and the successful hypothesis poses per
    # pair equal the oracle's (poses agree within 1e-4, far from the 15 deg / 30 cm thresholds)
    from paper_2507_01439_amd import experiments
    base = synth.CONFIGS["indoor_n1000"].replace(n=800, inlier_ratio=0.04)
    pairs = [synth.make_pair(base, synth.pair_seed(11, 30 + b)) for b in range(3)]
    got = experiments.sweep_point(reg, torch, pairs, *point)
    want = oracle_sweep_point(pairs, *point)
    say(param, point, got, want)
    assert got == want
