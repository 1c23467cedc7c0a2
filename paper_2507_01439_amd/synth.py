"""Seeded synthetic correspondence sets.

This module is the only code the GPU path and the CPU oracle both use: it
draws inputs and holds none of the registration method's arithmetic. It
depends on numpy alone.

Model (paper, Appendix A.1): a correspondence m_i = (x_i, y_i) is an inlier
when y_i = R x_i + t + r_i with isotropic Gaussian noise r_i ~ N(0, sigma^2 I).
Outliers have targets drawn uniformly in a box of the source box's size,
centred on t. Points are generated in float64 and stored as float32, N x 3,
row-major. Inliers sit at a seeded random permutation of indices, because the
O2Graph orientation (Definition 2) depends on index order.

Rotations are uniform on SO(3) by Shoemake's quaternion construction
(Graphics Gems III, 1992); translations are uniform in the ball |t| <= t_max.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = ["PairConfig", "Pair", "CONFIGS", "make_pair", "pair_seed", "rotation_error_deg",
           "translation_error", "random_rotation"]


@dataclasses.dataclass(frozen=True)
class PairConfig:
    """Shape of one synthetic pair."""
    n: int
    inlier_ratio: float
    sigma: float                 # inlier noise std-dev, metres
    box: tuple = (3.0, 3.0, 3.0)  # source box edge lengths, metres, centred at the origin
    t_max: float = 1.0           # translation drawn uniformly in the ball of this radius
    tau: float = 0.1             # compatibility threshold (Eq. 1)
    theta: float = 0.1           # inlier threshold for hypothesis scoring (Eq. 9)
    k1: int = 500                # pivots
    k2: int = 2                  # TurboCliques per pivot
    outdoor: bool = False        # success thresholds: RE<=5 deg, TE<=0.6 m if outdoor

    def replace(self, **kw) -> "PairConfig":
        return dataclasses.replace(self, **kw)


# The five workloads. The clique counts 1000/2000/5000 are K1*K2 with K2 = 2.
CONFIGS = {
    # small single pair, indoor
    "indoor_n1000": PairConfig(n=1000, inlier_ratio=0.20, sigma=0.01, tau=0.1, theta=0.1, k1=500, k2=2),
    # single pair at N = 5000, 5% inliers: the throughput / roofline workload
    "indoor_n5000": PairConfig(n=5000, inlier_ratio=0.05, sigma=0.02, tau=0.1, theta=0.1, k1=1000, k2=2),
    # outdoor pair, N = 20000, 1% inliers, 100 x 100 x 10 m box
    "outdoor_n20000": PairConfig(n=20000, inlier_ratio=0.01, sigma=0.05, box=(100.0, 100.0, 10.0),
                                 tau=0.6, theta=0.6, k1=2500, k2=2, outdoor=True),
}


@dataclasses.dataclass
class Pair:
    src: np.ndarray      # N x 3 float32
    dst: np.ndarray      # N x 3 float32
    labels: np.ndarray   # N bool, True = inlier
    R: np.ndarray        # 3 x 3 float64 ground-truth rotation
    t: np.ndarray        # 3 float64 ground-truth translation
    cfg: PairConfig


def pair_seed(workload: int, index: int, salt: int = 0) -> int:
    """A 63-bit seed for pair `index` of workload `workload`."""
    ss = np.random.SeedSequence([0x7A11, int(workload), int(index), int(salt)])
    return int(ss.generate_state(1, dtype=np.uint64)[0] >> np.uint64(1))


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform rotation on SO(3) via Shoemake's unit-quaternion construction."""
    u1, u2, u3 = rng.random(3)
    a, b = math.sqrt(1.0 - u1), math.sqrt(u1)
    w = a * math.sin(2 * math.pi * u2)
    x = a * math.cos(2 * math.pi * u2)
    y = b * math.sin(2 * math.pi * u3)
    z = b * math.cos(2 * math.pi * u3)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ], dtype=np.float64)


def _ball(rng: np.random.Generator, radius: float) -> np.ndarray:
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    return d * radius * rng.random() ** (1.0 / 3.0)


def make_pair(cfg: PairConfig, seed: int) -> Pair:
    """Draw one correspondence set of shape `cfg` from `seed`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = int(cfg.n)
    box = np.asarray(cfg.box, dtype=np.float64)
    R = random_rotation(rng)
    t = _ball(rng, cfg.t_max)
    x = (rng.random((n, 3)) - 0.5) * box
    n_in = int(round(cfg.inlier_ratio * n))
    perm = rng.permutation(n)
    labels = np.zeros(n, dtype=bool)
    labels[perm[:n_in]] = True
    y = (rng.random((n, 3)) - 0.5) * box + t            # outlier targets
    noise = rng.standard_normal((n, 3)) * cfg.sigma
    y_in = x @ R.T + t + noise
    y[labels] = y_in[labels]
    return Pair(src=np.ascontiguousarray(x, dtype=np.float32),
                dst=np.ascontiguousarray(y, dtype=np.float32),
                labels=labels, R=R, t=t, cfg=cfg)


def batch_configs(count: int, seed: int, n_lo: int = 500, n_hi: int = 5000,
                  ratio_lo: float = 0.02, ratio_hi: float = 0.30, base: PairConfig | None = None):
    """Per-pair configs of an uneven batch: N ~ U{n_lo..n_hi}, ratio ~ U[ratio_lo, ratio_hi]."""
    base = base or CONFIGS["indoor_n1000"]
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ratios = rng.uniform(ratio_lo, ratio_hi, size=count)
    return [base.replace(n=int(n), inlier_ratio=float(r)) for n, r in zip(ns, ratios)]


def rotation_error_deg(R_est: np.ndarray, R_gt: np.ndarray) -> float:
    """RE = arccos((tr(R_gt^T R) - 1) / 2) in degrees (the paper's registration metric)."""
    c = (np.trace(np.asarray(R_gt, np.float64).T @ np.asarray(R_est, np.float64)) - 1.0) / 2.0
    return math.degrees(math.acos(max(-1.0, min(1.0, c))))


def translation_error(t_est: np.ndarray, t_gt: np.ndarray) -> float:
    """TE = |t_gt - t| in metres."""
    return float(np.linalg.norm(np.asarray(t_gt, np.float64) - np.asarray(t_est, np.float64)))


def success(R_est, t_est, pair: Pair) -> bool:
    """Registration success: RE < 15 deg and TE < 30 cm indoors (strict, as the throughput target
    states it; the paper's own criterion uses <=, which differs only on a set of measure zero);
    RE <= 5 deg and TE <= 60 cm outdoors (the paper's KITTI criterion)."""
    re = rotation_error_deg(R_est, pair.R)
    te = translation_error(t_est, pair.t)
    if pair.cfg.outdoor:
        return re <= 5.0 and te <= 0.6
    return re < 15.0 and te < 0.30


def near_collinear_triplets(seed: int, count: int, box=(100.0, 100.0, 10.0), sigma: float = 0.05,
                            log10_off=(-6.0, -1.0)):
    """`count` match triplets whose source points lie nearly on a line, for the conditioning of
    three-point fits: a and b uniform in the box, c = a + u (b - a) + e n with u ~ U[-0.5, 1.5],
    n a unit vector orthogonal to b - a and e = 10^U(log10_off) metres; targets are a rigid
    motion of the sources plus N(0, sigma^2 I) noise. Returns (X, Y) float32 (3 count x 3) and
    the cliques int32 (count x 3) = (3k, 3k+1, 3k+2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    box = np.asarray(box, dtype=np.float64)
    R = random_rotation(rng)
    t = _ball(rng, 1.0)
    X = np.empty((3 * count, 3))
    for k in range(count):
        a, b = (rng.random((2, 3)) - 0.5) * box
        d = b - a
        n = np.cross(d, rng.standard_normal(3))
        n /= np.linalg.norm(n)
        c = a + rng.uniform(-0.5, 1.5) * d + 10.0 ** rng.uniform(*log10_off) * n
        X[3 * k:3 * k + 3] = (a, b, c)
    Y = X @ R.T + t + rng.standard_normal(X.shape) * sigma
    cl = np.arange(3 * count, dtype=np.int32).reshape(count, 3)
    return (np.ascontiguousarray(X, dtype=np.float32), np.ascontiguousarray(Y, dtype=np.float32), cl)
