"""TurboReg CPU oracle -- TEST INFRASTRUCTURE ONLY.

Python access (ctypes + numpy) to the plain C oracle in ``turboreg_oracle.c``.
Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package; the HIP library and its binding never do. Nothing here
shares code with the GPU path.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "turboreg_oracle.c")
_LIB = os.path.join(_HERE, "libturboreg_oracle.so")          # one thread
_LIB_OMP = os.path.join(_HERE, "libturboreg_oracle_omp.so")  # the same code with OpenMP loops
_libs = {}
_threaded = False


def build() -> str:
    """Compile the oracle with gcc (no contraction, no fast-math), once plain and once with
    OpenMP over the host's cores (same arithmetic: the pragmas only split independent loops)."""
    base = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-Wall"]
    for out, extra in ((_LIB, ["-Wno-unknown-pragmas"]), (_LIB_OMP, ["-fopenmp"])):
        subprocess.run(base + extra + ["-o", out + ".tmp", _SRC, "-lm"], check=True)
        os.replace(out + ".tmp", out)
    return _LIB


def set_threaded(flag: bool) -> bool:
    """Route the functions below to the OpenMP build (True) or the one-thread build; returns the
    previous setting."""
    global _threaded
    prev, _threaded = _threaded, bool(flag)
    return prev


def lib(threaded=None):
    threaded = _threaded if threaded is None else threaded
    if threaded not in _libs:
        path = _LIB_OMP if threaded else _LIB
        if not os.path.exists(path):
            build()
        L = ct.CDLL(path)
        _declare(L)
        _libs[threaded] = L
    return _libs[threaded]


_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_i64ptr = ct.POINTER(ct.c_int64)


class Params(ct.Structure):
    _fields_ = [("tau", ct.c_float), ("theta", ct.c_float), ("k1", ct.c_int32),
                ("k2", ct.c_int32), ("graph", ct.c_int32)]


class Result(ct.Structure):
    _fields_ = [("R", ct.c_double * 9), ("t", ct.c_double * 3), ("R32", ct.c_float * 9),
                ("t32", ct.c_float * 3), ("best_inliers", ct.c_int32), ("best_hyp", ct.c_int32),
                ("n_valid_hyp", ct.c_int32), ("status", ct.c_int32),
                ("n_boundary32", ct.c_int64), ("n_boundary64", ct.c_int64), ("n_flip", ct.c_int64),
                ("n_pivots", ct.c_int64)]


def _declare(L):
    I, I64 = ct.c_int32, ct.c_int64
    L.tro_compat.argtypes = [_f32p, _f32p, I, ct.c_float, _u8p, _i64ptr, _i64ptr, _i64ptr]
    L.tro_sc2.argtypes = [_u8p, I, _i32p]
    L.tro_o2graph.argtypes = [_i32p, I, _i32p]
    L.tro_pivots.argtypes = [_i32p, I, I, _i32p]
    L.tro_pivots.restype = I64
    L.tro_cliques.argtypes = [_i32p, I, _i32p, I, I, I, _i32p]
    L.tro_kabsch.argtypes = [_f32p, _f32p, _i32p, I, _f64p, _f64p, _i32p]
    L.tro_score.argtypes = [_f32p, _f32p, I, _f32p, _i32p, I, ct.c_float, _i32p]
    L.tro_mask.argtypes = [_f32p, _f32p, I, _f32p, ct.c_float, _u8p]
    L.tro_select.argtypes = [_i32p, I]
    L.tro_select.restype = I
    L.tro_score_metric.argtypes = [_f32p, _f32p, I, _f32p, _i32p, I, ct.c_float, I, _f32p]
    L.tro_select_score.argtypes = [_f32p, I]
    L.tro_select_score.restype = I
    L.tro_register.argtypes = [_f32p, _f32p, I, ct.POINTER(Params), ct.POINTER(Result), ct.c_void_p]
    vp = ct.c_void_p
    L.tro_register_ex.argtypes = [_f32p, _f32p, I, ct.POINTER(Params), I, vp, vp, ct.POINTER(Result), vp,
                                  vp, vp, vp, vp, vp, vp]
    L.tro_features.argtypes = [_f32p, _f32p, I, ct.c_float, _u8p, _i32p, _f64p]
    L.tro_mlp_fwd.argtypes = [_f64p, I] + [_f64p] * 6 + [_f64p]
    bwd = [_f64p, _u8p, I] + [_f64p] * 6 + [_f64p] * 6 + [ct.POINTER(ct.c_double)]
    L.tro_mlp_bwd.argtypes = bwd
    L.tro_mlp_bwd_exact.argtypes = bwd
    L.tro_adam.argtypes = [_f64p, _f64p, _f64p, _f64p, I64, I, ct.c_double, ct.c_double,
                           ct.c_double, ct.c_double]
    L.tro_pivots_learned.argtypes = [_i32p, I, _f32p, I, _i32p]
    L.tro_bf16_round.argtypes = [ct.c_float]
    L.tro_bf16_round.restype = ct.c_float
    L.tro_threads.argtypes = []
    L.tro_threads.restype = I


def _pts(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    assert a.ndim == 2 and a.shape[1] == 3
    return a


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what} failed with {rc}")


def compat(X, Y, tau):
    """Eq. 1 -> (C uint8 NxN, n_boundary32, n_boundary64, n_flip)."""
    X, Y = _pts(X), _pts(Y)
    n = X.shape[0]
    C = np.empty((n, n), np.uint8)
    b32, b64, fl = ct.c_int64(), ct.c_int64(), ct.c_int64()
    _check(lib().tro_compat(X, Y, n, float(tau), C, ct.byref(b32), ct.byref(b64), ct.byref(fl)), "compat")
    return C, b32.value, b64.value, fl.value


def sc2(C):
    """Eq. 2 -> symmetric Ghat int32."""
    C = np.ascontiguousarray(C, dtype=np.uint8)
    n = C.shape[0]
    G = np.empty((n, n), np.int32)
    _check(lib().tro_sc2(C, n, G), "sc2")
    return G


def o2graph(G):
    """Definition 2 -> strictly upper-triangular copy."""
    G = np.ascontiguousarray(G, dtype=np.int32)
    out = np.empty_like(G)
    _check(lib().tro_o2graph(G, G.shape[0], out), "o2graph")
    return out


def pivots(Gbar, k1):
    """Eq. 4 -> (P int32 k1x3 of (i, j, w), count)."""
    Gbar = np.ascontiguousarray(Gbar, dtype=np.int32)
    P = np.empty((k1, 3), np.int32)
    c = lib().tro_pivots(Gbar, Gbar.shape[0], int(k1), P)
    _check(c, "pivots")
    return P, int(c)


def cliques(Gbar, P, n_pivots, k1, k2):
    """Eqs. 5-8 -> int32 (k1*k2) x 3, slot-major."""
    Gbar = np.ascontiguousarray(Gbar, dtype=np.int32)
    P = np.ascontiguousarray(P, dtype=np.int32)
    out = np.empty((k1 * k2, 3), np.int32)
    _check(lib().tro_cliques(Gbar, Gbar.shape[0], P, int(n_pivots), int(k1), int(k2), out), "cliques")
    return out


def kabsch(X, Y, cl):
    """float64 fit per clique -> (R Hx3x3, t Hx3, flags H)."""
    X, Y = _pts(X), _pts(Y)
    cl = np.ascontiguousarray(cl, dtype=np.int32)
    H = cl.shape[0]
    R = np.empty((H, 9), np.float64)
    t = np.empty((H, 3), np.float64)
    fl = np.empty(H, np.int32)
    _check(lib().tro_kabsch(X, Y, cl, H, R, t, fl), "kabsch")
    return R.reshape(H, 3, 3), t, fl


def score(X, Y, poses, valid, theta):
    """Eq. 9 inlier numbers for float32 poses (H x 12)."""
    X, Y = _pts(X), _pts(Y)
    poses = np.ascontiguousarray(poses, dtype=np.float32).reshape(-1, 12)
    valid = np.ascontiguousarray(valid, dtype=np.int32)
    IN = np.empty(poses.shape[0], np.int32)
    _check(lib().tro_score(X, Y, X.shape[0], poses, valid, poses.shape[0], float(theta), IN), "score")
    return IN


def mask(X, Y, pose, theta):
    X, Y = _pts(X), _pts(Y)
    pose = np.ascontiguousarray(pose, dtype=np.float32).reshape(12)
    m = np.empty(X.shape[0], np.uint8)
    _check(lib().tro_mask(X, Y, X.shape[0], pose, float(theta), m), "mask")
    return m


def select(IN):
    IN = np.ascontiguousarray(IN, dtype=np.int32)
    return int(lib().tro_select(IN, IN.shape[0]))


METRIC_MAE, METRIC_MSE = 1, 2


def score_metric(X, Y, poses, valid, theta, metric):
    """Error-based hypothesis scores (MAE or MSE form; larger is better, -1 if invalid)."""
    X, Y = _pts(X), _pts(Y)
    poses = np.ascontiguousarray(poses, dtype=np.float32).reshape(-1, 12)
    valid = np.ascontiguousarray(valid, dtype=np.int32)
    S = np.empty(poses.shape[0], np.float32)
    _check(lib().tro_score_metric(X, Y, X.shape[0], poses, valid, poses.shape[0], float(theta), int(metric), S),
           "score_metric")
    return S


def select_score(S):
    S = np.ascontiguousarray(S, dtype=np.float32)
    return int(lib().tro_select_score(S, S.shape[0]))


def register(X, Y, tau, theta, k1, k2, graph=0, threaded=None):
    """Whole path -> (Result, mask)."""
    X, Y = _pts(X), _pts(Y)
    p = Params(tau, theta, k1, k2, graph)
    r = Result()
    m = np.empty(X.shape[0], np.uint8)
    _check(lib(threaded).tro_register(X, Y, X.shape[0], ct.byref(p), ct.byref(r), m.ctypes.data), "register")
    return r, m


def register_ex(X, Y, tau, theta, k1, k2, graph=0, pool_factor=0, scores=None, poses=None, threaded=None):
    """Whole path with the learned reorder of the pool by `scores` (N float32, or None for plain
    pivots) and scoring on the given float32 `poses` (H x 12, or None for the path's own fits
    rounded to float32) -> (Result, mask, per-hypothesis arrays)."""
    X, Y = _pts(X), _pts(Y)
    n, H = X.shape[0], int(k1) * int(k2)
    p = Params(tau, theta, k1, k2, graph)
    r = Result()
    m = np.empty(n, np.uint8)
    out = dict(cliques=np.empty((H, 3), np.int32), R=np.empty((H, 3, 3)), t=np.empty((H, 3)),
               flags=np.empty(H, np.int32), IN=np.empty(H, np.int32), pivots=np.empty((int(k1), 3), np.int32))
    if scores is not None:
        scores = np.ascontiguousarray(scores, np.float32)
        assert scores.shape == (n,)
    if poses is not None:
        poses = np.ascontiguousarray(poses, np.float32)
        assert poses.shape == (H, 12)
    ptr = lambda a: None if a is None else a.ctypes.data  # noqa: E731
    _check(lib(threaded).tro_register_ex(X, Y, n, ct.byref(p), int(pool_factor), ptr(scores), ptr(poses),
                                         ct.byref(r), m.ctypes.data, *(ptr(out[k]) for k in
                                         ("cliques", "R", "t", "flags", "IN", "pivots"))), "register_ex")
    return r, m, out


def features(X, Y, tau, C, Ghat):
    X, Y = _pts(X), _pts(Y)
    n = X.shape[0]
    F = np.empty((n, 19), np.float64)
    _check(lib().tro_features(X, Y, n, float(tau), np.ascontiguousarray(C, np.uint8),
                              np.ascontiguousarray(Ghat, np.int32), F), "features")
    return F


def _w(ws):
    return [np.ascontiguousarray(w, dtype=np.float64) for w in ws]


def mlp_fwd(F, weights):
    """weights = (W1 64x19, b1, W2 64x64, b2, W3 1x64, b3) -> s (n,)"""
    F = np.ascontiguousarray(F, np.float64)
    s = np.empty(F.shape[0], np.float64)
    _check(lib().tro_mlp_fwd(F, F.shape[0], *_w(weights), s), "mlp_fwd")
    return s


def mlp_bwd(F, labels, weights, exact=False):
    """-> (loss, [gW1, gb1, gW2, gb2, gW3, gb3])"""
    F = np.ascontiguousarray(F, np.float64)
    labels = np.ascontiguousarray(labels, np.uint8)
    ws = _w(weights)
    grads = [np.empty_like(w) for w in ws]
    loss = ct.c_double()
    fn = lib().tro_mlp_bwd_exact if exact else lib().tro_mlp_bwd
    _check(fn(F, labels, F.shape[0], *ws, *grads, ct.byref(loss)), "mlp_bwd")
    return loss.value, grads


def adam(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam step on float64 arrays."""
    for a in (w, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _check(lib().tro_adam(w, g, m, v, w.size, int(t), lr, beta1, beta2, eps), "adam")


def pivots_learned(P_plain, s, k1):
    P_plain = np.ascontiguousarray(P_plain, np.int32)
    s = np.ascontiguousarray(s, np.float32)
    P = np.empty((k1, 3), np.int32)
    rc = lib().tro_pivots_learned(P_plain, P_plain.shape[0], s, int(k1), P)
    _check(rc, "pivots_learned")
    return P, bool(rc)


def threads(threaded=None) -> int:
    """Threads the selected build's loops use."""
    return int(lib(threaded).tro_threads())


def bf16_round(x):
    return float(lib().tro_bf16_round(float(x)))
