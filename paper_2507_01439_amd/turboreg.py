"""Python binding of libturboreg (the gfx950 HIP library): argument marshalling only.

The functions keep the C names of include/turboreg.h. Device buffers are torch
tensors on a ROCm device; the stream is torch's current stream. Every step of
the registration path runs in the library's HIP kernels; there is no fallback:
if the library is not built, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libturboreg.so")

TR_OK, TR_ERR_INVALID_ARG, TR_ERR_NONFINITE, TR_ERR_NO_HYPOTHESIS = 0, 1, 2, 3
TR_ERR_WORKSPACE, TR_ERR_HIP, TR_WARN_SCORER_FALLBACK, TR_ERR_NO_SCORER, TR_ERR_BAD_BLOB = 4, 5, 6, 7, 8
TR_GRAPH_O2, TR_GRAPH_SC2 = 0, 1
TR_PIVOTS_PLAIN, TR_PIVOTS_LEARNED = 0, 1
TR_FLAG_PROFILE, TR_FLAG_PROFILE_SC2, TR_FLAG_RANK_MAE, TR_FLAG_RANK_MSE = 1, 2, 4, 8
TR_MAX_K2 = 8
TR_SC2_SPARSE_CAP_MAX = 8192
TR_NOALLOC_MAX_N = 2048
TR_NOALLOC_MAX_K1 = 1024
TR_MLP_NPARAM = 5505
(TR_TAP_C, TR_TAP_G, TR_TAP_PIVOTS, TR_TAP_CLIQUES, TR_TAP_POSES, TR_TAP_IN, TR_TAP_FEATURES,
 TR_TAP_SCORES, TR_TAP_PLAIN_PIVOTS, TR_TAP_RANK_SCORES) = range(10)
STAGES = ("plan", "compat", "sc2", "pivots", "learned", "cliques", "kabsch", "score", "select")
TR_NUM_STAGES = len(STAGES)

EXPORTS = ("tr_create", "tr_destroy", "tr_register", "tr_register_batch", "tr_scorer_load",
           "tr_scorer_save", "tr_scorer_set", "tr_scorer_get", "tr_features_batch", "tr_mlp_forward",
           "tr_mlp_grads", "tr_train_step", "tr_debug_copy", "tr_stage_times", "tr_status_string",
           "tr_tuning_get", "tr_tuning_set", "tr_autotune", "tr_score_poses", "tr_fit_triplets",
           "tr_register_noalloc", "tr_tuning_save", "tr_tuning_load")


class tr_params(ct.Structure):
    _fields_ = [("tau", ct.c_float), ("inlier_thresh", ct.c_float), ("k1", ct.c_int32), ("k2", ct.c_int32),
                ("graph", ct.c_int32), ("pivot_mode", ct.c_int32), ("pool_factor", ct.c_int32),
                ("flags", ct.c_uint32)]


class tr_result(ct.Structure):
    _fields_ = [("R", ct.c_float * 9), ("t", ct.c_float * 3), ("best_inliers", ct.c_int32),
                ("best_hyp", ct.c_int32), ("n_valid_hyp", ct.c_int32), ("status", ct.c_int32),
                ("n_boundary_pairs", ct.c_int32), ("n_pivots", ct.c_int32), ("n_edges", ct.c_int32),
                ("reserved", ct.c_int32)]


class tr_tuning(ct.Structure):
    _fields_ = [("sc2_super", ct.c_int32), ("compat_per_cu", ct.c_int32), ("hyp_ppw", ct.c_int32),
                ("hyp_per_cu", ct.c_int32), ("sc2_sparse_cap", ct.c_int32)]


assert ct.sizeof(tr_result) == 80 and ct.sizeof(tr_params) == 32 and ct.sizeof(tr_tuning) == 20

_lib = None


def lib():
    """Load libturboreg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ct.CDLL(LIB_PATH)
        vp, I32, I64 = ct.c_void_p, ct.c_int32, ct.c_int64
        L.tr_create.argtypes = [ct.POINTER(vp), I32, I32, I32, I32, I32]
        L.tr_destroy.argtypes = [vp]
        L.tr_register.argtypes = [vp, vp, vp, I32, ct.POINTER(tr_params), vp, vp, vp]
        L.tr_register_batch.argtypes = [vp, vp, vp, vp, I32, I32, ct.POINTER(tr_params), vp, vp, vp]
        L.tr_register_noalloc.argtypes = [vp, vp, I32, ct.POINTER(tr_params), vp, vp, vp]
        L.tr_scorer_load.argtypes = [vp, vp, ct.c_size_t]
        L.tr_scorer_save.argtypes = [vp, vp, ct.c_size_t, ct.POINTER(ct.c_size_t)]
        L.tr_scorer_set.argtypes = [vp, vp]
        L.tr_scorer_get.argtypes = [vp, vp]
        L.tr_features_batch.argtypes = [vp, vp, vp, vp, I32, I32, ct.POINTER(tr_params), vp, vp]
        L.tr_mlp_forward.argtypes = [vp, vp, I64, vp, vp]
        L.tr_mlp_grads.argtypes = [vp, vp, vp, I64, vp, vp, vp]
        L.tr_train_step.argtypes = [vp, vp, vp, I64, ct.c_float, vp, vp]
        L.tr_debug_copy.argtypes = [vp, I32, I32, vp, ct.c_size_t, ct.POINTER(ct.c_size_t)]
        L.tr_stage_times.argtypes = [vp, ct.POINTER(ct.c_float), I32]
        L.tr_score_poses.argtypes = [vp, vp, vp, I32, vp, I32, ct.c_float, I32, vp, vp, vp]
        L.tr_fit_triplets.argtypes = [vp, vp, vp, I32, vp, I32, vp, vp, vp]
        L.tr_tuning_get.argtypes = [vp, I32, I32, ct.POINTER(tr_tuning)]
        L.tr_tuning_set.argtypes = [vp, I32, I32, ct.POINTER(tr_tuning)]
        L.tr_tuning_save.argtypes = [vp, ct.c_char_p]
        L.tr_tuning_load.argtypes = [vp, ct.c_char_p]
        L.tr_autotune.argtypes = [vp, vp, vp, vp, I32, I32, ct.POINTER(tr_params), vp, vp, vp,
                                  ct.POINTER(tr_tuning), ct.POINTER(ct.c_float)]
        L.tr_status_string.argtypes = [I32]
        L.tr_status_string.restype = ct.c_char_p
        for name in EXPORTS:
            if name != "tr_status_string":
                getattr(L, name).restype = I32
        _lib = L
    return _lib


class TurboRegError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {tr_status_string(status)} ({status})")


def tr_status_string(status: int) -> str:
    return lib().tr_status_string(int(status)).decode()


def _ck(status, where):
    if status != TR_OK:
        raise TurboRegError(status, where)


def _stream():
    import torch
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ct.c_void_p(t.data_ptr())


def make_params(tau, inlier_thresh, k1, k2=2, graph=TR_GRAPH_O2, pivot_mode=TR_PIVOTS_PLAIN, pool_factor=4,
                flags=0) -> tr_params:
    return tr_params(float(tau), float(inlier_thresh), int(k1), int(k2), int(graph), int(pivot_mode),
                     int(pool_factor), int(flags))


def params_from_config(cfg, **kw) -> tr_params:
    d = dict(tau=cfg.tau, inlier_thresh=cfg.theta, k1=cfg.k1, k2=cfg.k2)
    d.update(kw)
    return make_params(**d)


# ---------------------------------------------------------------- C-named calls

def tr_create(max_n, max_batch=1, max_k1=2500, max_k2=2, device=0):
    h = ct.c_void_p()
    _ck(lib().tr_create(ct.byref(h), int(max_n), int(max_batch), int(max_k1), int(max_k2), int(device)), "tr_create")
    return h


def tr_destroy(h):
    _ck(lib().tr_destroy(h), "tr_destroy")


def tr_register(h, src, dst, n, params, out, mask=None):
    _ck(lib().tr_register(h, _ptr(src), _ptr(dst), int(n), ct.byref(params), _ptr(out), _ptr(mask), _stream()),
        "tr_register")


def tr_register_noalloc(src, dst, n, params, out, mask=None):
    _ck(lib().tr_register_noalloc(_ptr(src), _ptr(dst), int(n), ct.byref(params), _ptr(out), _ptr(mask), _stream()),
        "tr_register_noalloc")


def tr_register_batch(h, src, dst, offsets, B, max_n, params, out, masks=None):
    _ck(lib().tr_register_batch(h, _ptr(src), _ptr(dst), _ptr(offsets), int(B), int(max_n), ct.byref(params),
                                _ptr(out), _ptr(masks), _stream()), "tr_register_batch")


def tr_fit_triplets(h, src, dst, n, triplets, T_, poses_out, ok_out):
    _ck(lib().tr_fit_triplets(h, _ptr(src), _ptr(dst), int(n), _ptr(triplets), int(T_), _ptr(poses_out),
                              _ptr(ok_out), _stream()), "tr_fit_triplets")


def tr_score_poses(h, src, dst, n, poses, P, theta, metric, in_out, score_out=None):
    _ck(lib().tr_score_poses(h, _ptr(src), _ptr(dst), int(n), _ptr(poses), int(P), float(theta), int(metric),
                             _ptr(in_out), _ptr(score_out), _stream()), "tr_score_poses")


def tr_tuning_get(h, max_n, B=1) -> tr_tuning:
    t = tr_tuning()
    _ck(lib().tr_tuning_get(h, int(max_n), int(B), ct.byref(t)), "tr_tuning_get")
    return t


def tr_tuning_set(h, max_n, B, t: tr_tuning):
    _ck(lib().tr_tuning_set(h, int(max_n), int(B), ct.byref(t)), "tr_tuning_set")


def tr_tuning_save(h, path):
    _ck(lib().tr_tuning_save(h, os.fsencode(path)), "tr_tuning_save")


def tr_tuning_load(h, path):
    _ck(lib().tr_tuning_load(h, os.fsencode(path)), "tr_tuning_load")


def tr_autotune(h, src, dst, offsets, B, max_n, params, out, masks=None):
    """Returns (best tr_tuning, milliseconds per call under it); offsets None = one pair of N = max_n."""
    t, ms = tr_tuning(), ct.c_float()
    _ck(lib().tr_autotune(h, _ptr(src), _ptr(dst), _ptr(offsets), int(B), int(max_n), ct.byref(params), _ptr(out),
                          _ptr(masks), _stream(), ct.byref(t), ct.byref(ms)), "tr_autotune")
    return t, float(ms.value)


def tr_features_batch(h, src, dst, offsets, B, max_n, params, feat):
    _ck(lib().tr_features_batch(h, _ptr(src), _ptr(dst), _ptr(offsets), int(B), int(max_n), ct.byref(params),
                                _ptr(feat), _stream()), "tr_features_batch")


def tr_scorer_set(h, params_np):
    a = np.ascontiguousarray(params_np, dtype=np.float32)
    assert a.size == TR_MLP_NPARAM
    _ck(lib().tr_scorer_set(h, a.ctypes.data), "tr_scorer_set")


def tr_scorer_get(h):
    a = np.empty(TR_MLP_NPARAM, np.float32)
    _ck(lib().tr_scorer_get(h, a.ctypes.data), "tr_scorer_get")
    return a


def tr_scorer_save(h) -> bytes:
    need = ct.c_size_t()
    _ck(lib().tr_scorer_save(h, None, 0, ct.byref(need)), "tr_scorer_save")
    buf = ct.create_string_buffer(need.value)
    _ck(lib().tr_scorer_save(h, buf, need.value, ct.byref(need)), "tr_scorer_save")
    return buf.raw[:need.value]


def tr_scorer_load(h, blob: bytes):
    buf = ct.create_string_buffer(bytes(blob), len(blob))
    _ck(lib().tr_scorer_load(h, buf, len(blob)), "tr_scorer_load")


def tr_mlp_forward(h, feat, m, scores):
    _ck(lib().tr_mlp_forward(h, _ptr(feat), int(m), _ptr(scores), _stream()), "tr_mlp_forward")


def tr_mlp_grads(h, feat, labels, m, grads, loss=None):
    _ck(lib().tr_mlp_grads(h, _ptr(feat), _ptr(labels), int(m), _ptr(grads), _ptr(loss), _stream()), "tr_mlp_grads")


def tr_train_step(h, feat, labels, m, lr, loss=None):
    _ck(lib().tr_train_step(h, _ptr(feat), _ptr(labels), int(m), float(lr), _ptr(loss), _stream()), "tr_train_step")


_TAP_DTYPES = {TR_TAP_C: (np.uint8, "nn"), TR_TAP_G: (np.uint16, "nn"), TR_TAP_PIVOTS: (np.int32, 3),
               TR_TAP_PLAIN_PIVOTS: (np.int32, 3), TR_TAP_CLIQUES: (np.int32, 3), TR_TAP_POSES: (np.float32, 12),
               TR_TAP_IN: (np.int32, 1), TR_TAP_FEATURES: (np.uint16, 19), TR_TAP_SCORES: (np.float32, 1),
               TR_TAP_RANK_SCORES: (np.float32, 1)}


def tr_debug_copy(h, tap, pair=0):
    """Intermediate `tap` of pair `pair` of the last call, as a numpy array."""
    need = ct.c_size_t()
    _ck(lib().tr_debug_copy(h, int(tap), int(pair), None, 0, ct.byref(need)), "tr_debug_copy")
    dt, cols = _TAP_DTYPES[tap]
    a = np.empty(need.value // np.dtype(dt).itemsize, dt)
    _ck(lib().tr_debug_copy(h, int(tap), int(pair), a.ctypes.data, need.value, ct.byref(need)), "tr_debug_copy")
    if cols == "nn":
        n = int(round(a.size ** 0.5))
        return a.reshape(n, n)
    return a.reshape(-1, cols) if cols != 1 else a


def tr_stage_times(h):
    ms = (ct.c_float * TR_NUM_STAGES)()
    _ck(lib().tr_stage_times(h, ms, TR_NUM_STAGES), "tr_stage_times")
    return dict(zip(STAGES, list(ms)))


def parse_results(out_tensor, count=1):
    """tr_result records from a device (or host) uint8 tensor of count*80 bytes."""
    raw = out_tensor.detach().cpu().numpy().tobytes()
    return [tr_result.from_buffer_copy(raw, 80 * b) for b in range(count)]


def result_dict(r: tr_result) -> dict:
    return dict(R=np.array(r.R, np.float32).reshape(3, 3), t=np.array(r.t, np.float32),
                best_inliers=r.best_inliers, best_hyp=r.best_hyp, n_valid_hyp=r.n_valid_hyp, status=r.status,
                n_boundary_pairs=r.n_boundary_pairs, n_pivots=r.n_pivots, n_edges=r.n_edges)


class Registrar:
    """Owns a handle; registers torch device tensors (N x 3 float32)."""

    def __init__(self, max_n, max_batch=1, max_k1=2500, max_k2=2, device=0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.h = tr_create(max_n, max_batch, max_k1, max_k2, device)
        self.max_n, self.max_batch = max_n, max_batch

    def close(self):
        if self.h is not None:
            tr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def register(self, src, dst, params: tr_params, out=None, mask=None):
        torch = self.torch
        n = src.shape[0]
        out = out if out is not None else torch.empty(80, dtype=torch.uint8, device=self.device)
        mask = mask if mask is not None else torch.empty(n, dtype=torch.uint8, device=self.device)
        tr_register(self.h, src, dst, n, params, out, mask)
        return out, mask

    def register_batch(self, src, dst, offsets, params: tr_params, max_n=None, out=None, masks=None):
        torch = self.torch
        B = offsets.shape[0] - 1
        out = out if out is not None else torch.empty(80 * B, dtype=torch.uint8, device=self.device)
        masks = masks if masks is not None else torch.empty(src.shape[0], dtype=torch.uint8, device=self.device)
        tr_register_batch(self.h, src, dst, offsets, B, max_n or self.max_n, params, out, masks)
        return out, masks

    def debug(self, tap, pair=0):
        return tr_debug_copy(self.h, tap, pair)
