"""GPU: the registration entry point that allocates nothing (its workspace is a static device
array) against tr_register on the same inputs: the result record and the inlier mask bit for bit,
on two calls in a row, the second with a smaller input; and its size and mode limits."""
import numpy as np
import pytest

from paper_2507_01439_amd import synth
from paper_2507_01439_amd import turboreg as T
from parity import say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def registered(reg, p, prm):
    """tr_register (handle workspace) and tr_register_noalloc (static workspace) on one pair."""
    src, dst = to_dev(torch, p.src), to_dev(torch, p.dst)
    n = p.src.shape[0]
    out_h = torch.full((80,), 0xAB, dtype=torch.uint8, device="cuda")
    mask_h = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    out_s = torch.full((80,), 0xCD, dtype=torch.uint8, device="cuda")
    mask_s = torch.full((n,), 9, dtype=torch.uint8, device="cuda")
    T.tr_register(reg.h, src, dst, n, prm, out_h, mask_h)
    T.tr_register_noalloc(src, dst, n, prm, out_s, mask_s)
    torch.cuda.synchronize()
    return out_h.cpu().numpy(), mask_h.cpu().numpy(), out_s.cpu().numpy(), mask_s.cpu().numpy()


def test_noalloc_matches_tr_register_on_two_calls():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    reg = T.Registrar(max_n=T.TR_NOALLOC_MAX_N, max_batch=1, max_k1=T.TR_NOALLOC_MAX_K1, max_k2=T.TR_MAX_K2)
    try:
        cases = [(synth.CONFIGS["indoor_n1000"].replace(n=T.TR_NOALLOC_MAX_N, k1=T.TR_NOALLOC_MAX_K1, k2=3), 0),
                 (synth.CONFIGS["indoor_n1000"].replace(n=700, inlier_ratio=0.1, k1=300, k2=2), 1)]
        for cfg, k in cases:   # the second call is smaller: no state of the first may leak into it
            p = synth.make_pair(cfg, synth.pair_seed(13, k))
            prm = T.params_from_config(cfg)
            say(f"no-alloc call {k}: n={cfg.n} k1={cfg.k1} k2={cfg.k2}")
            out_h, mask_h, out_s, mask_s = registered(reg, p, prm)
            r = T.parse_results(torch.from_numpy(out_s))[0]
            assert r.status == T.TR_OK and r.best_inliers > 0
            assert np.array_equal(out_s, out_h), k
            assert np.array_equal(mask_s, mask_h), k
            assert synth.success(np.array(r.R).reshape(3, 3), np.array(r.t), p)
    finally:
        reg.close()


def test_noalloc_limits():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    n = T.TR_NOALLOC_MAX_N + 1
    src = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
    out = torch.empty(80, dtype=torch.uint8, device="cuda")
    cases = [(n, T.make_params(0.1, 0.1, k1=100, k2=2), T.TR_ERR_WORKSPACE),
             (100, T.make_params(0.1, 0.1, k1=T.TR_NOALLOC_MAX_K1 + 1, k2=2), T.TR_ERR_WORKSPACE),
             (100, T.make_params(0.1, 0.1, k1=100, k2=2, pivot_mode=T.TR_PIVOTS_LEARNED, pool_factor=4),
              T.TR_ERR_INVALID_ARG),
             (100, T.make_params(0.1, 0.1, k1=100, k2=2, flags=T.TR_FLAG_PROFILE), T.TR_ERR_INVALID_ARG),
             (2, T.make_params(0.1, 0.1, k1=100, k2=2), T.TR_ERR_INVALID_ARG)]
    for nn, prm, want in cases:
        with pytest.raises(T.TurboRegError) as e:
            T.tr_register_noalloc(src, src, nn, prm, out)
        assert e.value.status == want, (nn, want, e.value.status)
