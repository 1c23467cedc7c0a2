"""GPU: launch configurations and the autotuner.

No launch configuration may change a result: every valid configuration must
give the same bits as the default one, and one non-default configuration is
checked against the oracle stage by stage. The autotuner must return a valid
configuration, store it for the shape group, and leave results unchanged.
"""
import numpy as np
import pytest

from paper_2507_01439_amd import synth
from paper_2507_01439_amd import turboreg as T
from parity import check_taps, run_single, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TAPS = (T.TR_TAP_C, T.TR_TAP_G, T.TR_TAP_PIVOTS, T.TR_TAP_CLIQUES, T.TR_TAP_POSES, T.TR_TAP_IN)


@pytest.fixture(scope="module")
def reg():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    r = T.Registrar(max_n=3000, max_batch=8, max_k1=600, max_k2=3)
    yield r
    r.close()


def snapshot(reg, r, mask, pair=0):
    return [reg.debug(t, pair) for t in TAPS] + [np.frombuffer(bytes(r), np.uint8).copy(), mask.copy()]


def same(a, b):
    return all(np.array_equal(x.view(np.uint8), y.view(np.uint8)) for x, y in zip(a, b))


def cfg(sup, compat, ppw, per_cu, sparse=0):
    return T.tr_tuning(sup, compat, ppw, per_cu, sparse)


def test_defaults_and_argument_errors(reg):
    d1 = T.tr_tuning_get(reg.h, 5000, 1)
    assert (d1.sc2_super, d1.compat_per_cu, d1.hyp_ppw, d1.hyp_per_cu, d1.sc2_sparse_cap) == (5, 8, 4, 4, 0)
    d8 = T.tr_tuning_get(reg.h, 1500, 8)
    assert d8.hyp_ppw == 16
    for bad in (cfg(0, 4, 4, 4), cfg(17, 4, 4, 4), cfg(5, 0, 4, 4), cfg(5, 4, 6, 4), cfg(5, 4, 20, 4),
                cfg(5, 4, 4, 0), cfg(5, 4, 4, 17), cfg(5, 4, 4, 4, -1), cfg(5, 4, 4, 4, T.TR_SC2_SPARSE_CAP_MAX + 1)):
        with pytest.raises(T.TurboRegError) as e:
            T.tr_tuning_set(reg.h, 1000, 1, bad)
        assert e.value.status == T.TR_ERR_INVALID_ARG
    with pytest.raises(T.TurboRegError):
        T.tr_tuning_get(reg.h, 2, 1)


def test_single_pair_results_do_not_depend_on_configuration(reg):
    c = synth.CONFIGS["indoor_n1000"].replace(n=2900, k1=600, k2=3)
    p = synth.make_pair(c, synth.pair_seed(6, 1))
    prm = T.params_from_config(c)
    default = T.tr_tuning_get(reg.h, c.n, 1)
    try:
        r0, m0 = run_single(reg, torch, p.src, p.dst, prm)
        ref = snapshot(reg, r0, m0)
        for k, t in enumerate([cfg(1, 1, 8, 1), cfg(16, 16, 16, 16, 8192), cfg(3, 2, 12, 2, 1024),
                               cfg(8, 8, 4, 8, 3000)]):
            say(f"configuration {k}: super {t.sc2_super} compat {t.compat_per_cu} ppw {t.hyp_ppw} per_cu {t.hyp_per_cu} "
                f"sparse {t.sc2_sparse_cap}")
            T.tr_tuning_set(reg.h, c.n, 1, t)
            assert T.tr_tuning_get(reg.h, c.n, 1).hyp_ppw == t.hyp_ppw
            r, m = run_single(reg, torch, p.src, p.dst, prm)
            assert same(snapshot(reg, r, m), ref), k
        check_taps(reg, p.src, p.dst, prm, r, m, label="tuned single pair")
    finally:
        T.tr_tuning_set(reg.h, c.n, 1, default)


def test_batch_results_do_not_depend_on_configuration(reg):
    ns = [1400, 2, 777, 1500, 64, 1001]   # pair 1 is invalid (N < 3)
    pairs = [synth.make_pair(synth.CONFIGS["indoor_n1000"].replace(n=n, k1=300), synth.pair_seed(6, 10 + b))
             for b, n in enumerate(ns)]
    src = to_dev(torch, np.concatenate([q.src for q in pairs]))
    dst = to_dev(torch, np.concatenate([q.dst for q in pairs]))
    offs = to_dev(torch, np.concatenate([[0], np.cumsum(ns)]).astype(np.int32))
    prm = T.make_params(0.1, 0.1, k1=300, k2=2)
    B, max_n = len(ns), max(ns)
    default = T.tr_tuning_get(reg.h, max_n, B)
    side = torch.cuda.Stream()
    outs = []
    try:
        for t in (default, cfg(2, 1, 4, 1), cfg(6, 16, 12, 8)):
            T.tr_tuning_set(reg.h, max_n, B, t)
            with torch.cuda.stream(side):   # a non-default stream: captured into a hipGraph per configuration
                out, masks = reg.register_batch(src, dst, offs, prm, max_n=max_n)
                out2, masks2 = reg.register_batch(src, dst, offs, prm, max_n=max_n)   # replay
            side.synchronize()
            res = T.parse_results(out, B)
            assert np.array_equal(out.cpu().numpy(), out2.cpu().numpy())
            outs.append((out.cpu().numpy(), masks.cpu().numpy(), [reg.debug(T.TR_TAP_IN, b) for b in range(B) if b != 1]))
            assert res[1].status == T.TR_ERR_INVALID_ARG and res[0].status == T.TR_OK
        for o in outs[1:]:
            assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
            assert all(np.array_equal(a, b) for a, b in zip(o[2], outs[0][2]))
    finally:
        T.tr_tuning_set(reg.h, max_n, B, default)


def test_autotune_single_pair(reg):
    c = synth.CONFIGS["indoor_n1000"].replace(n=3000, k1=500)
    p = synth.make_pair(c, synth.pair_seed(6, 2))
    prm = T.params_from_config(c)
    r0, m0 = run_single(reg, torch, p.src, p.dst, prm)
    ref = snapshot(reg, r0, m0)
    src, dst = to_dev(torch, p.src), to_dev(torch, p.dst)
    out = torch.empty(80, dtype=torch.uint8, device="cuda")
    mask = torch.empty(c.n, dtype=torch.uint8, device="cuda")
    best, ms = T.tr_autotune(reg.h, src, dst, None, 1, c.n, prm, out, mask)
    torch.cuda.synchronize()
    say(f"autotune n={c.n}: super {best.sc2_super} compat {best.compat_per_cu} ppw {best.hyp_ppw} "
        f"per_cu {best.hyp_per_cu}: {ms * 1000:.1f} us")
    assert 0.0 < ms < 100.0
    got = T.tr_tuning_get(reg.h, c.n, 1)
    assert bytes(got) == bytes(best)
    assert same(snapshot(reg, T.parse_results(out)[0], mask.cpu().numpy()), ref)
    r1, m1 = run_single(reg, torch, p.src, p.dst, prm)   # later calls of the group use the tuned configuration
    assert same(snapshot(reg, r1, m1), ref)


def test_autotune_batch(reg):
    ns = [900, 1500, 1200, 400]
    pairs = [synth.make_pair(synth.CONFIGS["indoor_n1000"].replace(n=n, k1=300), synth.pair_seed(6, 20 + b))
             for b, n in enumerate(ns)]
    src = to_dev(torch, np.concatenate([q.src for q in pairs]))
    dst = to_dev(torch, np.concatenate([q.dst for q in pairs]))
    offs = to_dev(torch, np.concatenate([[0], np.cumsum(ns)]).astype(np.int32))
    prm = T.make_params(0.1, 0.1, k1=300, k2=2)
    B, max_n = len(ns), max(ns)
    out0, masks0 = reg.register_batch(src, dst, offs, prm, max_n=max_n)
    torch.cuda.synchronize()
    ref = out0.cpu().numpy()
    out = torch.empty(80 * B, dtype=torch.uint8, device="cuda")
    masks = torch.empty(sum(ns), dtype=torch.uint8, device="cuda")
    best, ms = T.tr_autotune(reg.h, src, dst, offs, B, max_n, prm, out, masks)
    torch.cuda.synchronize()
    say(f"autotune batch: super {best.sc2_super} compat {best.compat_per_cu} ppw {best.hyp_ppw} "
        f"per_cu {best.hyp_per_cu}: {ms * 1000:.1f} us")
    assert np.array_equal(out.cpu().numpy(), ref) and np.array_equal(masks.cpu().numpy(), masks0.cpu().numpy())
    assert bytes(T.tr_tuning_get(reg.h, max_n, B)) == bytes(best)
    with pytest.raises(T.TurboRegError):
        T.tr_autotune(reg.h, src, dst, None, 2, max_n, prm, out, masks)   # several pairs need offsets


def test_tuning_cache_roundtrip(reg, tmp_path):
    """Tuned configurations persist: a saved file loaded into a new handle (explicitly, and by
    tr_create through TURBOREG_TUNING_CACHE) gives the same configuration and the same bits;
    files of another version, architecture, CU count or with a bad line are refused."""
    import os
    c = synth.CONFIGS["indoor_n1000"].replace(n=1500, k1=300)
    p = synth.make_pair(c, synth.pair_seed(6, 30))
    prm = T.params_from_config(c)
    src, dst = to_dev(torch, p.src), to_dev(torch, p.dst)
    out = torch.empty(80, dtype=torch.uint8, device="cuda")
    mask = torch.empty(c.n, dtype=torch.uint8, device="cuda")
    best, _ = T.tr_autotune(reg.h, src, dst, None, 1, c.n, prm, out, mask)
    T.tr_tuning_set(reg.h, 4000, 8, cfg(7, 3, 8, 5, 4096))   # a second group
    path = str(tmp_path / "tuning.txt")
    T.tr_tuning_save(reg.h, path)
    r0, m0 = run_single(reg, torch, p.src, p.dst, prm)
    ref = snapshot(reg, r0, m0)
    header = open(path).readline().split()
    assert header[0] == "turboreg-tuning" and header[1] == "1"
    fresh = T.Registrar(max_n=3000, max_batch=8, max_k1=600, max_k2=3)
    try:
        T.tr_tuning_load(fresh.h, path)
        assert bytes(T.tr_tuning_get(fresh.h, c.n, 1)) == bytes(best)
        assert bytes(T.tr_tuning_get(fresh.h, 4000, 8)) == bytes(cfg(7, 3, 8, 5, 4096))
        r1, m1 = run_single(fresh, torch, p.src, p.dst, prm)
        assert same(snapshot(fresh, r1, m1), ref)
    finally:
        fresh.close()
    os.environ["TURBOREG_TUNING_CACHE"] = path
    try:
        env = T.Registrar(max_n=3000, max_batch=1, max_k1=600, max_k2=3)
        assert bytes(T.tr_tuning_get(env.h, c.n, 1)) == bytes(best)
        env.close()
    finally:
        del os.environ["TURBOREG_TUNING_CACHE"]
    lines = open(path).read().splitlines()
    extra = "9 2 3 3 4 3 1024"   # a group (2304 rows, B = 2) that a refused file must not set
    bad = {"version": [lines[0].replace("turboreg-tuning 1", "turboreg-tuning 2")] + lines[1:] + [extra],
           "arch": [" ".join(header[:2] + ["gfx000"] + header[3:])] + lines[1:] + [extra],
           "cus": [" ".join(header[:3] + [str(int(header[3]) + 1)])] + lines[1:] + [extra],
           "range": lines + [extra, "6 1 5 4 6 4 0"],
           "short": lines + [extra, "6 1 5"]}
    before = bytes(T.tr_tuning_get(reg.h, 2304, 2))
    assert before != bytes(cfg(3, 3, 4, 3, 1024))
    for name, content in bad.items():
        q = str(tmp_path / f"bad_{name}.txt")
        open(q, "w").write("\n".join(content) + "\n")
        with pytest.raises(T.TurboRegError):
            T.tr_tuning_load(reg.h, q)
        assert bytes(T.tr_tuning_get(reg.h, 2304, 2)) == before, name
    good = str(tmp_path / "good_extra.txt")
    open(good, "w").write("\n".join(lines + [extra]) + "\n")
    T.tr_tuning_load(reg.h, good)
    assert bytes(T.tr_tuning_get(reg.h, 2304, 2)) == bytes(cfg(3, 3, 4, 3, 1024))
