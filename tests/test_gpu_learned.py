"""GPU: the learned pivot scorer against the oracle.

Features are bit-exact (bfloat16 bit patterns); the MLP forward matches the
float64 oracle on the same bfloat16 weights to float32-accumulation accuracy;
gradients match within 2e-2 relative L2 per tensor; training lowers the loss;
learned pivots equal the oracle's reorder of the plain pool by the GPU scores;
non-finite scores fall back to plain order.
"""
import numpy as np
import pytest

import oracle
from paper_2507_01439_amd import synth
from paper_2507_01439_amd import turboreg as T
from parity import check_taps, run_single, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = [(64, 19), (64,), (64, 64), (64,), (1, 64), (1,)]


def bf16(a):
    a = np.ascontiguousarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def bf16_bits_to_f64(bits):
    return (np.asarray(bits, np.uint32) << 16).view(np.float32).astype(np.float64)


def flat(ws):
    return np.concatenate([np.asarray(w, np.float32).reshape(-1) for w in ws])


def unflat(v):
    out, k = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(v[k:k + n], np.float64).reshape(s))
        k += n
    return out


def rand_params(seed, scale=0.25):
    rng = np.random.default_rng(seed)
    return flat([rng.standard_normal(s) * scale for s in SHAPES]).astype(np.float32)


def oracle_weights(params):
    """The weights the GPU computes with: bfloat16 copies of W, float32 biases."""
    ws = unflat(params)
    for k in (0, 2, 4):
        ws[k] = bf16(ws[k]).astype(np.float64)
    return ws


@pytest.fixture(scope="module")
def reg():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    r = T.Registrar(max_n=5000, max_batch=8, max_k1=1000, max_k2=2)
    yield r
    r.close()


def test_features_bit_exact(reg):
    ns = [300, 1000, 57]
    pairs = [synth.make_pair(synth.CONFIGS["indoor_n1000"].replace(n=n, inlier_ratio=0.2), 700 + n) for n in ns]
    src = np.concatenate([p.src for p in pairs])
    dst = np.concatenate([p.dst for p in pairs])
    offs = np.concatenate([[0], np.cumsum(ns)]).astype(np.int32)
    feat = torch.empty((int(offs[-1]), 19), dtype=torch.int16, device="cuda")
    prm = T.make_params(0.1, 0.1, k1=1, k2=1)
    T.tr_features_batch(reg.h, to_dev(torch, src), to_dev(torch, dst), to_dev(torch, offs), len(ns), 1000, prm, feat)
    torch.cuda.synchronize()
    got = feat.cpu().numpy().view(np.uint16)
    for b, p in enumerate(pairs):
        C, _, _, _ = oracle.compat(p.src, p.dst, 0.1)
        F = oracle.features(p.src, p.dst, 0.1, C, oracle.sc2(C))
        want = (bf16(F.astype(np.float32)).view(np.uint32) >> 16).astype(np.uint16)
        assert np.array_equal(got[offs[b]:offs[b + 1]], want), f"pair {b}: {np.argwhere(got[offs[b]:offs[b + 1]] != want)[:5]}"


def test_mlp_forward_matches_oracle(reg):
    params = rand_params(1)
    T.tr_scorer_set(reg.h, params)
    rng = np.random.default_rng(2)
    m = 3000
    F = rng.random((m, 19)).astype(np.float32)
    bits = (bf16(F).view(np.uint32) >> 16).astype(np.uint16)
    d_feat = torch.from_numpy(bits.view(np.int16)).cuda()
    scores = torch.empty(m, dtype=torch.float32, device="cuda")
    T.tr_mlp_forward(reg.h, d_feat, m, scores)
    torch.cuda.synchronize()
    s = scores.cpu().numpy().astype(np.float64)
    so = oracle.mlp_fwd(bf16_bits_to_f64(bits), oracle_weights(params))
    err = np.abs(s - so) / (1.0 + np.abs(so))
    assert err.max() < 2e-2 and np.median(err) < 1e-3, (err.max(), np.median(err))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


# 2048: whole 256-sample tiles; 2125: a last tile of 77 samples (a partial 32-sample block, then
# empty blocks); 9000: 36 tiles, so the tile reduction runs one full batch of 32 tiles and a partial one
@pytest.mark.parametrize("m", [2048, 2125, 9000])
def test_mlp_gradients_match_oracle(reg, m):
    params = rand_params(3)
    T.tr_scorer_set(reg.h, params)
    rng = np.random.default_rng(4)
    F = rng.random((m, 19)).astype(np.float32)
    y = (rng.random(m) < 0.3).astype(np.uint8)
    bits = (bf16(F).view(np.uint32) >> 16).astype(np.uint16)
    d_feat = torch.from_numpy(bits.view(np.int16)).cuda()
    d_lab = torch.from_numpy(y).cuda()
    grads = torch.empty(T.TR_MLP_NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    T.tr_mlp_grads(reg.h, d_feat, d_lab, m, grads, loss)
    torch.cuda.synchronize()
    g = unflat(grads.cpu().numpy())
    lo, go = oracle.mlp_bwd(bf16_bits_to_f64(bits), y, oracle_weights(params))
    assert abs(float(loss.cpu()[0]) - lo) < 1e-3 * (1 + abs(lo))
    for k, (a, b) in enumerate(zip(g, go)):
        assert rel_l2(a, b) < 2e-2, (k, rel_l2(a, b))


def test_adam_steps_match_oracle(reg):
    # four training steps (the first from zero moments, the others from the moments the GPU
    # kept): each step's float32 weights against the oracle's float64 Adam on the same gradients
    params = rand_params(21)
    T.tr_scorer_set(reg.h, params)          # also resets the Adam state
    rng = np.random.default_rng(22)
    m = 1024
    F = rng.random((m, 19)).astype(np.float32)
    y = (rng.random(m) < 0.4).astype(np.uint8)
    bits = (bf16(F).view(np.uint32) >> 16).astype(np.uint16)
    d_feat = torch.from_numpy(bits.view(np.int16)).cuda()
    d_lab = torch.from_numpy(y).cuda()
    grads = torch.empty(T.TR_MLP_NPARAM, dtype=torch.float32, device="cuda")
    w = params.astype(np.float64)
    mo = np.zeros_like(w)
    vo = np.zeros_like(w)
    lr = 3e-3
    for t in range(1, 5):
        T.tr_mlp_grads(reg.h, d_feat, d_lab, m, grads)          # the gradients the step will use
        T.tr_train_step(reg.h, d_feat, d_lab, m, lr)
        torch.cuda.synchronize()
        g = grads.cpu().numpy().astype(np.float64)
        w_gpu = T.tr_scorer_get(reg.h).astype(np.float64)
        oracle.adam(w, g, mo, vo, t, lr)
        tol = 4 * np.spacing(np.abs(w).astype(np.float32)).astype(np.float64) + 1e-5 * lr
        err = np.abs(w_gpu - w)
        say(f"adam step {t}: max |dw| {np.abs(w_gpu - params).max():.3e}, max err {err.max():.3e}")
        assert (err <= tol).all(), (t, int(np.argmax(err - tol)), float(err.max()))
        assert np.abs(w_gpu - params).max() > 0
        w = w_gpu.copy()                      # the next step starts from the GPU's float32 weights


def test_training_lowers_loss_and_blob_roundtrip(reg):
    T.tr_scorer_set(reg.h, rand_params(5, scale=0.1))
    # features and labels of generated pairs
    ns = [1500, 1500, 1500, 1500]
    cfgs = [synth.CONFIGS["indoor_n1000"].replace(n=n, inlier_ratio=r) for n, r in zip(ns, [0.05, 0.1, 0.2, 0.3])]
    pairs = [synth.make_pair(c, synth.pair_seed(3, b)) for b, c in enumerate(cfgs)]
    src = np.concatenate([p.src for p in pairs])
    dst = np.concatenate([p.dst for p in pairs])
    labels = np.concatenate([p.labels for p in pairs]).astype(np.uint8)
    offs = np.concatenate([[0], np.cumsum(ns)]).astype(np.int32)
    m = int(offs[-1])
    feat = torch.empty((m, 19), dtype=torch.int16, device="cuda")
    T.tr_features_batch(reg.h, to_dev(torch, src), to_dev(torch, dst), to_dev(torch, offs), len(ns), 1500,
                        T.make_params(0.1, 0.1, 1, 1), feat)
    d_lab = torch.from_numpy(labels).cuda()
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    losses = []
    for step in range(60):
        T.tr_train_step(reg.h, feat, d_lab, m, 1e-2, loss)
        losses.append(float(loss.cpu()[0]))
    say(f"loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.7 * losses[0]
    blob = T.tr_scorer_save(reg.h)
    w1 = T.tr_scorer_get(reg.h)
    T.tr_scorer_set(reg.h, rand_params(9))
    T.tr_scorer_load(reg.h, blob)
    assert np.array_equal(T.tr_scorer_get(reg.h), w1)
    bad = bytearray(blob)
    bad[100] ^= 1
    with pytest.raises(T.TurboRegError) as e:
        T.tr_scorer_load(reg.h, bytes(bad))
    assert e.value.status == T.TR_ERR_BAD_BLOB
    with pytest.raises(T.TurboRegError):
        T.tr_scorer_load(reg.h, blob[:-1])


@pytest.mark.parametrize("pool", [1, 4])
def test_learned_registration_parity(reg, pool):
    T.tr_scorer_set(reg.h, rand_params(11))
    cfg = synth.CONFIGS["indoor_n1000"].replace(k1=200)
    p = synth.make_pair(cfg, synth.pair_seed(3, 40 + pool))
    prm = T.params_from_config(cfg, pivot_mode=T.TR_PIVOTS_LEARNED, pool_factor=pool)
    r, mask = run_single(reg, torch, p.src, p.dst, prm)
    assert r.status == T.TR_OK
    check_taps(reg, p.src, p.dst, prm, r, mask, label=f"learned pool={pool}")
    # the GPU's features and scores of this call match the oracle's computation from the same inputs
    # only the endpoints of the plain pool's pivots are featurised and scored
    rows = np.unique(reg.debug(T.TR_TAP_PLAIN_PIVOTS)[:, :2])
    rows = rows[rows >= 0]
    assert rows.size > 0
    C = reg.debug(T.TR_TAP_C)
    F = oracle.features(p.src, p.dst, cfg.tau, C, oracle.sc2(C))[rows]
    fbits = reg.debug(T.TR_TAP_FEATURES)[rows]
    assert np.array_equal(fbits, (bf16(F.astype(np.float32)).view(np.uint32) >> 16).astype(np.uint16))
    s = reg.debug(T.TR_TAP_SCORES).astype(np.float64)[rows]
    so = oracle.mlp_fwd(bf16_bits_to_f64(fbits), oracle_weights(rand_params(11)))
    assert (np.abs(s - so) / (1 + np.abs(so))).max() < 2e-2


def test_learned_fallback_on_nonfinite_scores(reg):
    params = rand_params(12)
    params[:64 * 19] = 3e38       # W1 overflows: every score is NaN or inf
    T.tr_scorer_set(reg.h, params)
    cfg = synth.CONFIGS["indoor_n1000"].replace(k1=100)
    p = synth.make_pair(cfg, synth.pair_seed(3, 77))
    prm = T.params_from_config(cfg, pivot_mode=T.TR_PIVOTS_LEARNED, pool_factor=4)
    r, mask = run_single(reg, torch, p.src, p.dst, prm)
    assert r.status == T.TR_WARN_SCORER_FALLBACK
    plain = reg.debug(T.TR_TAP_PLAIN_PIVOTS)
    assert np.array_equal(reg.debug(T.TR_TAP_PIVOTS), plain[:cfg.k1])


def test_trained_scorer_gain_on_held_out_hard_pairs():
    # What the committed network gains: on 64 held-out pairs of the hard slice (N = 5000,
    # 0.5-1 % inliers, seeds disjoint from training), learned pivots reach the success rate of
    # plain pivots at K1 = 1000 with fewer pivots than plain pivots need.
    import os
    from paper_2507_01439_amd import eval_learned
    weights = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2507_01439_amd",
                           "weights", "scorer_indoor.bin")
    r = T.Registrar(max_n=5000, max_batch=1, max_k1=1000, max_k2=2)
    try:
        with open(weights, "rb") as f:
            T.tr_scorer_load(r.h, f.read())
        _, hard = eval_learned.held_out(0, 64)
        res = eval_learned.compare(r, torch, hard, k1_sweep=(8, 16, 32, 64, 125, 250, 1000), ref_k1=1000)
    finally:
        r.close()
    tab = {m: {k: round(v["success_rate"], 3) for k, v in res["table"][m].items()} for m in res["table"]}
    say(tab, res["operating_k1"])
    op = res["operating_k1"]
    assert op["learned"] is not None and op["plain"] is not None
    assert op["learned"] < op["plain"]
    assert all(tab["learned"][k] >= tab["plain"][k] for k in (8, 16, 32, 64))
