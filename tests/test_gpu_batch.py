"""GPU: batched registration of uneven pairs in one pass, and its hipGraph replay.

Every pair of a batch must equal the oracle exactly as a single pair does;
graph replays (same buffers, new contents, eager work in between) must equal
the eager result each time.
"""
import numpy as np
import pytest

from paper_2507_01439_amd import synth
from paper_2507_01439_amd import turboreg as T
from parity import check_taps, say, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def reg():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    r = T.Registrar(max_n=1500, max_batch=16, max_k1=400, max_k2=3)
    yield r
    r.close()


def make_batch(ns, seed):
    pairs = []
    for b, n in enumerate(ns):
        cfg = synth.CONFIGS["indoor_n1000"].replace(n=max(n, 1), inlier_ratio=0.05 + 0.05 * (b % 5))
        pairs.append(synth.make_pair(cfg, synth.pair_seed(2, seed * 100 + b)))
    src = np.concatenate([p.src[:n] for p, n in zip(pairs, ns)]).astype(np.float32)
    dst = np.concatenate([p.dst[:n] for p, n in zip(pairs, ns)]).astype(np.float32)
    offs = np.concatenate([[0], np.cumsum(ns)]).astype(np.int32)
    return pairs, src, dst, offs


def test_batch_uneven_matches_oracle(reg):
    ns = [700, 3, 1500, 64, 2, 1001, 250]
    pairs, src, dst, offs = make_batch(ns, 1)
    prm = T.make_params(0.1, 0.1, k1=300, k2=2)
    say("batch uneven")
    out, masks = reg.register_batch(to_dev(torch, src), to_dev(torch, dst), to_dev(torch, offs), prm, max_n=1500)
    torch.cuda.synchronize()
    res = T.parse_results(out, len(ns))
    masks = masks.cpu().numpy()
    for b, n in enumerate(ns):
        r = res[b]
        if n < 3:
            assert r.status == T.TR_ERR_INVALID_ARG and r.best_hyp == -1
            continue
        X, Y = src[offs[b]:offs[b + 1]], dst[offs[b]:offs[b + 1]]
        check_taps(reg, X, Y, prm, r, masks[offs[b]:offs[b + 1]], pair=b, label=f"batch pair {b} n={n}")


@pytest.mark.parametrize("count", [15, 16, 21])
def test_batch_in_size_order_matches_oracle(count):
    # 21 pairs (from 16 on, a batch takes the size-ordered work lists: pairs sorted by tile count
    # and dealt to the XCDs; 15 keeps index order), with sizes across several tile counts, equal
    # sizes and invalid pairs
    ns = [700, 2, 256, 257, 640, 3, 512, 700, 100, 0, 513, 300, 699, 64, 255, 600, 5, 450, 700, 1, 333][:count]
    r = T.Registrar(max_n=700, max_batch=len(ns), max_k1=200, max_k2=2)
    try:
        pairs, src, dst, offs = make_batch([max(n, 0) for n in ns], 5)
        prm = T.make_params(0.1, 0.1, k1=150, k2=2)
        say(f"batch in size order: {len(ns)} pairs")
        out, masks = r.register_batch(to_dev(torch, src), to_dev(torch, dst), to_dev(torch, offs), prm, max_n=700)
        torch.cuda.synchronize()
        res = T.parse_results(out, len(ns))
        masks = masks.cpu().numpy()
        for b, n in enumerate(ns):
            if n < 3:
                assert res[b].status == T.TR_ERR_INVALID_ARG and res[b].best_hyp == -1, b
                continue
            X, Y = src[offs[b]:offs[b + 1]], dst[offs[b]:offs[b + 1]]
            check_taps(r, X, Y, prm, res[b], masks[offs[b]:offs[b + 1]], pair=b, label=f"pair {b} n={n}")
    finally:
        r.close()


def test_batch_of_more_pairs_than_planner_threads():
    # 1100 small pairs: the planner walks them in two chunks of its 1024 threads, reads the order
    # back from device memory (not its LDS copy) and deals 1100 slots to the XCDs; invalid pairs
    # (N < 3) are mixed in. Every record and mask against the oracle, all taps for a sample.
    rng = np.random.default_rng(7)
    ns = [int(x) for x in rng.integers(0, 129, size=1100)]
    ns[5] = ns[700] = 1
    ns[1024] = 0
    r = T.Registrar(max_n=128, max_batch=len(ns), max_k1=40, max_k2=2)
    try:
        pairs, src, dst, offs = make_batch(ns, 6)
        prm = T.make_params(0.1, 0.1, k1=30, k2=2)
        say(f"batch of {len(ns)} pairs, N 0..128")
        out, masks = r.register_batch(to_dev(torch, src), to_dev(torch, dst), to_dev(torch, offs), prm, max_n=128)
        torch.cuda.synchronize()
        res = T.parse_results(out, len(ns))
        masks = masks.cpu().numpy()
        for b, n in enumerate(ns):
            if n < 3:
                assert res[b].status == T.TR_ERR_INVALID_ARG and res[b].best_hyp == -1, b
                continue
            X, Y = src[offs[b]:offs[b + 1]], dst[offs[b]:offs[b + 1]]
            check_taps(r, X, Y, prm, res[b], masks[offs[b]:offs[b + 1]], pair=b, label=f"pair {b} n={n}",
                       dense=b % 50 == 0 or b >= 1020)
    finally:
        r.close()


def test_batch_equals_single(reg):
    ns = [400, 900, 128]
    pairs, src, dst, offs = make_batch(ns, 2)
    prm = T.make_params(0.1, 0.1, k1=200, k2=3)
    out, masks = reg.register_batch(to_dev(torch, src), to_dev(torch, dst), to_dev(torch, offs), prm, max_n=1500)
    torch.cuda.synchronize()
    batch = [bytes(r) for r in T.parse_results(out, len(ns))]
    bm = masks.cpu().numpy()
    for b, n in enumerate(ns):
        s_out, s_mask = reg.register(to_dev(torch, src[offs[b]:offs[b + 1]]), to_dev(torch, dst[offs[b]:offs[b + 1]]), prm)
        torch.cuda.synchronize()
        assert bytes(T.parse_results(s_out)[0]) == batch[b]
        assert np.array_equal(s_mask.cpu().numpy(), bm[offs[b]:offs[b + 1]])


def test_graph_replay_matches_eager(reg):
    ns = [600, 1200, 333, 90]
    prm = T.make_params(0.1, 0.1, k1=250, k2=2)
    side = torch.cuda.Stream()            # default priority
    pairs, src, dst, offs = make_batch(ns, 3)
    d_src, d_dst, d_offs = to_dev(torch, src), to_dev(torch, dst), to_dev(torch, offs)
    out = torch.empty(80 * len(ns), dtype=torch.uint8, device="cuda")
    masks = torch.empty(int(offs[-1]), dtype=torch.uint8, device="cuda")
    for rep in range(4):
        # new contents in the same buffers every time; eager work of our own in between
        _, s2, d2, _ = make_batch(ns, 10 + rep)
        d_src.copy_(torch.from_numpy(s2))
        d_dst.copy_(torch.from_numpy(d2))
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            T.tr_register_batch(reg.h, d_src, d_dst, d_offs, len(ns), 1500, prm, out, masks)
        side.synchronize()
        graph_res = [bytes(r) for r in T.parse_results(out, len(ns))]
        graph_masks = masks.cpu().numpy().copy()
        # eager reference: the default stream is never captured
        e_out, e_masks = reg.register_batch(d_src, d_dst, d_offs, prm, max_n=1500)
        torch.cuda.synchronize()
        assert graph_res == [bytes(r) for r in T.parse_results(e_out, len(ns))], f"replay {rep}"
        assert np.array_equal(graph_masks, e_masks.cpu().numpy()), f"replay {rep}"
        res = T.parse_results(e_out, len(ns))
        for b in range(len(ns)):
            X, Y = s2[offs[b]:offs[b + 1]], d2[offs[b]:offs[b + 1]]
            check_taps(reg, X, Y, prm, res[b], graph_masks[offs[b]:offs[b + 1]], pair=b, label=f"replay {rep} pair {b}")


def test_graph_cache_eviction(reg):
    # twelve output buffer sets on one side stream, more than the eight graphs a handle keeps,
    # then the first sets again (evicted by now, so captured anew): every launch equals the
    # eager result, and the graphs launched before an eviction finished with their own bits
    ns = [500, 260, 1100]
    prm = T.make_params(0.1, 0.1, k1=200, k2=2)
    side = torch.cuda.Stream()            # default priority
    _, src, dst, offs = make_batch(ns, 4)
    d_src, d_dst, d_offs = to_dev(torch, src), to_dev(torch, dst), to_dev(torch, offs)
    e_out, e_masks = reg.register_batch(d_src, d_dst, d_offs, prm, max_n=1500)
    torch.cuda.synchronize()
    want, want_masks = e_out.cpu().numpy(), e_masks.cpu().numpy()
    sets = [(torch.full((80 * len(ns),), 0xAB, dtype=torch.uint8, device="cuda"),
             torch.full((int(offs[-1]),), 0xAB, dtype=torch.uint8, device="cuda")) for _ in range(12)]
    torch.cuda.synchronize()
    order = list(range(12)) + [0, 1, 2]
    say(f"graph cache: {len(order)} launches over {len(sets)} buffer sets")
    with torch.cuda.stream(side):
        for k in order:
            out, masks = sets[k]
            out.fill_(0xAB)
            masks.fill_(0xAB)
            T.tr_register_batch(reg.h, d_src, d_dst, d_offs, len(ns), 1500, prm, out, masks)
    side.synchronize()
    for k, (out, masks) in enumerate(sets):
        assert np.array_equal(out.cpu().numpy(), want), f"buffer set {k}"
        assert np.array_equal(masks.cpu().numpy(), want_masks), f"buffer set {k}"


def test_batch_success_on_indoor_pairs(reg):
    cfgs = synth.batch_configs(12, seed=5, n_lo=500, n_hi=1500)
    pairs = [synth.make_pair(c.replace(k1=250), synth.pair_seed(2, 500 + b)) for b, c in enumerate(cfgs)]
    ns = [p.src.shape[0] for p in pairs]
    src = np.concatenate([p.src for p in pairs])
    dst = np.concatenate([p.dst for p in pairs])
    offs = np.concatenate([[0], np.cumsum(ns)]).astype(np.int32)
    prm = T.make_params(0.1, 0.1, k1=250, k2=2)
    out, _ = reg.register_batch(to_dev(torch, src), to_dev(torch, dst), to_dev(torch, offs), prm, max_n=1500)
    torch.cuda.synchronize()
    res = T.parse_results(out, len(ns))
    ok = [synth.success(np.array(r.R).reshape(3, 3), np.array(r.t), p) for r, p in zip(res, pairs)]
    assert np.mean(ok) >= 0.9, ok


def test_independent_handles_on_two_streams(reg):
    # registrations on two handles, each on its own stream, interleaved without synchronisation:
    # every result and mask must equal the same registration run alone on the fixture's handle
    ns = [1500, 900, 1200, 640, 1500, 1100]
    pairs = [synth.make_pair(synth.CONFIGS["indoor_n1000"].replace(n=n, inlier_ratio=0.08), synth.pair_seed(2, 900 + b))
             for b, n in enumerate(ns)]
    prm = T.make_params(0.1, 0.1, 300, 2)
    alone = []
    for p in pairs:
        out, mask = reg.register(to_dev(torch, p.src), to_dev(torch, p.dst), prm)
        torch.cuda.synchronize()
        alone.append((bytes(out.cpu().numpy()), mask.cpu().numpy().copy()))
    handles = [T.Registrar(max_n=1500, max_batch=1, max_k1=400, max_k2=3) for _ in range(2)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]   # default priority
    try:
        outs = []
        inputs = [(to_dev(torch, p.src), to_dev(torch, p.dst)) for p in pairs]
        torch.cuda.synchronize()
        for k, (src, dst) in enumerate(inputs):
            with torch.cuda.stream(streams[k % 2]):
                outs.append(handles[k % 2].register(src, dst, prm))
        torch.cuda.synchronize()
        for k, ((o, m), (ao, am)) in enumerate(zip(outs, alone)):
            assert bytes(o.cpu().numpy()) == ao, k
            assert np.array_equal(m.cpu().numpy(), am), k
    finally:
        for h in handles:
            h.close()
